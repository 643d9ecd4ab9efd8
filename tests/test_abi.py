"""Host-side checks of the C ABI (no compute call is made): the library loads, exports every
entry point include/paris.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2009_00166_amd as paris
from paper_2009_00166_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "paris.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(paris_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = paris.load_library()
    names = _declared()
    assert "paris_build" in names and "paris_query_exact" in names and "paris_query_batch" in names
    for name in names:
        assert hasattr(lib, name), name
    bound = {n for n, _, _ in B.SIGNATURES}
    assert bound == set(names)


def test_default_config_and_workspace_size():
    cfg = paris.default_config()
    assert (cfg.segments, cfg.card_bits, cfg.leaf_mode, cfg.n_leaves, cfg.seed_cap) == (16, 8, 0, 4096, 16384)
    small = paris.workspace_size(1000, 256, cfg)
    big = paris.workspace_size(10_000_000, 256, cfg)
    assert big > 10_000_000 * 44 and small > 1000 * 44
    assert paris.workspace_size(1000, 256, cfg) == paris.workspace_size(1000, 1024, cfg)


@pytest.mark.parametrize("N,n", [(0, 256), (10, 250), (10, 8), (10, 4096), (2**32, 256)])
def test_workspace_size_rejects_bad_shapes(N, n):
    lib = paris.load_library()
    cfg = paris.default_config()
    out = ctypes.c_size_t(0)
    assert lib.paris_workspace_size(N, n, ctypes.byref(cfg), ctypes.byref(out)) == B.PARIS_EINVAL


@pytest.mark.parametrize("field,value", [("segments", 8), ("card_bits", 4), ("leaf_mode", 7),
                                         ("seed_cap", -1)])
def test_bad_config_rejected(field, value):
    lib = paris.load_library()
    cfg = paris.default_config(**{field: value})
    out = ctypes.c_size_t(0)
    assert lib.paris_workspace_size(100, 256, ctypes.byref(cfg), ctypes.byref(out)) == B.PARIS_EINVAL
    cfg2 = paris.default_config(leaf_mode=1, n_leaves=0)
    assert lib.paris_workspace_size(100, 256, ctypes.byref(cfg2), ctypes.byref(out)) == B.PARIS_EINVAL


def test_build_argument_errors_before_any_launch():
    lib = paris.load_library()
    cfg = paris.default_config()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x100000)
    # null series / workspace / out
    assert lib.paris_build(None, 100, 256, ctypes.byref(cfg), fake, 1 << 30, None, ctypes.byref(h)) == B.PARIS_EINVAL
    assert lib.paris_build(fake, 100, 256, ctypes.byref(cfg), None, 1 << 30, None, ctypes.byref(h)) == B.PARIS_EINVAL
    assert lib.paris_build(fake, 100, 256, ctypes.byref(cfg), fake, 1 << 30, None, None) == B.PARIS_EINVAL
    # length not a multiple of the segment count
    assert lib.paris_build(fake, 100, 250, ctypes.byref(cfg), fake, 1 << 30, None, ctypes.byref(h)) == B.PARIS_EINVAL
    # misaligned series pointer
    assert lib.paris_build(ctypes.c_void_p(0x100004), 100, 256, ctypes.byref(cfg), fake, 1 << 30, None,
                           ctypes.byref(h)) == B.PARIS_EINVAL
    # workspace smaller than required
    need = paris.workspace_size(100, 256, cfg)
    assert lib.paris_build(fake, 100, 256, ctypes.byref(cfg), fake, need - 1, None, ctypes.byref(h)) == B.PARIS_ENOMEM


def test_no_device_reported_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present: the no-device path cannot be exercised")
    lib = paris.load_library()
    cfg = paris.default_config()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x100000)
    need = paris.workspace_size(100, 256, cfg)
    assert lib.paris_build(fake, 100, 256, ctypes.byref(cfg), fake, need, None, ctypes.byref(h)) == B.PARIS_ENODEV


def test_invalid_handles_rejected():
    lib = paris.load_library()
    bogus = ctypes.c_void_p(0xDEAD0000)
    i = ctypes.c_int64()
    d = ctypes.c_double()
    assert lib.paris_free(None) == B.PARIS_OK
    assert lib.paris_free(bogus) == B.PARIS_ESTATE
    assert lib.paris_query_exact(bogus, ctypes.c_void_p(0x1000), ctypes.byref(i), ctypes.byref(d), None,
                                 None) == B.PARIS_ESTATE
    assert lib.paris_query_batch(None, None, 1, None, None, None, None) == B.PARIS_ESTATE
    assert lib.paris_set_bsf_sharing(None, 1) == B.PARIS_ESTATE
    assert lib.paris_set_bsf_sharing(bogus, 0) == B.PARIS_ESTATE
    lay = B.ParisLayout()
    assert lib.paris_get_layout(bogus, ctypes.byref(lay)) == B.PARIS_ESTATE


def test_status_strings():
    lib = paris.load_library()
    for s in range(-6, 1):
        assert lib.paris_status_string(s)
    assert lib.paris_status_string(-99) == b"unknown status"


def test_seed_network_argument_errors_before_any_launch():
    lib = paris.load_library()
    cnt = ctypes.c_int64(0)
    assert lib.paris_mlp_param_count(4096, ctypes.byref(cnt)) == B.PARIS_OK and cnt.value == 1_122_816
    for bad in (0, 8, 100, 65600):
        assert lib.paris_mlp_param_count(bad, ctypes.byref(cnt)) == B.PARIS_EINVAL
    h = ctypes.c_void_p()
    nb = ctypes.c_int64(0)
    assert lib.paris_mlp_workspace_size(4096, 64, ctypes.byref(nb)) == B.PARIS_OK
    # the parameters, their bfloat16 copy, gradient and two moments alone take 18 bytes each
    assert nb.value >= 18 * 1_122_816
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: every call below fails its argument checks
    for nl, rows in ((100, 64), (4096, 100), (4096, 0), (0, 64)):
        assert lib.paris_mlp_workspace_size(nl, rows, ctypes.byref(nb)) == B.PARIS_EINVAL
        assert lib.paris_mlp_create(nl, rows, fake, 1 << 40, ctypes.byref(h)) == B.PARIS_EINVAL
    assert lib.paris_mlp_create(4096, 64, fake, 1 << 40, None) == B.PARIS_EINVAL
    assert lib.paris_mlp_create(4096, 64, None, 1 << 40, ctypes.byref(h)) == B.PARIS_EINVAL
    assert lib.paris_mlp_create(4096, 64, ctypes.c_void_p((1 << 20) + 4), 1 << 40, ctypes.byref(h)) == B.PARIS_EINVAL
    lib.paris_mlp_workspace_size(4096, 64, ctypes.byref(nb))
    assert lib.paris_mlp_create(4096, 64, fake, nb.value - 1, ctypes.byref(h)) == B.PARIS_EINVAL
    null = ctypes.c_void_p()
    opt = B.ParisAdam(1e-3, 0.9, 0.999, 1e-8)
    assert lib.paris_mlp_set_params(null, null, null) == B.PARIS_ESTATE
    assert lib.paris_mlp_forward(null, null, 1, null, null) == B.PARIS_ESTATE
    assert lib.paris_mlp_top_leaves(null, null, 1, null, null) == B.PARIS_ESTATE
    assert lib.paris_mlp_grad(null, null, null, null, 1, null, null, null) == B.PARIS_ESTATE
    assert lib.paris_mlp_train_step(null, null, null, null, 1, ctypes.byref(opt), null, null) == B.PARIS_ESTATE
    assert lib.paris_mlp_apply(null, null, ctypes.byref(opt), null) == B.PARIS_ESTATE
    assert lib.paris_mlp_free(null) == B.PARIS_OK
    assert lib.paris_leaf_of(null, null, 1, null, null) == B.PARIS_ESTATE
    assert lib.paris_set_seed_model(null, null, 0) == B.PARIS_ESTATE
    assert lib.paris_query_features(null, 1, 256, null, null) == B.PARIS_EINVAL
    fake = ctypes.c_void_p(16)
    for n in (0, 8, 250, 4096):
        assert lib.paris_query_features(fake, 1, n, fake, null) == B.PARIS_EINVAL
