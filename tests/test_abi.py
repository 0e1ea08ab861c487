"""C-ABI checks that need no GPU: the library loads, exports every entry point the
header declares, and rejects invalid arguments on the host before enqueueing work."""
import ctypes as C
import os
import re

import pytest

import paper_2512_12442_amd as lcp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "lcp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_header_function():
    names = header_functions()
    assert {"gp_fit_factor", "gp_posterior", "lcp_dense", "lcp_adaptive", "lcp_backward"} <= set(names)
    L = lcp.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lcp.lcp.EXPORTS) == names


def test_status_strings_and_model_bytes():
    L = lcp.lib()
    assert L.lcp_status_str(0) == b"ok"
    assert L.lcp_status_str(2).startswith(b"covariance")
    assert L.lcp_model_bytes(0, 3) == 0 and L.lcp_model_bytes(1025, 3) == 0
    assert L.lcp_model_bytes(500, 3) > 500 * 500 * 8 * 3


def _fit(kind=0, dim=3, s2=1.0, ell=(0.1, 0.1, 0.1), noise=1e-4, m=10, X=None, y=None, mem=None, nb=0):
    L = lcp.lib()
    k = lcp.lcp.Kernel(kind, dim, s2, (C.c_double * 3)(*ell), noise)
    h = C.c_void_p()
    rc = L.gp_fit_factor(C.byref(k), m, X, y, mem, nb, None, C.byref(h))
    return rc, L.lcp_last_error().decode(), h


@pytest.mark.parametrize("kw,frag", [
    (dict(dim=4), "dim"), (dict(kind=7), "kernel"), (dict(s2=0.0), "signal_var"), (dict(s2=float("nan")), "signal_var"),
    (dict(noise=-1.0), "noise_var"), (dict(ell=(0.1, -1.0, 0.1)), "lengthscale"), (dict(m=0), "m = 0"),
    (dict(m=2000), "m = 2000"), (dict(), "must not be NULL"),
])
def test_fit_rejects_invalid_arguments(kw, frag):
    rc, msg, h = _fit(**kw)
    assert rc == lcp.lcp.LCP_EINVAL and frag in msg and not h.value


def test_fit_rejects_small_or_misaligned_model_memory():
    fake = C.c_void_p(0x1000)     # never dereferenced: validation fails first
    rc, msg, _ = _fit(X=fake, y=fake, mem=fake, nb=16)
    assert rc == lcp.lcp.LCP_ENOMEM and "model memory" in msg
    rc, msg, _ = _fit(X=fake, y=fake, mem=C.c_void_p(0x1010), nb=1 << 30)
    assert rc == lcp.lcp.LCP_EINVAL and "aligned" in msg


def test_sparse_fit_validates_on_the_host():
    L = lcp.lib()
    k = lcp.lcp.Kernel(0, 3, 1.0, (C.c_double * 3)(0.1, 0.1, 0.1), 1e-6)
    fake = C.c_void_p(0x1000)     # never dereferenced: validation fails first
    h, sh = C.c_void_p(), C.c_double(-1.0)
    rc = L.gp_fit_sgpr(C.byref(k), 10, fake, fake, None, fake, 1 << 30, None, C.byref(sh), C.byref(h))
    assert rc == lcp.lcp.LCP_EINVAL and "A_M" in L.lcp_last_error().decode() and not h.value and sh.value == 0.0
    rc = L.gp_fit_sgpr(C.byref(k), 0, fake, fake, fake, fake, 1 << 30, None, None, C.byref(h))
    assert rc == lcp.lcp.LCP_EINVAL and "m = 0" in L.lcp_last_error().decode()
    rc = L.gp_fit_sgpr(C.byref(k), 10, fake, fake, fake, fake, 16, None, None, C.byref(h))
    assert rc == lcp.lcp.LCP_ENOMEM


def test_backward_validates_on_the_host():
    L = lcp.lib()
    rc = L.lcp_backward(None, None, 0.0, None, 0, None, None, None, None, 0, None)
    assert rc == lcp.lcp.LCP_EINVAL and "model" in L.lcp_last_error().decode()
    b = C.c_size_t()
    assert L.lcp_backward_workspace(None, None, 0, 16, C.byref(b)) == lcp.lcp.LCP_EINVAL
    rc = L.gp_posterior_backward(None, 4, None, 0, None, None, None, None, None, 0, None)
    assert rc == lcp.lcp.LCP_EINVAL


def test_null_model_rejected_everywhere():
    L = lcp.lib()
    b = C.c_size_t()
    assert L.lcp_dense_workspace(None, None, 0, 1600, C.byref(b)) == lcp.lcp.LCP_EINVAL
    assert L.lcp_adaptive_workspace(None, None, None, 0, 1600, C.byref(b)) == lcp.lcp.LCP_EINVAL
    assert L.gp_posterior(None, 1, None, 0, None, None, None, 0, None) == lcp.lcp.LCP_EINVAL
    assert L.lcp_dense(None, None, 0.0, None, 0, None, None, 0, None) == lcp.lcp.LCP_EINVAL
    assert L.lcp_adaptive(None, None, 0.0, None, None, 0, None, None, 0, None, None, None, 0, None) == lcp.lcp.LCP_EINVAL
    assert L.lcp_bound_workspace(None, 4, C.byref(b)) == lcp.lcp.LCP_EINVAL
    assert L.lcp_bound_certified(None, 4, None, None, None, 0, None) == lcp.lcp.LCP_EINVAL
    assert L.lcp_cell_moments_workspace(None, None, 4, 0, C.byref(b)) == lcp.lcp.LCP_EINVAL
    assert L.lcp_cell_moments(None, None, 4, None, 0, None, None, None, 0, None) == lcp.lcp.LCP_EINVAL
    assert "model" in L.lcp_last_error().decode()


def test_adapt_struct_carries_the_bound_kind():
    a = lcp.adapt_of(type("W", (), {"alpha": 1e-3, "min_leaf": 4})(), bound_kind=lcp.BOUND_CERTIFIED)
    assert a.bound_kind == 1 and a.descent_steps == 4 and a.min_leaf_cells == 4
    assert lcp.lcp.Adapt.bound_kind.offset == 20 and lcp.lcp.Adapt.split.offset == 24
    assert lcp.lcp.Adapt.beta.offset == 32 and lcp.lcp.Adapt.edge_bound.offset == 40
    assert C.sizeof(lcp.lcp.Adapt) == 48
    assert lcp.adapt_of(type("W", (), {"alpha": 1e-3, "min_leaf": 4})(), edge_bound=1).edge_bound == 1
    a = lcp.adapt_of(type("W", (), {"alpha": 1e-3, "min_leaf": 4})(), bound_kind=lcp.BOUND_LOCAL, beta=2.5)
    assert a.bound_kind == 2 and a.beta == 2.5
    assert lcp.adapt_of(type("W", (), {"alpha": 1e-3, "min_leaf": 2})(), split=lcp.SPLIT_KD).split == 1


def _fit_batch(kernels, ms, X=None, y=None, mem=None, nbytes=0):
    L = lcp.lib()
    nb = len(kernels)
    K = (lcp.lcp.Kernel * max(nb, 1))()
    for b, (kind, dim, s2, ell, noise) in enumerate(kernels):
        K[b] = lcp.lcp.Kernel(kind, dim, s2, (C.c_double * 3)(*ell), noise)
    m = (C.c_int * max(nb, 1))(*ms)
    h = C.c_void_p()
    rc = L.gp_fit_factor_batch(nb, K, m, X, y, mem, nbytes, None, C.byref(h))
    return rc, L.lcp_last_error().decode(), h


def test_batch_model_bytes_and_validation():
    L = lcp.lib()
    ok_k = (0, 3, 1.0, (0.1, 0.1, 0.1), 1e-4)
    m2 = (C.c_int * 2)(10, 700)
    assert L.lcp_batch_model_bytes(2, m2, 3) >= L.lcp_model_bytes(10, 3) + L.lcp_model_bytes(700, 3)
    assert L.lcp_batch_model_bytes(2, (C.c_int * 2)(10, 0), 3) == 0
    assert L.lcp_batch_model_bytes(0, m2, 3) == 0
    rc, msg, h = _fit_batch([], [])
    assert rc == lcp.lcp.LCP_EINVAL and "nb" in msg and not h.value
    rc, msg, _ = _fit_batch([ok_k, (0, 3, 1.0, (0.1, 0.1, 0.1), -1.0)], [10, 10])
    assert rc == lcp.lcp.LCP_EINVAL and "model 1" in msg and "noise_var" in msg
    rc, msg, _ = _fit_batch([ok_k, (0, 2, 1.0, (0.1, 0.1, 0.1), 1e-4)], [10, 10])
    assert rc == lcp.lcp.LCP_EINVAL and "dim" in msg
    rc, msg, _ = _fit_batch([ok_k, ok_k], [10, 2000])
    assert rc == lcp.lcp.LCP_EINVAL and "model 1" in msg
    fake = C.c_void_p(0x1000)     # never dereferenced: validation fails first
    rc, msg, _ = _fit_batch([ok_k, ok_k], [10, 10], X=fake, y=fake, mem=fake, nbytes=16)
    assert rc == lcp.lcp.LCP_ENOMEM and "model memory" in msg
    b = C.c_size_t()
    assert L.lcp_dense_batch_workspace(None, None, 0, 1600, C.byref(b)) == lcp.lcp.LCP_EINVAL
    assert L.lcp_dense_batch(None, None, None, None, 0, None, None, 0, None) == lcp.lcp.LCP_EINVAL


def test_noalloc_scratch_size_matches_header():
    src = open(os.path.join(ROOT, "include", "lcp.h")).read()
    m = re.search(r"#define LCP_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == lcp.lcp.NOALLOC_SCRATCH_BYTES


def test_noalloc_rejects_null_model_on_the_host():
    L = lcp.lib()
    assert L.lcp_dense_noalloc(None, None, 0.0, None, 0, None, None) == lcp.lcp.LCP_EINVAL
    assert "model is NULL" in L.lcp_last_error().decode()
