"""Host logic of bench.py (no GPU): which kernel classes the timed region
brackets with events, which factored kernels run in their full-space form, and
the algorithmic bytes each roofline divides by."""
from types import SimpleNamespace

import bench

KINDS = ("dtilde_build", "ham_apply", "gemv", "gemv_t", "reduce", "energy", "lanczos", "ritz",
         "gemv_fp32", "gemv_t_fp32", "vmc")
B = SimpleNamespace(STAT_KINDS=KINDS)


def _args(**kw):
    a = dict(graph=False, no_events=False, all_events=False)
    a.update(kw)
    return SimpleNamespace(**a)


def _info(full=True, ns=853776, n=12, nA=924, nB=924, ham_kernel=2, conns=1818):
    return SimpleNamespace(full_space=int(full), n_dets=ns, n_orb=n, n_alpha_strings=nA, n_beta_strings=nB,
                           ham_kernel=ham_kernel, max_connections=conns)


def test_live_kinds_dominant_roofline_class():
    warm = {k: (0.0, 0) for k in KINDS}
    warm.update(ham_apply=(6.0, 15), gemv=(1.4, 15), ritz=(9.0, 20), gemv_t=(1.3, 15))
    has = lambda k: k in ("ham_apply", "gemv", "gemv_t", "dtilde_build")
    # the Ritz kernels take longer here but have no roofline: the dominant roofline class
    assert bench.select_live_kinds(_args(), B, warm, has) == ["ham_apply"]
    assert bench.select_live_kinds(_args(all_events=True), B, warm, has) == list(KINDS)
    assert bench.select_live_kinds(_args(graph=True), B, warm, has) == []
    assert bench.select_live_kinds(_args(no_events=True), B, warm, has) == []
    # no warm-up figures: every class
    assert bench.select_live_kinds(_args(), B, {k: (0.0, 0) for k in KINDS}, has) == list(KINDS)


def test_full_space_kernel_selection():
    c2 = _info()
    for kind in ("gemv", "gemv_t", "dtilde_build"):
        assert bench.fac_full_kernel(kind, c2, c2.n_dets, 64)
    # H > 64: only the backward pass has a full-space form
    assert bench.fac_full_kernel("gemv_t", c2, c2.n_dets, 100)
    assert not bench.fac_full_kernel("gemv", c2, c2.n_dets, 100)
    assert not bench.fac_full_kernel("dtilde_build", c2, c2.n_dets, 100)
    # a row list (gathered sampled rows), a selected set, a small space, many beta strings
    assert not bench.fac_full_kernel("gemv_t", c2, 120000, 64)
    assert not bench.fac_full_kernel("gemv_t", _info(full=False), c2.n_dets, 64)
    assert not bench.fac_full_kernel("gemv_t", _info(ns=4900, n=8, nA=70, nB=70), 4900, 16)
    assert not bench.fac_full_kernel("gemv_t", _info(ns=12870 ** 2, n=16, nA=12870, nB=12870), 12870 ** 2, 64)


def test_factored_roofline_bytes():
    c2 = _info()
    ns, H, P1 = c2.n_dets, 64, 1625
    name, bound, nbytes, unit, peak, src = bench.kernel_roofline("gemv", ns, P1, H, True, 0, c2, 0)
    assert (name, bound, unit, peak) == ("fac_jvp", "hbm", "GB/s", 8000.0)
    assert nbytes == ns * (8 * H + 16) + 8 * P1           # d, psi, w
    assert bench.kernel_roofline("gemv_t", ns, P1, H, True, 0, c2, 0)[2] == ns * (8 * H + 24) + 16 * P1
    assert bench.kernel_roofline("dtilde_build", ns, P1, H, True, 0, c2, 0)[2] == ns * (8 * H + 8)
    # the matrix-core forms read the keys too
    sel = _info(full=False, ns=1 << 20, n=20, nA=0, nB=0)
    assert bench.kernel_roofline("gemv", 1 << 20, P1, H, True, 0, sel, 0)[2] == (1 << 20) * (8 * H + 24) + 8 * P1
    # the enumerating Hamiltonian kernels: 2 flops per candidate against the FP64 peak
    name, bound, work, unit, peak, _ = bench.kernel_roofline("ham_apply", ns, P1, H, True, 0, c2, 0)
    assert (bound, unit, peak, work) == ("alu", "TFLOP/s", 78.6, 2.0 * ns * c2.max_connections)
