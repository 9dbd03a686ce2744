"""Per-kernel timing through the C ABI (irl_stats_enable / irl_stats_select /
irl_stats_get): events leave every result unchanged, a step times one Hamiltonian
launch per operator apply plus those of the evaluations, a restricted kind mask
records only its kinds (with the same launch counts as the full mask), and a
bit beyond the last kind is rejected."""
import pytest

import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _fields(r):
    return tuple(repr(x) for x in (r.E_before, r.lambda_min, r.E_after, r.c0, r.residual_est,
                                   r.residual_explicit, r.n_apply, r.n_restart, r.converged))


def _steps(stats_kinds, steps=2):
    """Run `steps` IRL steps of a small full space; stats_kinds: None (no events),
    "all", or a list of kind names."""
    from paper_2601_01437_amd import IRL_WS_FACTORED, System
    from paper_2601_01437_amd import binding as B
    n, na, nb, H, seed = 8, 4, 4, 16, 2
    h, g = synth.integrals(n, seed)
    s = System(n, na, nb, h, g)
    th = dev(synth.nqs_theta(2 * n, H, seed, scale=0.2))
    if stats_kinds is not None:
        B.irl_stats_select(s.handle, None if stats_kinds == "all" else stats_kinds)
        B.irl_stats_enable(s.handle, True)
    out = []
    for _ in range(steps):
        rc, r, dth, _ = s.step(th, 2 * n, H, m=12, k_keep=3, ws_flags=IRL_WS_FACTORED)
        out.append((rc, _fields(r), host(dth).tobytes()))
    stats = B.irl_stats_get(s.handle) if stats_kinds is not None else None
    if stats_kinds is not None:
        B.irl_stats_enable(s.handle, False)
    return out, stats


def test_stats_leave_results_unchanged_and_count_launches():
    announce("stats: all kinds against none")
    ref, _ = _steps(None)
    got, st = _steps("all")
    assert got == ref
    n_apply = sum(int(x[1][6]) for x in got)
    # one Hamiltonian launch per apply, plus H psi at each evaluation (before and
    # after each step)
    assert st["ham_apply"][1] >= n_apply + 2
    assert st["dtilde_build"][1] >= 2
    for k in ("ham_apply", "gemv", "gemv_t", "lanczos", "ritz"):
        assert st[k][1] > 0 and st[k][0] > 0.0, k


def test_stats_select_restricts_kinds():
    announce("stats: ham_apply only")
    ref, full = _steps("all")
    got, part = _steps(["ham_apply", "gemv_t"])
    assert got == ref
    for k, (ms, cnt) in part.items():
        if k in ("ham_apply", "gemv_t"):
            assert cnt == full[k][1] and ms > 0.0, k
        else:
            assert cnt == 0 and ms == 0.0, k


def test_stats_select_rejects_unknown_bits():
    from paper_2601_01437_amd import System
    from paper_2601_01437_amd import binding as B
    announce("stats: invalid mask")
    h, g = synth.integrals(4, 0)
    s = System(4, 2, 2, h, g)
    rc = B._lib.irl_stats_select(s.handle, 1 << len(B.STAT_KINDS))
    assert rc == -1
    assert B._lib.irl_stats_select(s.handle, 0) == 0
