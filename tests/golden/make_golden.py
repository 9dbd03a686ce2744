"""Write stored expected values that are too slow to recompute inside a test.

Calls only the oracle (and the seeded input generators).  Outputs:
tests/golden/c3s_step.json -- one mode-A optimisation step on the scaled-down
precision workload: 20 spatial orbitals, 10 alpha + 10 beta electrons, the 2^14
determinants of the seeded CISD-like selection, network V = 40, H = 256
(P = 10,536), dense FP64 solve of the centred S ~ I eigenproblem.
tests/golden/c2_eval.json -- the full-space workload of 12 spatial orbitals,
6 alpha + 6 beta electrons (853,776 determinants), network V = 24, H = 64
(P = 1,624) at its seeded theta: Z, E, the whole gradient and the raw operator
pair (D~^T H D~ v, D~^T D~ v) for the seeded probe vector v, computed with D~
rows recomputed chunk by chunk and the matrix-free C Slater-Condon apply.

Run from the repository root:  python tests/golden/make_golden.py [c3s] [c2]
(no argument: both).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import capply, lm, nqs, step  # noqa: E402


def c3s():
    w = synth.WORKLOADS["c3s"]
    h, g = w.integrals()
    keys = w.dets()
    theta = w.theta()
    t0 = time.time()
    Hm = capply.csr(w.n, h, g, keys)
    res, th_new, E_after = step.lm_step(keys, w.n, w.V, w.H, theta, Hm)
    Dt = nqs.dtilde(keys, w.n, w.V, w.H, theta)
    grad = lm.gradient(Dt, Hm)
    evals = np.linalg.eigvalsh(res.Hp)
    out = {
        "workload": "c3s",
        "n_dets": int(keys.size),
        "P": int(w.P),
        "E": res.E,
        "Z": res.Z,
        "lambda_min": float(res.lam),
        "lambda_2": float(evals[1]),
        "gap": float(res.gap),
        "norm_Hp": float(np.abs(evals).max()),
        "c0": float(res.c[0]),
        "E_after": float(E_after),
        "dtheta_norm": float(np.linalg.norm(res.dtheta)),
        "dtheta_head": [float(x) for x in res.dtheta[:32]],
        "grad_norm": float(np.linalg.norm(grad)),
        "grad_head": [float(x) for x in grad[:32]],
        "oracle_seconds": time.time() - t0,
    }
    return out


C2_PROBE_SEED = 2


def c2():
    from oracle import space
    w = synth.WORKLOADS["c2"]
    h, g = w.integrals()
    keys = space.full_space(w.n, w.na, w.nb)
    theta = w.theta()
    v = synth.probe_vector(w.P + 1, C2_PROBE_SEED)
    t0 = time.time()
    Z, E_el, grad, pairs = lm.streamed_evaluation(
        keys, w.n, w.V, w.H, theta, lambda x: capply.apply(w.n, h, g, keys, x), [v])
    yH, yS = pairs[0]
    return {
        "workload": "c2",
        "n_dets": int(keys.size),
        "P": int(w.P),
        "probe_seed": C2_PROBE_SEED,
        "Z": Z,
        "E": E_el,
        "grad": [float(x) for x in grad],
        "yH": [float(x) for x in yH],
        "yS": [float(x) for x in yS],
        "oracle_seconds": time.time() - t0,
    }


def _write(name, out):
    path = os.path.join(ROOT, "tests", "golden", name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if not isinstance(v, list)}, indent=1))


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3s", "c2"]
    if "c3s" in which:
        _write("c3s_step.json", c3s())
    if "c2" in which:
        _write("c2_eval.json", c2())
