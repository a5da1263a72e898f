#!/usr/bin/env python
"""Write the oracle's reference results for full-size elements (test fixtures).

Runs only the CPU oracle (``oracle/``) on inputs from ``workloads`` and stores,
per element, what the GPU parity tests compare against:

* the oracle's LOBPCG Ritz values (Algorithm 1, run to max_i ||r_i|| <= 1e-10,
  tighter than the 1e-8 Ha target), their residual norms and iteration count,
  and the gap between the last wanted and the first guard Ritz value;
* the ALB singular values (SVD of the eigenvectors restricted to E_k, the ALB
  construction of the "Generating ALB functions" subsection);
* for the elements named in ALB_ELEMENTS, an orthonormal ALB basis U stored in
  float32 (re-orthonormalised in float64 on load; the rounding moves the span
  by ~4e-8 rad, far below the 1e-6 rad angle tolerance).  These elements are
  solved to 1e-12: the ALB span amplifies an eigenvector error by 1 / sigma_min
  of the restriction (down to 6e-7 on this slab), so the angle test needs
  eigenvectors well inside the 1e-6 rad it asserts.

Output: tests/golden/fullsize/<config>_oracle.json and
<config>_e<k>_alb_f32.npy.  Usage:
    python tests/golden/make_fullsize_refs.py c2 [element ...]
Each element is solved from the seeded start initial_block(N, J + g,
seed_base + k) of its config; every run is deterministic up to BLAS rounding.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import alb as oalb  # noqa: E402
from oracle import lobpcg as olob  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize")
TOL = 1e-10
TOL_ALB = 1e-12
# elements whose ALB basis is stored (the angle tests); the other elements keep
# eigenvalues, residuals, gaps and singular values only
ALB_ELEMENTS = {"c2": (0, 9, 10, 11), "c3": (0,), "c4": ()}


def solve_element(cfg, k, tol):
    el = cfg.elements[k]
    J = el.n_states
    g = W.guard_count(J)
    x0 = W.initial_block(el.npts, J + g, cfg.x0_seed_base + k).T
    t0 = time.perf_counter()
    r = olob.lobpcg(el, x0, J, tol=tol, max_iter=800)
    dt = time.perf_counter() - t0
    U, s = oalb.make_alb(el, r.X, J)
    rec = {
        "grid": list(el.n), "n_states": J, "n_guard": g, "tol": tol, "iters": int(r.iters),
        "converged": bool(r.converged), "seconds": round(dt, 1),
        "eigvals": [float(v) for v in r.eigvals],
        "resid": [float(v) for v in r.resid],
        "gap": float(r.eigvals[J] - r.eigvals[J - 1]),
        "sigma": [float(v) for v in s],
    }
    return rec, U


def main(argv):
    name = argv[1]
    cfg = W.make_config(name)
    ks = [int(a) for a in argv[2:]] or list(range(cfg.n_elem))
    os.makedirs(OUT, exist_ok=True)
    path = os.path.join(OUT, f"{name}_oracle.json")
    data = {"config": name, "tol": TOL, "method": "oracle LOBPCG (Algorithm 1), FP64", "elements": {}}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    for k in ks:
        rec, U = solve_element(cfg, k, TOL_ALB if k in ALB_ELEMENTS.get(name, ()) else TOL)
        data["elements"][str(k)] = rec
        if k in ALB_ELEMENTS.get(name, ()):
            np.save(os.path.join(OUT, f"{name}_e{k}_alb_f32.npy"), U.astype(np.float32))
        data["elements"] = dict(sorted(data["elements"].items(), key=lambda kv: int(kv[0])))
        with open(path, "w") as f:
            json.dump(data, f, indent=1)
        print(f"{name} element {k}: {rec['iters']} iterations, {rec['seconds']} s, "
              f"max residual {max(rec['resid'][:rec['n_states']]):.1e}, gap {rec['gap']:.3e}", flush=True)


if __name__ == "__main__":
    main(sys.argv)
