"""Write the oracle's reference solution of the k = 10 periodic workload
(first seeded incidence) to tests/golden/periodic_k10_wave0.json.

Calls only the CPU oracle (oracle/) on the inputs of workloads/; takes
several minutes on a workstation.  The GPU parity test compares libmfs's
solve of the same incidence with these values.

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import geometry, onebody, periodic  # noqa: E402


def main():
    pr = W.periodic_k10(1)
    b, lat = pr.body, pr.lattice
    t0 = time.time()
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    ps = periodic.PeriodicSolver(b, lat, g, A)
    w = pr.waves[0]
    ps.set_wave(w)
    fh = onebody.rhs_modes(b, g, w)
    res = ps.solve(fh, tol=1e-12, maxit=pr.maxit)
    u, _ = ps.field_and_grad(res["c"], res["d"], pr.targets, pr.q_field, want_grad=False)
    o = ps.orders
    out = {
        "source": "oracle (tests/golden/make_golden.py)",
        "workload": "periodic_k10, incidence 0, GMRES tol 1e-12",
        "lattice": {"ex": lat.ex, "ey": lat.ey, "z0": lat.z0, "p": lat.p, "N0": lat.N0, "M1": lat.M1},
        "theta": w.theta, "phi": w.phi,
        "iters": int(res["iters"]),
        "gmres_resid": float(res["hist"][-1]),
        "eps_flux": ps.eps_flux(res["a"], res["b"]),
        "eps_per": ps.eps_per(res["c"], res["d"], pr.q_field),
        "eps_bc": ps.eps_bc(res["c"], res["d"], b.q),
        "m": o.m.tolist(), "n": o.n.tolist(),
        "a_re": res["a"].real.tolist(), "a_im": res["a"].imag.tolist(),
        "b_re": res["b"].real.tolist(), "b_im": res["b"].imag.tolist(),
        "targets": pr.targets.tolist(), "q_field": pr.q_field,
        "u_re": u.real.tolist(), "u_im": u.imag.tolist(),
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "periodic_k10_wave0.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote golden in {out['seconds']:.0f} s, {out['iters']} iterations, eps_flux {out['eps_flux']:.2e}, "
          f"eps_per {out['eps_per']:.2e}, eps_bc {out['eps_bc']:.2e}")


if __name__ == "__main__":
    main()
