"""Writes tests/golden/ne_ar_64x1280_2000.json: sampled outputs of the CPU
oracle on the full-size Ne-Ar 64 x 1280 channel (C_l 0.3, theta 3, Kn_out
0.05, DBB r from Eq. (R) with c_m = 0.8183) after 2000 steps from the initial
state. Calls only oracle/ (and the seeded workload description). Run:
python tests/golden/make_ne_ar_64x1280_reference.py  (a few minutes)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import binary_lbm as O  # noqa: E402
from paper_1603_08221_amd.workloads import CONFIGS  # noqa: E402

STEPS = 2000
ROWS = [0, 1, 16, 31, 32, 62, 63]
COLS = list(range(0, 1280, 32)) + [1, 2, 1277, 1278, 1279]


def main():
    w = CONFIGS["ne_ar_64x1280"]
    r = O.dbb_r_from_cm(w.c_m, w.m_a, w.m_b, w.cl_in)
    p = O.Params(nx=w.nx, ny=w.ny, m_a=w.m_a, m_b=w.m_b, cl_in=w.cl_in, cl_out=w.cl_out, theta=w.theta,
                 kn_out=w.kn_out, dbb_r=r, accom=w.accom)
    f, _ = O.run(p, STEPS)
    d = O.diagnostics(f, p)
    mf = O.moment_fields(f, p)
    out = {"source": "oracle/binary_lbm.py, Ne-Ar 64 x 1280, C_l 0.3, theta 3, Kn_out 0.05, %d steps" % STEPS,
           "steps": STEPS, "dbb_r": r, "cl": d.cl, "cl_tilde": d.cl_tilde, "x_min": int(d.x_min),
           "cl_profile": d.cl_profile.tolist(), "rows": ROWS, "cols": COLS,
           "moments": {name: [[float(mf[k, j, x]) for x in COLS] for j in ROWS]
                       for k, name in enumerate(("rho_a", "rho_b", "u_ax", "u_ay", "u_bx", "u_by"))}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ne_ar_64x1280_2000.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(path, d.cl)


if __name__ == "__main__":
    main()
