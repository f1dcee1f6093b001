"""The seeded workloads against what they transcribe (CPU): the runs of the
parametric study are the cases of Table 1 (tests/golden/table1_cases.json,
transcribed from Sec. 2), expanded the way Sec. 4 uses them."""
import json
import os

from paper_1603_08221_amd.workloads import HE_AR, NE_AR, TABLE1, table1_instances

HERE = os.path.dirname(os.path.abspath(__file__))


def test_table1_matches_the_transcribed_cases():
    g = json.load(open(os.path.join(HERE, "golden", "table1_cases.json")))
    assert (g["lattice"]["ny"], g["lattice"]["nx"]) == (20, 700)
    cases = {c["case"]: c for c in g["cases"]}
    assert len(TABLE1) == len(cases) == 10
    for case, pair, cin, cout, kns, thetas in TABLE1:
        c = cases[case]
        assert c["mixture"] == pair and c["cl_in"] == cin and c["cl_out"] == cout
        assert list(kns) == c["kn_out"] and list(thetas) == c["theta"]
    masses = {"He-Ar": HE_AR, "Ne-Ar": NE_AR}
    for name, (a, b) in g["mass_ratio"].items():
        assert masses[name][1] / masses[name][0] == b / a


def test_table1_expansion():
    """Cases 2 and 7: the theta sweep at Kn_out = 0.3 (Sec. 4.1) and the Kn_out
    sweep at theta = 2 (Sec. 4.2) share one run; Cases 1, 3, 6, 8 at the listed
    theta = 4 and at the theta = 2 of Sec. 4.3; Cases 4, 5, 9, 10 at each
    listed Kn_out. 32 runs on the 20 x 700 lattice, all with C_in, C_out, theta,
    Kn_out and the pair of their case."""
    runs = table1_instances()
    names = [w.name for w in runs]
    assert len(runs) == len(set(names)) == 32
    assert all((w.ny, w.nx) == (20, 700) for w in runs)
    for c in (2, 7):
        assert {n for n in names if n.startswith(f"c{c}_")} == (
            {f"c{c}_th{t}_kn0.3" for t in (2, 3, 4, 5)} | {f"c{c}_th2_kn{k:g}" for k in (0.3, 0.5, 1, 3, 5)})
    for c in (1, 3, 6, 8):
        assert {n for n in names if n.startswith(f"c{c}_")} == {f"c{c}_th4_kn0.3", f"c{c}_th2_kn0.3"}
    for c in (4, 5, 9, 10):
        assert {n for n in names if n.startswith(f"c{c}_")} == {f"c{c}_th2_kn0.3", f"c{c}_th2_kn1"}
    w = next(w for w in runs if w.name == "c9_th2_kn1")
    assert (w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out) == (*NE_AR, 0.7, 0.3, 2.0, 1.0)
    assert table1_instances(10, 350)[0].nx == 350
