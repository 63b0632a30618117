"""Writes synthetic Les Houches event files for the tests (the paper's event
files are not available): seeded events of a process, each boosted along the
beam axis by its own random rapidity into a "lab" frame, particles listed in
a shuffled order with an intermediate (status 2) line, momenta printed with
17 significant digits."""
import numpy as np

PDG = {"gg_tt": [21, 21, 6, -6], "gg_ttg": [21, 21, 6, -6, 21], "gg_ttgg": [21, 21, 6, -6, 21, 21],
       "ee_5a": [-11, 11, 22, 22, 22, 22, 22]}
MASS = {21: 0.0, 6: 173.0, -6: 173.0, 11: 0.0, -11: 0.0, 22: 0.0}

HEADER = """<LesHouchesEvents version="3.0">
<header>
<!-- synthetic test sample -->
</header>
<init>
2212 2212 6.5e3 6.5e3 0 0 0 0 3 1
1.0e0 1.0e-2 1.0e0 1
</init>
"""


def write_lhe(path, proc, mom_cm, w, seed=3, rwgt_block=False):
    """mom_cm [n_ext, 4, N] (E, px, py, pz) in the partonic CM frame; returns
    the rapidities used for the boosts."""
    rng = np.random.default_rng(seed)
    n_ext, _, n = mom_cm.shape
    ids = PDG[proc]
    ys = rng.uniform(-1.5, 1.5, n)
    lines = [HEADER]
    for e in range(n):
        ch, sh = np.cosh(ys[e]), np.sinh(ys[e])
        parts = []
        for i in range(n_ext):
            E, px, py, pz = mom_cm[i, :, e]
            El, pzl = ch * E + sh * pz, sh * E + ch * pz
            status = -1 if i < 2 else 1
            parts.append((ids[i], status, (px, py, pzl, El, MASS[ids[i]])))
        order = [0, 1] + list(rng.permutation(np.arange(2, n_ext)))
        # an intermediate line, e.g. a resonance the generator recorded
        inter = (9000001, 2, (0.0, 0.0, 0.0, 1.0, 1.0))
        body = [parts[k] for k in order]
        body.insert(2, inter)
        lines.append("<event>\n")
        lines.append(f" {len(body)} 1 {w[e]:.17e} 1.00000000e+02 7.54677100e-03 1.18000000e-01\n")
        for pid, st, p in body:
            lines.append(f" {pid:8d} {st:2d} 1 2 501 0 " + " ".join(f"{x:.17e}" for x in p) + " 0.0 9.0\n")
        if rwgt_block:
            lines.append("<rwgt>\n<wgt id='old'> 1.5 </wgt>\n</rwgt>\n")
        lines.append("</event>\n")
    lines.append("</LesHouchesEvents>\n")
    with open(path, "w") as f:
        f.write("".join(lines))
    return ys
