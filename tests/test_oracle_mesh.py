"""Pins of the oracle's icosahedron subdivision mesh (Sec. II.D) against
Table 1 and the mean edge lengths quoted in Sec. IV.B."""
import os
from collections import defaultdict

import numpy as np
import pytest

from paper_1004_2416_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].split()
        if len(line) == 2:
            out[line[0]] = float(line[1])
    return out


def mesh_statistics(x, t):
    e = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]]), 1)
    ue = np.unique(e, axis=0)
    nnb = np.bincount(ue.ravel())
    cr = np.cross(x[t[:, 1]] - x[t[:, 0]], x[t[:, 2]] - x[t[:, 0]])
    A = 0.5 * np.linalg.norm(cr, axis=1)
    L = np.linalg.norm(x[ue[:, 0]] - x[ue[:, 1]], axis=1)
    nrm = cr / np.linalg.norm(cr, axis=1)[:, None]
    ef = defaultdict(list)
    for j, tr in enumerate(t):
        for a, b in ((0, 1), (1, 2), (2, 0)):
            ef[(min(tr[a], tr[b]), max(tr[a], tr[b]))].append(j)
    phn = np.array([np.arccos(np.clip(nrm[f[0]] @ nrm[f[1]], -1, 1)) for f in ef.values()])
    ang = []
    for tr in t:
        for k in range(3):
            a, b, c = x[tr[k]], x[tr[(k + 1) % 3]], x[tr[(k + 2) % 3]]
            u, v = b - a, c - a
            ang.append(np.arccos(u @ v / np.linalg.norm(u) / np.linalg.norm(v)))
    ang = np.array(ang)
    return dict(N_f=len(t), Nnn_min=nnb.min(), Nnn_max=nnb.max(),
                sigmaA_over_A=100 * A.std() / A.mean(),
                sigmal_over_l=100 * L.std() / L.mean(),
                sigmaphin_over_phin=100 * phn.std() / phn.mean(),
                sigmaphie_over_phie=100 * ang.std() / ang.mean(),
                lbar=L.mean(), edges_per=np.unique(e, axis=0, return_counts=True)[1])


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_counts_closed_oriented(orc, level):
    x, t = orc.icosphere(level, 2.0, (1.0, -2.0, 3.0))
    nn, nf = W.icosphere_counts(level)
    assert x.shape == (nn, 3) and t.shape == (nf, 3)
    assert np.allclose(np.linalg.norm(x - [1.0, -2.0, 3.0], axis=1), 2.0, atol=1e-14)
    # closed 2-manifold: every undirected edge shared by two faces, every
    # directed edge used once (consistent orientation)
    d = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    assert len(np.unique(d, axis=0)) == len(d)
    assert np.all(mesh_statistics(x, t)["edges_per"] == 2)
    # outward normals: positive enclosed volume, every face normal outward
    c = x[t].mean(1) - [1.0, -2.0, 3.0]
    cr = np.cross(x[t[:, 1]] - x[t[:, 0]], x[t[:, 2]] - x[t[:, 0]])
    assert np.all((cr * c).sum(1) > 0)


def test_table1_subdivision_column(orc):
    gold = _golden("table1_subdivision.txt")
    x, t = orc.icosphere(3, 1.0)
    st = mesh_statistics(x, t)
    assert st["N_f"] == gold["N_f"]
    assert st["Nnn_min"] == gold["Nnn_min"] and st["Nnn_max"] == gold["Nnn_max"]
    for k in ("sigmaA_over_A", "sigmal_over_l", "sigmaphin_over_phin", "sigmaphie_over_phie"):
        assert round(st[k], 1) == gold[k], (k, st[k])


def test_mean_edge_length(orc):
    gold = _golden("mean_edge_length_r5.txt")
    for level, nf in ((2, 320), (3, 1280), (4, 5120)):
        x, t = orc.icosphere(level, 5.0)
        assert round(mesh_statistics(x, t)["lbar"], 2) == gold[str(nf)]
