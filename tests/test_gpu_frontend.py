"""GPU parity of the physical front end: the Fock operator of the reference's
density built from the one-electron operator h (esmp2_fock_from_core) against
the oracle's, elementwise, and the whole pipeline started from h at a
workload size against the stored oracle E2.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import frontend

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12923_amd as p
    return p


@pytest.mark.parametrize("no,nv,na,seed", [(2, 3, 5, 0), (4, 16, 48, 1), (8, 80, 240, 4), (16, 160, 480, 2)])
def test_fock_from_core(lib, no, nv, na, seed):
    print(f"[case] n_occ={no} n_vir={nv} n_aux={na} seed={seed}", flush=True)
    p = synth.make_problem(no, nv, na, seed)
    hcore = p.F - frontend.g_matrix(frontend.density(p.C, no), p.B)
    ref = frontend.fock_from_core(hcore, p.B, p.C, no)
    h = lib.Handle(0)
    ht, Bt, Ct = (torch.from_numpy(a).cuda() for a in (hcore, p.B, p.C))
    Fo = torch.full((no + nv, no + nv), float("nan"), dtype=torch.float64, device="cuda")
    h.fock_from_core(ht, Bt, Ct, no, nv, na, Fo)
    F = Fo.cpu().numpy()
    scale = max(1.0, np.abs(ref).max(), np.abs(hcore).max())     # G[gamma] may be larger than F
    assert np.abs(F - ref).max() <= 1e-13 * scale
    assert np.abs(F - p.F).max() <= 1e-12 * scale
    h.close()


def test_pipeline_from_core(lib):
    """h -> F on the GPU -> rotation, RHS, solve: E2 of the c5 workload."""
    g = GOLD["c5"]
    p = synth.config_problem("c5")
    no, nv, na = p.n_occ, p.n_vir, p.n_aux
    hcore = p.F - frontend.g_matrix(frontend.density(p.C, no), p.B)
    h = lib.Handle(0)
    ht, Bt, Ct = (torch.from_numpy(a).cuda() for a in (hcore, p.B, p.C))
    Fo = torch.empty((no + nv, no + nv), dtype=torch.float64, device="cuda")
    h.fock_from_core(ht, Bt, Ct, no, nv, na, Fo)
    h._n_occ = no
    h.set_problem(Fo, Bt, Ct, no, nv, na)
    h.rotate_top()
    r = h.solve(tol=1e-10, max_iter=300, basis=lib.ESMP2_BASIS_SEMICANONICAL)
    print(f"[c5 from h] E2 diff {r['e2'] - g['e2']:.3e}", flush=True)
    assert r["status"] == 0 and abs(r["e2"] - g["e2"]) < 1e-10
    h.close()
