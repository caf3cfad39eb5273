"""GPU parity of the solve in the pinned-semicanonical basis.

The library rotates the occupied orbitals other than t and the virtuals other
than t' so that their Fock blocks are diagonal, rotates b, solves there and
rotates x back.  E2 and the solution (in the TOP basis) must equal the
oracle's TOP-basis values: E2 to 1e-10 Eh, sampled amplitudes to 1e-8
relative at a residual of 1e-10.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import structured

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12923_amd as p
    return p


def _handle(lib, prob):
    print(f"[case] n_occ={prob.n_occ} n_vir={prob.n_vir} n_aux={prob.n_aux} seed={prob.seed}", flush=True)
    return lib.Handle(0).load(prob)


@pytest.mark.parametrize("no,nv,na,seed", [(3, 5, 8, 1), (4, 7, 9, 4), (5, 12, 14, 2), (2, 6, 5, 3)])
def test_semican_small_random_basis(lib, no, nv, na, seed):
    prob = synth.make_problem(no, nv, na, seed)
    h = _handle(lib, prob)
    h.rotate_top()
    res = h.solve(tol=1e-12, max_iter=200, basis=lib.ESMP2_BASIS_SEMICANONICAL)
    ref = structured.solve_problem(prob, tol=1e-13)
    assert res["status"] == 0
    assert abs(res["e2"] - ref["e2"]) < 1e-10
    h.close()


@pytest.mark.parametrize("name", ["c1", "c5", "c2", "c3"])
def test_semican_workloads(lib, name):
    g = GOLD[name]
    prob = synth.config_problem(name)
    h = _handle(lib, prob)
    h.rotate_top()
    n, _ = h.space()
    xo = torch.empty(n, dtype=torch.float64, device="cuda")
    res = h.solve(tol=1e-10, max_iter=300, x_out=xo, basis=lib.ESMP2_BASIS_SEMICANONICAL)
    torch.cuda.synchronize()
    top = h.solve(tol=1e-10, max_iter=300)
    print(f"[{name} semican] E2 {res['e2']:.12f} oracle {g['e2']:.12f} diff {res['e2'] - g['e2']:.3e} "
          f"iters {res['iterations']} (TOP basis {top['iterations']})", flush=True)
    assert res["status"] == 0 and res["rel_resid"] <= 1e-10
    assert abs(res["e2"] - g["e2"]) < 1e-10
    assert abs(res["e2_s"] - g["e2_s"]) < 1e-10
    assert res["iterations"] < top["iterations"]
    idx = np.array(g["sample_idx"])
    xs = xo.cpu().numpy()[idx]
    assert np.abs(xs - np.array(g["x_sample"])).max() <= 1e-8 * np.abs(g["x_sample"]).max()
    # warm start from the TOP-basis solution: converged at entry
    r0 = h.solve(tol=1e-8, max_iter=300, x0=xo, basis=lib.ESMP2_BASIS_SEMICANONICAL)
    assert r0["iterations"] == 0 and r0["status"] == 0
    assert abs(r0["e2"] - g["e2"]) < 1e-9
    h.close()


@pytest.mark.parametrize("name", ["c5", "c3"])
def test_semican_mixed(lib, name):
    g = GOLD[name]
    prob = synth.config_problem(name)
    h = _handle(lib, prob)
    h.rotate_top()
    res = h.solve(tol=1e-8, max_iter=300, precision=lib.ESMP2_FP32, basis=lib.ESMP2_BASIS_SEMICANONICAL)
    print(f"[{name} semican mixed] diff {res['e2'] - g['e2']:.3e} inner {res['iterations']} outer {res['outer']}",
          flush=True)
    assert res["status"] == 0 and res["rel_resid"] <= 1e-8
    assert abs(res["e2"] - g["e2"]) <= 1e-6
    with pytest.raises(lib.Esmp2Error):
        h.solve(tol=1e-8, max_iter=10, basis=7)
    h.close()
