"""GPU parity of the FP32 operator and of the mixed-precision solve.

FP32 sigma: elementwise against the FP64 oracle within a forward error bound
of FP32 arithmetic.  Every output is a sum of at most K products (the two
Sylvester contractions over the padded virtual dimension, the occupied-index
contractions and the coupling terms), each input rounded once to FP32, so
|y32 - y| <= (gamma_K + 2u) * ||A||_inf * max|x| with u = 2^-24 and
gamma_K = K u / (1 - K u); ||A||_inf is bounded from the TOP-basis Fock blocks.

Mixed solve: E2 within 1e-6 Eh of the stored oracle value, at the FP64
stopping test (relative residual 1e-8).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import structured, topbasis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12923_amd as p
    return p


def _handle(lib, prob):
    print(f"[case] n_occ={prob.n_occ} n_vir={prob.n_vir} n_aux={prob.n_aux} seed={prob.seed}", flush=True)
    return lib.Handle(0).load(prob)


def _op_norm_bound(Ft, lam, no):
    """Upper bound of the infinity norm of A = H0 - E0 on doubles + L-triples."""
    fo, fv, fov = Ft[:no, :no], Ft[no:, no:], Ft[:no, no:]
    rs = lambda M: np.abs(M).sum(axis=1).max()
    om = float(np.sum(lam ** 2 * (np.diag(fv)[:no] - np.diag(fo))))
    ka = fv[0, 0] - fo[0, 0] - om
    return 2 * rs(fv) + 2 * rs(fo) + 12 * np.abs(fov).max() * max(no, Ft.shape[0] - no) + abs(om) + abs(ka)


CANON = [(3, 5, 8, 1), (4, 16, 48, 3), (5, 40, 30, 4), (6, 100, 40, 5), (3, 180, 20, 6), (8, 80, 20, 7),
         (3, 160, 20, 8), (4, 159, 24, 9), (6, 150, 16, 10)]


@pytest.mark.parametrize("no,nv,na,seed", CANON)
def test_sigma_fp32_elementwise(lib, no, nv, na, seed):
    prob = synth.make_canonical_problem(no, nv, na, seed)
    h = _handle(lib, prob)
    h.rotate_top()
    lam, R = topbasis.top_rotation(prob.F, prob.C, no)
    Ft, _ = topbasis.rotate(prob.F, prob.B, R)
    op = structured.Structured(Ft, lam, no)
    n, offs = h.space()
    x = synth.random_amplitudes(n, seed + 200)
    ref = op.sigma(x)
    xt = torch.from_numpy(x).to(torch.float32).cuda()
    yt = torch.full_like(xt, float("nan"))
    h.sigma(xt, yt, precision=lib.ESMP2_FP32)
    # FP64 operator on the same device buffers, for the launch path comparison
    y64 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    h.sigma(torch.from_numpy(x).cuda(), y64)
    torch.cuda.synchronize()
    y = yt.cpu().numpy().astype(np.float64)
    assert np.isfinite(y).all()
    mv = 16 * ((nv + 15) // 16)
    K = 2 * mv + 2 * no + 24
    gam = K * U32 / (1 - K * U32)
    bound = (gam + 2 * U32) * _op_norm_bound(Ft, lam, no) * np.abs(x).max()
    err = np.abs(y - ref)
    print(f"[fp32 sigma] max err {err.max():.3e} bound {bound:.3e} rms err {np.sqrt((err ** 2).mean()):.3e}",
          flush=True)
    for k in range(7):
        lo, hi = offs[k], offs[k + 1]
        if hi > lo:
            assert err[lo:hi].max() <= bound, (k, err[lo:hi].max(), bound)
    assert np.abs(y64.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    h.close()


@pytest.mark.parametrize("name", ["c1", "c5", "c2", "c3"])
def test_mixed_e2_workloads(lib, name):
    """Mixed-precision E2 within 1e-6 Eh of the oracle at relative residual 1e-8."""
    g = GOLD[name]
    prob = synth.config_problem(name)
    h = _handle(lib, prob)
    h.rotate_top()
    n, _ = h.space()
    xo = torch.empty(n, dtype=torch.float64, device="cuda")
    res = h.solve(tol=1e-8, max_iter=300, precision=lib.ESMP2_FP32, x_out=xo, history=True)
    torch.cuda.synchronize()
    print(f"[{name} mixed] E2 {res['e2']:.12f} oracle {g['e2']:.12f} diff {res['e2'] - g['e2']:.3e} "
          f"inner {res['iterations']} outer {res['outer']} resid {res['rel_resid']:.2e}", flush=True)
    assert res["status"] == 0
    assert res["rel_resid"] <= 1e-8
    assert res["outer"] >= 1
    assert abs(res["e2"] - g["e2"]) <= 1e-6
    assert abs(res["e2_s"] - g["e2_s"]) < 1e-10
    idx = np.array(g["sample_idx"])
    xs = xo.cpu().numpy()[idx]
    assert np.abs(xs - np.array(g["x_sample"])).max() <= 1e-6 * np.abs(g["x_sample"]).max()
    assert len(res["history"]) == res["iterations"]
    h.close()


def test_mixed_matches_fp64_and_inner_tolerances(lib):
    """FP64 and mixed solves of one problem; loose and tight inner solves agree."""
    prob = synth.config_problem("c5")
    h = _handle(lib, prob)
    h.rotate_top()
    r64 = h.solve(tol=1e-8, max_iter=300)
    out = []
    for itol in (1e-2, 1e-3, 1e-5):
        r = h.solve(tol=1e-8, max_iter=300, precision=lib.ESMP2_FP32, inner_tol=itol)
        print(f"[c5 mixed inner_tol={itol}] inner {r['iterations']} outer {r['outer']} "
              f"E2-E2_64 {r['e2'] - r64['e2']:.3e}", flush=True)
        assert r["status"] == 0 and r["rel_resid"] <= 1e-8
        assert abs(r["e2"] - r64["e2"]) <= 1e-6
        out.append(r)
    assert out[0]["outer"] >= out[2]["outer"]
    # warm start from the solution: converged at entry, no inner iteration
    n, _ = h.space()
    xo = torch.empty(n, dtype=torch.float64, device="cuda")
    h.solve(tol=1e-10, max_iter=300, x_out=xo)
    r = h.solve(tol=1e-8, max_iter=300, precision=lib.ESMP2_FP32, x0=xo)
    assert r["iterations"] == 0 and r["outer"] == 0 and r["status"] == 0
    h.close()


def test_mixed_max_iter_reports_not_converged(lib):
    prob = synth.config_problem("c1")
    h = _handle(lib, prob)
    h.rotate_top()
    r = h.solve(tol=1e-12, max_iter=3, precision=lib.ESMP2_FP32)
    assert r["status"] == lib.ESMP2_NOT_CONVERGED
    assert r["iterations"] == 3
    with pytest.raises(lib.Esmp2Error):
        h.solve(tol=1e-8, max_iter=10, precision=lib.ESMP2_FP32, inner_tol=1.5)
    h.close()
