"""GPU parity of the BF16 operator and of the solve refined around it.

BF16 sigma: the FP32 operator except that the virtual-pair Fock products take
BF16 operands (F' and x each rounded once to 8 significant bits, nearest even)
with FP32 matrix-core accumulation.  Every product in an output then carries a
relative error of at most 2 u_b + u_b^2 (u_b = 2^-8) from the two roundings,
plus the FP32 accumulation and input rounding of the FP32 operator, so
|y_bf16 - y| <= (2 u_b + u_b^2 + gamma_K + 2u) * ||A||_inf * max|x|
(u = 2^-24, K terms per output, ||A||_inf bounded from the TOP-basis Fock
blocks as in the FP32 test).  The RMS error must also sit at the BF16 level,
far below that worst case, and the difference to the FP32 operator is bounded
the same way.

Refined solve: E2 within 1e-6 Eh of the stored oracle value at the FP64
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
UB = 2.0 ** -8


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


# padded virtual dimensions 80, 112 and 160 (the sizes with a BF16 kernel), ragged n_vir included
CASES = [(3, 80, 20, 11), (8, 80, 20, 7), (4, 100, 30, 12), (5, 112, 16, 13), (3, 160, 20, 14), (4, 159, 12, 15)]


@pytest.mark.parametrize("no,nv,na,seed", CASES)
def test_sigma_bf16_elementwise(lib, no, nv, na, seed):
    prob = synth.make_canonical_problem(no, nv, na, seed)
    h = _handle(lib, prob)
    h.rotate_top()
    lam, R = topbasis.top_rotation(prob.F, prob.C, no)
    Ft, _ = topbasis.rotate(prob.F, prob.B, R)
    op = structured.Structured(Ft, lam, no)
    n, offs = h.space()
    x = synth.random_amplitudes(n, seed + 300)
    ref = op.sigma(x)
    xt = torch.from_numpy(x).to(torch.float32).cuda()
    yb = torch.full_like(xt, float("nan"))
    y32 = torch.full_like(xt, float("nan"))
    h.sigma(xt, yb, precision=lib.ESMP2_BF16)
    h.sigma(xt, y32, precision=lib.ESMP2_FP32)
    torch.cuda.synchronize()
    y = yb.cpu().numpy().astype(np.float64)
    assert np.isfinite(y).all()
    mv = 16 * ((nv + 15) // 16)
    K = 2 * mv + 2 * no + 24
    gam = K * U32 / (1 - K * U32)
    scale = _op_norm_bound(Ft, lam, no) * np.abs(x).max()
    bound = (2 * UB + UB * UB + gam + 2 * U32) * scale
    err = np.abs(y - ref)
    rms = np.sqrt((err ** 2).mean())
    print(f"[bf16 sigma] max err {err.max():.3e} bound {bound:.3e} rms err {rms:.3e} "
          f"rms |y| {np.sqrt((ref ** 2).mean()):.3e}", flush=True)
    for k in range(7):
        lo, hi = offs[k], offs[k + 1]
        if hi > lo:
            assert err[lo:hi].max() <= bound, (k, err[lo:hi].max(), bound)
    # rounding errors of independent products average out: the RMS error is at
    # the BF16 level of the typical output, not at the worst case
    assert rms <= 2 * UB * np.sqrt((ref ** 2).mean())
    assert np.abs(y - y32.cpu().numpy()).max() <= bound
    h.close()


@pytest.mark.parametrize("name", ["c5", "c2", "c3"])
def test_bf16_refined_e2_workloads(lib, name):
    """E2 of the solve refined around the BF16 operator within 1e-6 Eh of the oracle."""
    g = GOLD[name]
    prob = synth.config_problem(name)
    h = _handle(lib, prob)
    h.rotate_top()
    n, _ = h.space()
    xo = torch.empty(n, dtype=torch.float64, device="cuda")
    res = h.solve(tol=1e-8, max_iter=500, precision=lib.ESMP2_BF16, x_out=xo)
    torch.cuda.synchronize()
    print(f"[{name} bf16] E2 {res['e2']:.12f} oracle {g['e2']:.12f} diff {res['e2'] - g['e2']:.3e} "
          f"inner {res['iterations']} outer {res['outer']} resid {res['rel_resid']:.2e}", flush=True)
    assert res["status"] == 0
    assert res["rel_resid"] <= 1e-8
    assert res["outer"] >= 2
    assert abs(res["e2"] - g["e2"]) <= 1e-6
    idx = np.array(g["sample_idx"])
    assert np.abs(xo.cpu().numpy()[idx] - np.array(g["x_sample"])).max() <= 1e-6 * np.abs(g["x_sample"]).max()
    h.close()


def test_bf16_unsupported_cases(lib):
    # padded virtual dimension 16: no BF16 kernel
    prob = synth.config_problem("c1")
    h = _handle(lib, prob)
    h.rotate_top()
    n, _ = h.space()
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(lib.Esmp2Error) as e:
        h.sigma(x, y, precision=lib.ESMP2_BF16)
    assert e.value.status == lib.ESMP2_UNSUPPORTED
    with pytest.raises(lib.Esmp2Error) as e:
        h.solve(tol=1e-8, max_iter=10, precision=lib.ESMP2_BF16)
    assert e.value.status == lib.ESMP2_UNSUPPORTED
    h.close()
    # the pinned-semicanonical solve has no Sylvester products
    prob = synth.config_problem("c5")
    h = _handle(lib, prob)
    h.rotate_top()
    with pytest.raises(lib.Esmp2Error) as e:
        h.solve(tol=1e-8, max_iter=10, precision=lib.ESMP2_BF16, basis=lib.ESMP2_BASIS_SEMICANONICAL)
    assert e.value.status == lib.ESMP2_UNSUPPORTED
    h.close()


@pytest.mark.parametrize("no,nv,na,seed", [(4, 80, 16, 21), (3, 112, 12, 22)])
def test_sigma_bf16_triplet(lib, no, nv, na, seed):
    """The M_s = 0 triplet (flip partners with opposite amplitudes) through the BF16 kernel."""
    print(f"[case] triplet bf16 n_occ={no} n_vir={nv} n_aux={na} seed={seed}", flush=True)
    prob = synth.make_problem(no, nv, na, seed)
    lam, R = topbasis.top_rotation(prob.F, prob.C, no)
    Ft, Bt = topbasis.rotate(prob.F, prob.B, R)
    lam, Ft, Bt = (np.ascontiguousarray(a) for a in (lam, Ft, Bt))
    h = lib.Handle(0)
    dev = [torch.from_numpy(a).cuda() for a in (Ft, Bt, lam)]
    h.set_problem_top(dev[0], dev[1], dev[2], no, nv, na, spin=1)
    h.rotate_top(False)
    op = structured.Structured(Ft, lam, no, spin=1)
    n, offs = h.space()
    x = synth.random_amplitudes(n, seed + 600)
    ref = op.sigma(x)
    xt = torch.from_numpy(x).to(torch.float32).cuda()
    yb = torch.full_like(xt, float("nan"))
    h.sigma(xt, yb, precision=lib.ESMP2_BF16)
    torch.cuda.synchronize()
    y = yb.cpu().numpy().astype(np.float64)
    mv = 16 * ((nv + 15) // 16)
    K = 2 * mv + 2 * no + 24
    gam = K * U32 / (1 - K * U32)
    bound = (2 * UB + UB * UB + gam + 2 * U32) * _op_norm_bound(Ft, lam, no) * np.abs(x).max()
    err = np.abs(y - ref)
    print(f"[bf16 triplet sigma] max err {err.max():.3e} bound {bound:.3e}", flush=True)
    assert err.max() <= bound
    assert np.sqrt((err ** 2).mean()) <= 2 * UB * np.sqrt((ref ** 2).mean())
    h.close()


def test_bf16_refined_e2_triplet_workload(lib):
    g = GOLD["c5_triplet"]
    prob = synth.config_problem("c5")
    print("[case] triplet c5 bf16", flush=True)
    h = lib.Handle(0).load(prob, spin=1)
    h.rotate_top()
    res = h.solve(tol=1e-8, max_iter=500, precision=lib.ESMP2_BF16)
    print(f"[c5 triplet bf16] E2 {res['e2']:.12f} oracle {g['e2']:.12f} diff {res['e2'] - g['e2']:.3e} "
          f"outer {res['outer']}", flush=True)
    assert res["status"] == 0 and res["rel_resid"] <= 1e-8
    assert abs(res["e2"] - g["e2"]) <= 1e-6
    h.close()
