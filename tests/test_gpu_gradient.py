"""GPU parity of the derivatives of E2 with respect to the TOP-basis Fock
matrix and factor (esmp2_gradient, and its torch.autograd wrapper).

* tiny problems: every entry of both gradients against the oracle's
  (exact central differences of the stationary functional);
* the n_occ = 8, n_vir = 80, n_aux = 240 workload: 50 + 50 seeded entries
  against the stored oracle values, and 50 entries against central
  differences (step 1e-5) of the GPU's own E2, re-solved at each point;
* the N_o = 16 workload and the n_occ = 8 one: Euler's identity
  <F~, dF> + <B~, dB> / 2 = E2 (H scales by s under F~ -> s F~,
  B~ -> sqrt(s) B~), a property of the whole gradient at any size.
Relative errors are taken against the largest entry of the gradient.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import gradient, topbasis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12923_amd as p
    return p


def _top(prob):
    lam, R = topbasis.top_rotation(prob.F, prob.C, prob.n_occ)
    Ft, Bt = topbasis.rotate(prob.F, prob.B, R)
    return np.ascontiguousarray(lam), np.ascontiguousarray(Ft), np.ascontiguousarray(Bt)


def _gpu_grad(lib, h, Ft, Bt, lam, no, tol=1e-12, basis=None):
    n = Ft.shape[0]
    na = Bt.shape[0]
    dev = [torch.from_numpy(a).cuda() for a in (Ft, Bt, lam)]
    h.set_problem_top(dev[0], dev[1], dev[2], no, n - no, na)
    h.rotate_top(False)
    h.build_rhs()
    n_amp, _ = h.space()
    x = torch.empty(n_amp, dtype=torch.float64, device="cuda")
    b = lib.ESMP2_BASIS_SEMICANONICAL if basis is None else basis
    r = h.solve(tol=tol, max_iter=1000, basis=b, x_out=x, allow=())
    dF = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    dB = torch.full((na, n, n), float("nan"), dtype=torch.float64, device="cuda")
    h.gradient(x, dF, dB)
    torch.cuda.synchronize()
    return r, dF.cpu().numpy(), dB.cpu().numpy()


@pytest.mark.parametrize("no,nv,na,seed", [(3, 6, 5, 1), (2, 5, 4, 3), (4, 7, 6, 2), (2, 2, 3, 5)])
def test_gradient_tiny_every_entry(lib, no, nv, na, seed):
    print(f"[case] gradient n_occ={no} n_vir={nv} n_aux={na} seed={seed}", flush=True)
    prob = synth.make_problem(no, nv, na, seed)
    lam, Ft, Bt = _top(prob)
    L = gradient.Lagrangian(Ft, Bt, lam, no)
    GF, GB = L.full_gradient()
    h = lib.Handle(0)
    for basis in (lib.ESMP2_BASIS_TOP, lib.ESMP2_BASIS_SEMICANONICAL):
        r, dF, dB = _gpu_grad(lib, h, Ft, Bt, lam, no, tol=1e-13, basis=basis)
        assert abs(r["e2"] - L.e2) < 1e-12
        scale = max(np.abs(GF).max(), np.abs(GB).max())
        assert np.abs(dF - GF).max() <= 1e-10 * scale, (basis, np.abs(dF - GF).max(), scale)
        assert np.abs(dB - GB).max() <= 1e-10 * scale, (basis, np.abs(dB - GB).max(), scale)
        assert np.array_equal(dF, dF.T) and np.array_equal(dB, dB.transpose(0, 2, 1))
    h.close()


@pytest.fixture(scope="module")
def c5(lib):
    prob = synth.config_problem("c5")
    lam, Ft, Bt = _top(prob)
    h = lib.Handle(0)
    r, dF, dB = _gpu_grad(lib, h, Ft, Bt, lam, prob.n_occ, tol=1e-12)
    yield dict(prob=prob, lam=lam, Ft=Ft, Bt=Bt, h=h, r=r, dF=dF, dB=dB)
    h.close()


def test_gradient_c5_oracle_samples(c5):
    g = GOLD["c5_grad"]
    assert abs(c5["r"]["e2"] - GOLD["c5"]["e2"]) < 1e-10
    assert abs(c5["r"]["e2"] - g["e2"]) < 1e-10
    dF, dB = c5["dF"], c5["dB"]
    scale = max(np.abs(dF).max(), np.abs(dB).max())
    ef = max(abs(dF[p, q] - v) for (p, q), v in zip(g["f_entries"], g["f_grad"]))
    eb = max(abs(dB[Q, p, q] - v) for (Q, p, q), v in zip(g["b_entries"], g["b_grad"]))
    print(f"[c5 gradient] max |GPU - oracle| F {ef:.2e} B {eb:.2e} (largest entry {scale:.2e})", flush=True)
    assert ef <= 1e-7 * scale and eb <= 1e-7 * scale


def test_gradient_c5_finite_differences(lib, c5):
    """Central differences (step 1e-5) of the GPU's own E2, re-solved at each
    displaced point, on 50 seeded entries (25 of F~, 25 of B~)."""
    Ft, Bt, lam, no = c5["Ft"], c5["Bt"], c5["lam"], c5["prob"].n_occ
    n, na = Ft.shape[0], Bt.shape[0]
    dF, dB = c5["dF"], c5["dB"]
    scale = max(np.abs(dF).max(), np.abs(dB).max())
    h = lib.Handle(0)
    Ftd = torch.from_numpy(Ft).cuda()
    Btd = torch.from_numpy(Bt).cuda()
    lamd = torch.from_numpy(lam).cuda()
    rng = np.random.default_rng(77)
    step = 1e-5

    def e2_at(Fx, Bx):
        h.set_problem_top(Fx, Bx, lamd, no, n - no, na)
        h.rotate_top(False)
        h.build_rhs()
        return h.solve(tol=1e-12, max_iter=1000, basis=lib.ESMP2_BASIS_SEMICANONICAL, allow=())["e2"]

    worst = 0.0
    for k in range(50):
        if k < 25:
            p, q = sorted(int(v) for v in rng.integers(0, n, 2))
            E = torch.zeros_like(Ftd)
            E[p, q] = E[q, p] = step
            fd = (e2_at(Ftd + E, Btd) - e2_at(Ftd - E, Btd)) / (2 * step) / (1.0 if p == q else 2.0)
            g = dF[p, q]
        else:
            Q = int(rng.integers(0, na))
            p = int(rng.integers(0, 2 * no))
            q = int(rng.integers(0, n))
            E = torch.zeros_like(Btd)
            E[Q, p, q] = E[Q, q, p] = step
            fd = (e2_at(Ftd, Btd + E) - e2_at(Ftd, Btd - E)) / (2 * step) / (1.0 if p == q else 2.0)
            g = dB[Q, p, q]
        worst = max(worst, abs(fd - g))
    print(f"[c5 gradient] max |GPU - finite difference| {worst:.2e} (largest entry {scale:.2e})", flush=True)
    assert worst <= 1e-7 * scale
    h.close()


def _euler(Ft, Bt, dF, dB):
    return float(np.sum(Ft * dF) + 0.5 * np.sum(Bt * dB))


def test_gradient_c5_euler(c5):
    assert abs(_euler(c5["Ft"], c5["Bt"], c5["dF"], c5["dB"]) - c5["r"]["e2"]) <= 1e-11 * abs(c5["r"]["e2"])


def test_gradient_c3_euler(lib):
    """The N_o = 16, N_v = 160, N_aux = 480 workload: Euler's identity over the
    whole gradient, and zeros outside the factor blocks E2 depends on."""
    prob = synth.config_problem("c3")
    print("[case] gradient c3", flush=True)
    lam, Ft, Bt = _top(prob)
    h = lib.Handle(0)
    r, dF, dB = _gpu_grad(lib, h, Ft, Bt, lam, prob.n_occ, tol=1e-11)
    e = _euler(Ft, Bt, dF, dB)
    print(f"[c3 gradient] Euler {e:.12e} vs E2 {r['e2']:.12e}", flush=True)
    assert abs(e - r["e2"]) <= 1e-10 * abs(r["e2"])
    no = prob.n_occ
    assert np.all(dB[:, 2 * no:, 2 * no:] == 0.0)
    assert np.isfinite(dF).all() and np.isfinite(dB).all()
    h.close()


def test_set_problem_top_matches_rotation(lib):
    """Stating the problem in the TOP basis gives the E2 of the full pipeline."""
    prob = synth.config_problem("c5")
    lam, Ft, Bt = _top(prob)
    h = lib.Handle(0).load(prob)
    h.rotate_top()
    ref = h.solve(tol=1e-11, max_iter=500, basis=lib.ESMP2_BASIS_SEMICANONICAL)["e2"]
    h2 = lib.Handle(0)
    r, _, _ = _gpu_grad(lib, h2, Ft, Bt, lam, prob.n_occ, tol=1e-11)
    assert abs(r["e2"] - ref) < 1e-10 and abs(r["e2"] - GOLD["c5"]["e2"]) < 1e-10
    h.close()
    h2.close()


def test_autograd_function(lib, c5):
    Ft = torch.from_numpy(c5["Ft"]).cuda().requires_grad_()
    Bt = torch.from_numpy(c5["Bt"]).cuda().requires_grad_()
    lam = torch.from_numpy(c5["lam"]).cuda()
    e = lib.e2_top(Ft, Bt, lam, tol=1e-12)
    (3.0 * e).backward()
    assert abs(e.item() - c5["r"]["e2"]) < 1e-11
    scale = max(np.abs(c5["dF"]).max(), np.abs(c5["dB"]).max())
    assert np.abs(Ft.grad.cpu().numpy() - 3.0 * c5["dF"]).max() <= 1e-9 * scale
    assert np.abs(Bt.grad.cpu().numpy() - 3.0 * c5["dB"]).max() <= 1e-9 * scale
    # only the Fock matrix asks for a gradient
    Ft2 = torch.from_numpy(c5["Ft"]).cuda().requires_grad_()
    lib.e2_top(Ft2, torch.from_numpy(c5["Bt"]).cuda(), lam, tol=1e-12).backward()
    assert np.abs(Ft2.grad.cpu().numpy() - c5["dF"]).max() <= 1e-9 * scale


def test_gradient_errors(lib):
    prob = synth.make_problem(3, 6, 5, 1)
    lam, Ft, Bt = _top(prob)
    h = lib.Handle(0)
    Fd, Bd = torch.from_numpy(Ft).cuda(), torch.from_numpy(Bt).cuda()
    with pytest.raises(lib.Esmp2Error) as e:          # lam not normalised
        h.set_problem_top(Fd, Bd, torch.from_numpy(2 * lam).cuda(), 3, 6, 5)
    assert e.value.status == lib.ESMP2_INVALID_ARG
    with pytest.raises(lib.Esmp2Error) as e:          # lam[0] not the largest
        h.set_problem_top(Fd, Bd, torch.from_numpy(lam[::-1].copy()).cuda(), 3, 6, 5)
    assert e.value.status == lib.ESMP2_INVALID_ARG
    h.set_problem_top(Fd, Bd, torch.from_numpy(lam).cuda(), 3, 6, 5)
    n_amp = 0
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.Esmp2Error) as e:          # no right-hand side yet
        h.gradient(x, torch.empty_like(Fd), None)
    assert e.value.status == lib.ESMP2_BAD_ORDER
    h.rotate_top(False)
    h.build_rhs()
    n_amp, _ = h.space()
    with pytest.raises(lib.Esmp2Error) as e:          # neither output
        h.gradient(torch.zeros(n_amp, dtype=torch.float64, device="cuda"), None, None)
    assert e.value.status == lib.ESMP2_INVALID_ARG
    h.close()
