"""GPU parity on determinants: the library's solution, mapped to determinant
coefficients by esmp2_export_determinants, equals the explicit (tier-1)
oracle's solution of the first-order equation on doubles + L-triples
(paper Sec. II.B: Psi1 over the M_s = 0 doubles and triples; canonical phase
with the alpha string first, then the beta string).  This is the spin-flip
pin run on the HIP path: every stored amplitude and its flip partner land on
the oracle's determinants with the oracle's phases.
"""
import numpy as np
import pytest

import synth
from oracle import explicit, topbasis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12923_amd as p
    return p


def _decode(key, phi, n):
    """det_key (holes bits 0-29, particles 30-59, 10 bits each) -> the
    oracle's determinant bit string."""
    d = phi
    for s in range(3):
        h = (key >> (10 * s)) & 1023
        p = (key >> (30 + 10 * s)) & 1023
        if h != 1023:
            assert (d >> h) & 1
            d ^= 1 << h
        if p != 1023:
            assert not (d >> p) & 1
            d |= 1 << p
    return d


@pytest.mark.parametrize("no,nv,na,seed,spin", [(2, 2, 3, 0, 0), (2, 4, 6, 1, 0), (3, 5, 8, 2, 0), (3, 6, 7, 3, 0),
                                                (2, 4, 6, 4, 1), (3, 5, 8, 5, 1)])
def test_exported_determinants_equal_the_explicit_solution(lib, no, nv, na, seed, spin):
    print(f"[case] n_occ={no} n_vir={nv} n_aux={na} seed={seed} spin={spin}", flush=True)
    prob = synth.make_problem(no, nv, na, seed)
    lam, R = topbasis.top_rotation(prob.F, prob.C, no)
    Ft, Bt = topbasis.rotate(prob.F, prob.B, R)
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no, sign=-1 if spin else 1)
    ref = ex.solve(dense=True)
    h = lib.Handle(0).load(prob, spin=spin)
    h.rotate_top()
    n, offs = h.space()
    ns2 = offs[2] - offs[1]
    ndet = 2 * n - ns2
    xo = torch.empty(n, dtype=torch.float64, device="cuda")
    res = h.solve(tol=1e-13, max_iter=500, x_out=xo)
    assert res["status"] == 0 and abs(res["e2"] - ref["e2"]) < 1e-10
    coeff = torch.full((ndet,), float("nan"), dtype=torch.float64, device="cuda")
    keys = torch.full((ndet,), -1, dtype=torch.int64, device="cuda")
    h.export_determinants(xo, coeff, keys)
    torch.cuda.synchronize()
    c, k = coeff.cpu().numpy(), keys.cpu().numpy()
    dets = [_decode(int(v), ex.phi, ex.n) for v in k]
    # every determinant of D + L exactly once, nothing else
    assert len(set(dets)) == ndet == len(ex.DL)
    assert set(dets) == set(ex.DL)
    got = np.zeros(len(ex.DL))
    for d, v in zip(dets, c):
        got[ex.index[d]] = v
    err = np.abs(got - ex.x).max()
    print(f"[export] {ndet} determinants, max |c - c_oracle| {err:.3e} of max {np.abs(ex.x).max():.3e}", flush=True)
    assert err <= 1e-12 * max(1.0, np.abs(ex.x).max())
    # too short an output is refused
    with pytest.raises(lib.Esmp2Error):
        h._check(lib.lib.esmp2_export_determinants(h.h, xo.data_ptr(), coeff.data_ptr(), keys.data_ptr(), ndet - 1))
    h.close()
