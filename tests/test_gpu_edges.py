"""Edge cases of the HIP path through the C ABI: the smallest occupied space,
an occupied space beyond one 16 x 16 matrix-core tile (the per-amplitude
occupied-index fallback), the largest virtual space, error paths forced from
the host (NaN input, bad sizes, call order, an intruder that makes the operator
indefinite).  Values are compared with the CPU oracle as in the other tests.
"""
import numpy as np
import pytest

import synth
from oracle import structured, topbasis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12923_amd as p
    return p


def _handle(lib, prob):
    print(f"[case] n_occ={prob.n_occ} n_vir={prob.n_vir} n_aux={prob.n_aux} seed={prob.seed}", flush=True)
    return lib.Handle(0).load(prob)


@pytest.mark.parametrize("no,nv,na,seed", [(2, 2, 4, 1), (2, 9, 6, 2), (17, 18, 8, 3), (3, 192, 6, 4)])
def test_sigma_edges(lib, no, nv, na, seed):
    """sigma elementwise (FP64, TOP basis) at the extremes of the supported sizes."""
    prob = synth.make_canonical_problem(no, nv, na, seed)
    h = _handle(lib, prob)
    h.rotate_top()
    lam, R = topbasis.top_rotation(prob.F, prob.C, no)
    Ft, _ = topbasis.rotate(prob.F, prob.B, R)
    op = structured.Structured(Ft, lam, no)
    n, offs = h.space()
    assert n == op.dim
    x = synth.random_amplitudes(n, seed + 300)
    ref = op.sigma(x)
    xt = torch.from_numpy(x).cuda()
    yt = torch.full_like(xt, float("nan"))
    h.sigma(xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    h.close()


@pytest.mark.parametrize("no,nv,na,seed", [(2, 2, 4, 5), (17, 18, 8, 6)])
def test_e2_edges_both_bases(lib, no, nv, na, seed):
    prob = synth.make_problem(no, nv, na, seed)
    h = _handle(lib, prob)
    h.rotate_top()
    ref = structured.solve_problem(prob, tol=1e-13)
    for basis in (lib.ESMP2_BASIS_TOP, lib.ESMP2_BASIS_SEMICANONICAL):
        r = h.solve(tol=1e-12, max_iter=300, basis=basis)
        assert r["status"] == 0
        assert abs(r["e2"] - ref["e2"]) < 1e-10, (basis, r["e2"], ref["e2"])
    h.close()


def test_error_paths(lib):
    prob = synth.make_problem(3, 6, 5, 7)
    h = lib.Handle(0)
    # call order
    with pytest.raises(lib.Esmp2Error) as e:
        h.rotate_top(False)
    assert e.value.status == lib.ESMP2_BAD_ORDER
    F = torch.from_numpy(prob.F).cuda()
    B = torch.from_numpy(prob.B).cuda()
    C = torch.from_numpy(prob.C).cuda()
    # sizes: n_occ > n_vir, n_occ < 2
    for (no, nv) in [(4, 3), (1, 8)]:
        with pytest.raises(lib.Esmp2Error) as e:
            h.set_problem(F, B, C, no, nv, prob.n_aux)
        assert e.value.status == lib.ESMP2_INVALID_ARG
    # NaN in F
    Fb = F.clone()
    Fb[1, 2] = float("nan")
    with pytest.raises(lib.Esmp2Error) as e:
        h.set_problem(Fb, B, C, 3, 6, prob.n_aux)
    assert e.value.status == lib.ESMP2_INVALID_ARG
    # a valid problem afterwards works; sigma before rotate is refused
    h.set_problem(F, B, C, 3, 6, prob.n_aux)
    n, _ = h.space()
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.Esmp2Error) as e:
        h.sigma(x, torch.empty_like(x))
    assert e.value.status == lib.ESMP2_BAD_ORDER
    h.close()


def test_intruder_is_not_spd(lib):
    """The dominant pair moved to the deepest occupied and the highest virtual
    orbital: omega exceeds the smallest double excitation energy, a diagonal
    denominator turns negative and the library reports NOT_SPD (no level
    shift, as in the paper's ESMP2)."""
    prob = synth.make_problem(4, 8, 6, 8, dominant=(0, 7))
    h = _handle(lib, prob)
    h.rotate_top()
    with pytest.raises(lib.Esmp2Error) as e:
        h.build_rhs()
    assert e.value.status == lib.ESMP2_NOT_SPD
    h.close()
