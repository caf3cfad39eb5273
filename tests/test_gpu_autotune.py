"""The Sylvester-variant autotuner and every variant it chooses from.

Each available variant of the virtual-pair Sylvester products gives sigma
elementwise equal to the FP64 oracle (the same bar as the parity tests: sums
of a few hundred unit-scale terms, rounding-order differences ~1e-14); the
autotuner returns the fastest of the variants it timed, its choice is what an
automatic handle then uses, and unavailable variants and bad arguments are
rejected.
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


# padded virtual dimensions 16, 48 (generic kernel only), 80, 112 and 160 (specialised kernel too)
SIZES = [(4, 16, 20, 1), (5, 40, 30, 2), (8, 80, 20, 3), (3, 100, 16, 4), (4, 155, 16, 5)]


@pytest.mark.parametrize("no,nv,na,seed", SIZES)
def test_every_variant_and_the_tuned_choice(lib, no, nv, na, seed):
    print(f"[case] n_occ={no} n_vir={nv} n_aux={na} seed={seed}", flush=True)
    prob = synth.make_canonical_problem(no, nv, na, seed)
    h = lib.Handle(0).load(prob)
    h.rotate_top()
    lam, R = topbasis.top_rotation(prob.F, prob.C, no)
    Ft, _ = topbasis.rotate(prob.F, prob.B, R)
    ref = None
    n, _ = h.space()
    x = synth.random_amplitudes(n, seed + 400)
    ref = structured.Structured(Ft, lam, no).sigma(x)
    xt = torch.from_numpy(x).cuda()
    mv = 16 * ((nv + 15) // 16)
    special = mv in (80, 112, 160)
    best, ms = h.autotune(lib.ESMP2_FP64, reps=3)
    print(f"[autotune] mv={mv} best={best} ms={['%.4f' % t for t in ms]}", flush=True)
    avail = [v for v in range(len(ms)) if ms[v] >= 0]
    assert avail == ([0] if special else []) + [1, 2, 3, 4, 5]
    assert best in avail and ms[best] == min(ms[v] for v in avail)
    tol = 1e-12 * np.abs(ref).max()
    outs = {}
    for v in avail:
        h.set_sylvester_variant(lib.ESMP2_FP64, v)
        y = torch.full_like(xt, float("nan"))
        h.sigma(xt, y)
        torch.cuda.synchronize()
        outs[v] = y.cpu().numpy()
        err = np.abs(outs[v] - ref).max()
        print(f"[variant {v}] max err {err:.3e}", flush=True)
        assert err <= tol, (v, err, tol)
    # automatic again: the recorded choice
    h.set_sylvester_variant(lib.ESMP2_FP64, -1)
    y = torch.full_like(xt, float("nan"))
    h.sigma(xt, y)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), outs[best])
    # a second handle of the same sizes picks up the recorded choice
    h2 = lib.Handle(0).load(prob)
    h2.rotate_top()
    y2 = torch.full_like(xt, float("nan"))
    h2.sigma(xt, y2)
    torch.cuda.synchronize()
    assert np.array_equal(y2.cpu().numpy(), outs[best])
    h2.close()
    if not special:
        with pytest.raises(lib.Esmp2Error) as e:
            h.set_sylvester_variant(lib.ESMP2_FP64, 0)
        assert e.value.status == lib.ESMP2_INVALID_ARG
        with pytest.raises(lib.Esmp2Error) as e:
            h.autotune(lib.ESMP2_BF16)
        assert e.value.status == lib.ESMP2_UNSUPPORTED
    h.close()


@pytest.mark.parametrize("no,nv,na,seed", [(5, 40, 12, 31), (4, 80, 12, 32)])
def test_every_variant_triplet(lib, no, nv, na, seed):
    """Every variant with the M_s = 0 triplet reference (flip partners of opposite sign)."""
    print(f"[case] triplet variants n_occ={no} n_vir={nv} n_aux={na} seed={seed}", flush=True)
    prob = synth.make_problem(no, nv, na, seed)
    lam, R = topbasis.top_rotation(prob.F, prob.C, no)
    Ft, Bt = topbasis.rotate(prob.F, prob.B, R)
    lam, Ft, Bt = (np.ascontiguousarray(a) for a in (lam, Ft, Bt))
    h = lib.Handle(0)
    dev = [torch.from_numpy(a).cuda() for a in (Ft, Bt, lam)]
    h.set_problem_top(dev[0], dev[1], dev[2], no, nv, na, spin=1)
    h.rotate_top(False)
    n, _ = h.space()
    x = synth.random_amplitudes(n, seed + 700)
    ref = structured.Structured(Ft, lam, no, spin=1).sigma(x)
    xt = torch.from_numpy(x).cuda()
    mv = 16 * ((nv + 15) // 16)
    for v in ([0] if mv in (80, 112, 160) else []) + [1, 2, 3, 4, 5]:
        h.set_sylvester_variant(lib.ESMP2_FP64, v)
        y = torch.full_like(xt, float("nan"))
        h.sigma(xt, y)
        torch.cuda.synchronize()
        err = np.abs(y.cpu().numpy() - ref).max()
        print(f"[triplet variant {v}] max err {err:.3e}", flush=True)
        assert err <= 1e-12 * np.abs(ref).max()
    h.close()


def test_autotune_fp32_and_bad_arguments(lib):
    prob = synth.config_problem("c5")
    print(f"[case] n_occ={prob.n_occ} n_vir={prob.n_vir} n_aux={prob.n_aux}", flush=True)
    h = lib.Handle(0).load(prob)
    with pytest.raises(lib.Esmp2Error) as e:
        h.autotune(lib.ESMP2_FP64)                 # before the rotation
    assert e.value.status == lib.ESMP2_BAD_ORDER
    h.rotate_top()
    best, ms = h.autotune(lib.ESMP2_FP32, reps=2)
    assert best in range(6) and ms[best] >= 0
    best_b, ms_b = h.autotune(lib.ESMP2_BF16, reps=2)
    assert best_b == 0 and all(t < 0 for t in ms_b[1:])
    for bad in (0, 1001):
        with pytest.raises(lib.Esmp2Error) as e:
            h.autotune(lib.ESMP2_FP64, reps=bad)
        assert e.value.status == lib.ESMP2_INVALID_ARG
    with pytest.raises(lib.Esmp2Error) as e:
        h.set_sylvester_variant(lib.ESMP2_FP64, 6)
    assert e.value.status == lib.ESMP2_INVALID_ARG
    with pytest.raises(lib.Esmp2Error) as e:
        h.set_sylvester_variant(lib.ESMP2_BF16, 2)
    assert e.value.status == lib.ESMP2_INVALID_ARG
    h.close()
