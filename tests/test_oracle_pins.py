"""Pins of the CPU oracle against things other than itself (no GPU).

Each test names the property of the paper's method (or of the mathematics)
that fixes the expected value.
"""
import numpy as np
import pytest

import synth
from oracle import explicit, frontend, gradient, layout, opcount, structured, topbasis

MICRO = [(2, 4, 6, 0), (3, 5, 8, 1), (3, 6, 8, 2), (4, 6, 10, 3), (4, 7, 9, 4)]


def _rotated(no, nv, na, seed, **kw):
    p = synth.make_problem(no, nv, na, seed, **kw)
    lam, R = topbasis.top_rotation(p.F, p.C, no)
    Ft, Bt = topbasis.rotate(p.F, p.B, R)
    return p, lam, Ft, Bt


def _phi(rm, index, x):
    v = np.zeros(len(index))
    for k, (box, contrib, own) in enumerate(rm):
        for d, s in contrib:
            v[index[d]] += s * x[k]
    return v


@pytest.mark.parametrize("no,nv,na,seed", MICRO)
def test_structured_equals_explicit(no, nv, na, seed):
    """P-a: the N^5 seven-box operator, right-hand side, diagonal and E2 equal
    the explicit determinant construction (Slater determinants, second
    quantisation) on every box, at sizes that hit every index coincidence."""
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no)
    r1 = ex.solve()
    rm = layout.rep_map(no, nv)
    assert len(rm) == sum(layout.box_sizes(no, nv))
    st = structured.Structured(Ft, lam, no)
    x = np.random.default_rng(seed + 10).standard_normal(st.dim)
    y = ex.A @ _phi(rm, ex.index, x)
    sig_ex = np.array([own[1] * y[ex.index[own[0]]] for (_, _, own) in rm])
    np.testing.assert_allclose(st.sigma(x), sig_ex, rtol=0, atol=1e-13)
    hp = ex.h_psi0()
    b_ex = np.array([own[1] * hp.get(own[0], 0.0) for (_, _, own) in rm])
    rh = structured.RHS(Ft, Bt, lam, no)
    np.testing.assert_allclose(rh.rhs(), b_ex, rtol=0, atol=1e-15)
    D_ex = np.array([ex.diag_fock(own[0]) - ex.E0 for (_, _, own) in rm])
    np.testing.assert_allclose(st.diagonal(), D_ex, rtol=0, atol=1e-13)
    assert abs(st.E0 - ex.E0) < 1e-13
    r2 = structured.solve(Ft, Bt, lam, no, tol=1e-13)
    assert abs(r2["e2"] - r1["e2"]) < 1e-14
    assert abs(r2["e2_s"] - r1["e2_s"]) < 1e-15
    assert r1["max_bN"] == 0.0          # N-triples have no right-hand side (Sec. II.B)


@pytest.mark.parametrize("no,nv,na,seed", MICRO)
def test_structured_equals_explicit_triplet(no, nv, na, seed):
    """P-a for the M_s = 0 triplet reference (beta singles with the opposite
    sign): the seven-box operator, right-hand side and E2 with the spin-flip
    partners carrying opposite amplitudes equal the determinant construction."""
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no, sign=-1)
    r1 = ex.solve()
    rm = layout.rep_map(no, nv, spin=1)
    st = structured.Structured(Ft, lam, no, spin=1)
    x = np.random.default_rng(seed + 10).standard_normal(st.dim)
    y = ex.A @ _phi(rm, ex.index, x)
    sig_ex = np.array([own[1] * y[ex.index[own[0]]] for (_, _, own) in rm])
    np.testing.assert_allclose(st.sigma(x), sig_ex, rtol=0, atol=1e-13)
    hp = ex.h_psi0()
    b_ex = np.array([own[1] * hp.get(own[0], 0.0) for (_, _, own) in rm])
    np.testing.assert_allclose(structured.RHS(Ft, Bt, lam, no, spin=1).rhs(), b_ex, rtol=0, atol=1e-15)
    r2 = structured.solve(Ft, Bt, lam, no, tol=1e-13, spin=1)
    assert abs(r2["e2"] - r1["e2"]) < 1e-14
    assert abs(r2["e2_s"] - r1["e2_s"]) < 1e-15
    r0 = structured.solve(Ft, Bt, lam, no, tol=1e-13)
    assert abs(r2["e2"] - r0["e2"]) > 1e-6 * abs(r0["e2"])      # the two references differ


@pytest.mark.parametrize("no,nv,na,seed", MICRO[1:4])
def test_triplet_spin_purity(no, nv, na, seed):
    """The triplet reference and its first-order wave function are pure
    triplets: ||S+ Psi||^2 = S(S+1) ||Psi||^2 = 2 ||Psi||^2 for M_s = 0; the
    layout with antisymmetric flip partners reproduces the determinant
    solution."""
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no, sign=-1)
    ex.solve()
    for psi in (ex.psi0, None):
        if psi is None:
            psi = {d: c for d, c in zip(ex.DL, ex.x)}
            for d, b, D in zip(ex.S, ex.bS, ex.DS):
                psi[d] = -b / D
        sp = ex.s_plus(psi)
        n2 = sum(v * v for v in psi.values())
        assert abs(sum(v * v for v in sp.values()) - 2.0 * n2) < 1e-12 * n2
    x = structured.solve(Ft, Bt, lam, no, tol=1e-14, spin=1)["x"]
    v = _phi(layout.rep_map(no, nv, spin=1), ex.index, x)
    np.testing.assert_allclose(v, ex.x, atol=1e-13)


def test_structured_equals_explicit_config1():
    """P-a at the smallest workload (n_occ=4, n_vir=16, n_aux=48, seed 0)."""
    p = synth.config_problem("c1")
    ex = explicit.from_problem(p)
    r1 = ex.solve()
    r2 = structured.solve_problem(p, tol=1e-12)
    assert abs(r1["e2"] - r2["e2"]) < 1e-12
    assert r1["max_bN"] == 0.0


@pytest.mark.parametrize("no,nv,na,seed", MICRO[1:4])
def test_one_body_density_and_e0(no, nv, na, seed):
    """P-b: the spin-summed one-body density of Psi0 in the TOP basis is
    diag(2 - lambda^2 on occupied l, lambda^2 on its partner, 0 on AVOs) and
    E0 = <Psi0|F|Psi0> = tr(F gamma)."""
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no)
    n = no + nv
    from oracle import fermion as fm
    gam = np.zeros((n, n))
    for pp in range(n):
        for q in range(n):
            e = np.zeros((n, n))
            e[pp, q] = 1.0
            v = fm.apply_one_body(ex.psi0, e, n)
            gam[pp, q] = sum(c * v.get(d, 0.0) for d, c in ex.psi0.items())
    np.testing.assert_allclose(gam, ex.gamma, atol=1e-14)
    assert abs(ex.E0 - np.sum(Ft * gam)) < 1e-13
    assert abs(np.trace(gam) - 2 * no) < 1e-13


def test_weighted_symmetry_and_definiteness():
    """P-g: A is symmetric in the weighted inner product, positive definite
    (Jacobi-scaled), E2 < 0 and the Hylleraas energy decreases monotonically
    along the conjugate-gradient iterations towards E2 from above."""
    p = synth.config_problem("c1")
    lam, R = topbasis.top_rotation(p.F, p.C, p.n_occ)
    Ft, Bt = topbasis.rotate(p.F, p.B, R)
    st = structured.Structured(Ft, lam, p.n_occ)
    rng = np.random.default_rng(7)
    for _ in range(3):
        x, y = rng.standard_normal((2, st.dim))
        # flip-symmetric S2 parts (the vectors the layout represents)
        assert abs(st.dot(y, st.sigma(x)) - st.dot(st.sigma(y), x)) < 1e-11 * st.dim
    Dg = st.diagonal()
    assert Dg.min() > 0
    rh = structured.RHS(Ft, Bt, lam, p.n_occ)
    b = rh.rhs()
    hist = []
    x, r, it, rel = structured.pcg(st, b, tol=1e-12, history=hist)
    e_exact = st.dot(b, x) - st.dot(x, r)
    assert e_exact < 0
    eh = [h[1] for h in hist]
    assert all(eh[k + 1] <= eh[k] + 1e-15 for k in range(len(eh) - 1))
    assert all(e >= e_exact - 1e-14 for e in eh)


def test_counts_closed_form():
    """P-k: the number of determinants per class from brute-force enumeration
    equals the closed forms of the seven boxes (each non-S2 box = 2 dets)."""
    for (no, nv, na, seed) in MICRO + [(5, 8, 4, 5)]:
        p = synth.make_problem(no, nv, max(na, 2), seed)
        lam = np.sort(np.abs(np.random.default_rng(seed).standard_normal(no)))[::-1]
        f = np.diag(np.arange(no + nv, dtype=float))
        ex = explicit.ExplicitESMP2(f, np.zeros((no + nv,) * 4), lam, no)
        s = layout.box_sizes(no, nv)
        assert len(ex.D) == 2 * s[0] + s[1]
        assert len(ex.L) == 2 * sum(s[2:])
        c2 = lambda m: m * (m - 1) // 2
        c3 = lambda m: m * (m - 1) * (m - 2) // 6
        n_trip = 2 * c3(no) * c3(nv) + 2 * c2(no) * no * c2(nv) * nv
        assert len(ex.L) + len(ex.S) + len(ex.N) == n_trip


@pytest.mark.parametrize("no,nv,na,seed", MICRO[1:4])
def test_spin_purity(no, nv, na, seed):
    """P-h: with the spatial TOP-membership rule the first-order wave function
    (D + L solution plus the directly inverted S part) is a pure singlet,
    S+ Psi1 = 0; the same-spin rule breaks it (so the test discriminates)."""
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    eri = topbasis.eri_from_factor(Bt)
    for rule, pure in (("spatial", True), ("same-spin", False)):
        ex = explicit.ExplicitESMP2(Ft, eri, lam, no, rule=rule)
        ex.solve()
        psi1 = {d: c for d, c in zip(ex.DL, ex.x)}
        for d, b, D in zip(ex.S, ex.bS, ex.DS):
            psi1[d] = -b / D
        sp = ex.s_plus(psi1)
        norm = np.sqrt(sum(v * v for v in sp.values()))
        scale = np.sqrt(sum(v * v for v in psi1.values()))
        if pure:
            assert norm < 1e-13 * scale
        else:
            assert norm > 1e-6 * scale


@pytest.mark.parametrize("no,nv,na,seed", MICRO[1:4])
def test_layout_reproduces_determinant_solution(no, nv, na, seed):
    """P-i: the determinant solution has equal amplitudes on spin-flip partners,
    so the seven-box solution mapped to determinants reproduces it exactly."""
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no)
    ex.solve()
    x = structured.solve(Ft, Bt, lam, no, tol=1e-14)["x"]
    rm = layout.rep_map(no, nv)
    # S2 entries are single determinants with the flip-symmetrised vector
    v = _phi(rm, ex.index, x)
    np.testing.assert_allclose(v, ex.x, atol=1e-13)


def test_solvers_agree():
    """P-j: dense LU, SciPy's conjugate gradient and the oracle's Jacobi PCG
    in the seven-box layout give the same E2."""
    no, nv, na, seed = 3, 6, 8, 2
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no)
    r_lu = ex.solve(dense=True)
    r_cg = ex.solve(dense=False)
    r_pcg = structured.solve(Ft, Bt, lam, no, tol=1e-13)
    assert abs(r_lu["e2"] - r_cg["e2"]) < 1e-15
    assert abs(r_lu["e2"] - r_pcg["e2"]) < 1e-15


def _rand_orth(n, rng):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("name", ["micro", "c1"])
def test_rotation_invariance(name):
    """P-f: the reference is the same wave function in any orbital basis
    (Sec. II.A), so random occupied-occupied and virtual-virtual rotations of
    (F, B, C) leave E0 and E2 unchanged."""
    p = synth.make_problem(4, 7, 9, 4) if name == "micro" else synth.config_problem("c1")
    no, nv = p.n_occ, p.n_vir
    rng = np.random.default_rng(11)
    Uo, Uv = _rand_orth(no, rng), _rand_orth(nv, rng)
    R = np.zeros((no + nv,) * 2)
    R[:no, :no], R[no:, no:] = Uo, Uv
    F2 = R.T @ p.F @ R
    B2 = np.einsum("pk,Qpq,ql->Qkl", R, p.B, R)
    C2 = Uo.T @ p.C @ Uv
    p2 = synth.Problem(no, nv, p.n_aux, F2, B2, C2)
    r1 = structured.solve_problem(p, tol=1e-12)
    r2 = structured.solve_problem(p2, tol=1e-12)
    assert abs(r1["e2"] - r2["e2"]) < 1e-12 * abs(r1["e2"])
    assert abs(r1["e0"] - r2["e0"]) < 1e-12 * abs(r1["e0"])


@pytest.mark.parametrize("name", ["micro", "c1"])
def test_rotations_fixing_the_pinned_pair(name):
    """Doubles + L-triples are mapped onto themselves by any rotation of the
    occupied orbitals other than t and of the virtuals other than t' (an
    L-triple keeps t among its holes and t' among its particles), so the
    operator is covariant, sigma(T x) = T sigma(x) with the Fock matrix
    rotated, the right-hand side transforms like an amplitude vector, and
    E2_DL = -b^T A^-1 b is unchanged.  Such a rotation that diagonalises the
    non-pinned Fock blocks makes the operator nearly diagonal."""
    p = synth.make_problem(4, 7, 9, 4) if name == "micro" else synth.config_problem("c1")
    no, nv = p.n_occ, p.n_vir
    lam, R = topbasis.top_rotation(p.F, p.C, no)
    Ft, Bt = topbasis.rotate(p.F, p.B, R)
    rh = structured.RHS(Ft, Bt, lam, no)
    op, b = rh.op, rh.rhs()
    rng = np.random.default_rng(5)
    for kind in ("random", "semicanonical"):
        To, Tv = np.eye(no), np.eye(nv)
        if kind == "random":
            To[1:, 1:], Tv[1:, 1:] = _rand_orth(no - 1, rng), _rand_orth(nv - 1, rng)
        else:
            To[1:, 1:] = np.linalg.eigh(Ft[1:no, 1:no])[1]
            Tv[1:, 1:] = np.linalg.eigh(Ft[no + 1:, no + 1:])[1]
        T = np.zeros_like(Ft)
        T[:no, :no], T[no:, no:] = To, Tv
        op2 = structured.Structured(T.T @ Ft @ T, lam, no, omega=op.omega)
        assert abs(op2.E0 - op.E0) < 1e-12 and abs(op2.kappa - op.kappa) < 1e-12
        x = synth.random_amplitudes(op.dim, 3)
        tx = structured.transform_amplitudes(x, no, nv, To, Tv)
        np.testing.assert_allclose(op2.sigma(tx), structured.transform_amplitudes(op.sigma(x), no, nv, To, Tv),
                                   rtol=0, atol=1e-12 * np.abs(op.sigma(x)).max())
        assert abs(op2.dot(tx, tx) - op.dot(x, x)) < 1e-12 * op.dot(x, x)
        b2 = structured.transform_amplitudes(b, no, nv, To, Tv)
        x1, _, it1, _ = structured.pcg(op, b, tol=1e-12)
        x2, _, it2, _ = structured.pcg(op2, b2, tol=1e-12)
        assert abs(op.dot(b, x1) - op2.dot(b2, x2)) < 1e-12 * abs(op.dot(b, x1))
        if kind == "semicanonical":
            assert it2 < it1


@pytest.mark.parametrize("no,nv,na,seed", [(2, 4, 6, 0), (3, 5, 8, 1)])
def test_original_h0_shift(no, nv, na, seed):
    """The original zeroth-order Hamiltonian (full Fock operator on all
    triples) differs from the modified one only through the S/N blocks: the
    shift of E2 is small against E2, vanishes when the Fock matrix is
    diagonal in the TOP basis (then F^(diag) = F on every block), and the
    original operator is symmetric positive definite on D + T."""
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    eri = topbasis.eri_from_factor(Bt)
    ex = explicit.ExplicitESMP2(Ft, eri, lam, no)
    mod = ex.solve()
    org = ex.solve_original()
    assert org["dim"] == len(ex.D) + len(ex.L) + len(ex.S) + len(ex.N)
    assert org["e2"] < 0
    shift = org["e2"] - mod["e2"]
    assert 0 < abs(shift) < 0.05 * abs(mod["e2"])
    # diagonal Fock matrix: both theories give the same E2
    Fd = np.diag(np.diag(Ft))
    exd = explicit.ExplicitESMP2(Fd, eri, lam, no)
    assert abs(exd.solve_original()["e2"] - exd.solve()["e2"]) < 1e-14 * abs(exd.solve()["e2"])


def test_rank_one_reference_has_no_s_rhs():
    """For a single-CSF reference (rank-1 C) only TOP t has a non-zero
    coefficient, so the S-triples have no right-hand side and E2_S = 0.
    Treating every TOP as large does change E2 (the added L-triples still
    couple through the full Fock operator), which this also checks, so the
    class logic is exercised."""
    no, nv, na, seed = 3, 5, 8, 1
    p = synth.make_problem(no, nv, na, seed)
    rng = np.random.default_rng(3)
    u, v = 0.2 * rng.standard_normal(no), 0.2 * rng.standard_normal(nv)
    u[-1] += 1.0          # HOMO-like hole, LUMO-like particle (no intruders)
    v[0] += 1.0
    C = np.outer(u, v)
    C /= np.linalg.norm(C)
    lam, R = topbasis.top_rotation(p.F, C, no)
    Ft, Bt = topbasis.rotate(p.F, p.B, R)
    eri = topbasis.eri_from_factor(Bt)
    ex1 = explicit.ExplicitESMP2(Ft, eri, lam, no, n_top=1)
    e1 = ex1.solve()
    ea = explicit.ExplicitESMP2(Ft, eri, lam, no, n_top=no).solve()
    assert np.max(np.abs(ex1.bS)) < 1e-15 and abs(e1["e2_s"]) < 1e-28
    assert abs(ea["e2_s"]) == 0.0
    assert abs(e1["e2"] - ea["e2"]) > 1e-9
    r2 = structured.solve(Ft, Bt, lam, no, tol=1e-13)
    assert abs(r2["e2"] - e1["e2"]) < 1e-15


def _fragments(noA, nvA, naA, noB, nvB, naB, seed):
    """Two non-interacting fragments; C rank-1 on A; F_A without ov block;
    F_B diagonal.  Orbital order: occ A, occ B, vir A, vir B."""
    rng = np.random.default_rng(seed)
    eoA = np.sort(rng.uniform(-1.5, -0.3, noA)); evA = np.sort(rng.uniform(0.1, 3.0, nvA))
    eoB = np.sort(rng.uniform(-1.5, -0.3, noB)); evB = np.sort(rng.uniform(0.1, 3.0, nvB))
    def fock_A():
        F = np.diag(np.concatenate([eoA, evA]))
        E = rng.normal(0, 1e-2, F.shape)
        E = np.triu(E, 1) + np.triu(E, 1).T
        E[:noA, noA:] = 0
        E[noA:, :noA] = 0
        return F + E
    FA = fock_A()
    GA = rng.standard_normal((naA, noA + nvA, noA + nvA))
    BA = 0.05 * (GA + GA.transpose(0, 2, 1)) / 2
    GB = rng.standard_normal((naB, noB + nvB, noB + nvB))
    BB = 0.05 * (GB + GB.transpose(0, 2, 1)) / 2
    u, v = 0.2 * rng.standard_normal(noA), 0.2 * rng.standard_normal(nvA)
    u[-1] += 1.0          # HOMO-like hole, LUMO-like particle (no intruders)
    v[0] += 1.0
    CA = np.outer(u, v)
    CA /= np.linalg.norm(CA)
    no, nv = noA + noB, nvA + nvB
    n = no + nv
    ia = list(range(noA)) + list(range(no, no + nvA))
    ib = list(range(noA, no)) + list(range(no + nvA, n))
    F = np.zeros((n, n))
    F[np.ix_(ia, ia)] = FA
    F[np.ix_(ib, ib)] = np.diag(np.concatenate([eoB, evB]))
    B = np.zeros((naA + naB, n, n))
    B[np.ix_(range(naA), ia, ia)] = BA
    B[np.ix_(range(naA, naA + naB), ib, ib)] = BB
    C = np.zeros((no, nv))
    C[:noA, :nvA] = CA
    A = synth.Problem(noA, nvA, naA, FA, BA, CA)
    AB = synth.Problem(no, nv, naA + naB, F, B, C)
    # textbook closed-shell MP2 of fragment B
    iajb = np.einsum("Qia,Qjb->iajb", BB[:, :noB, noB:], BB[:, :noB, noB:])
    den = evB[None, :, None, None] + evB[None, None, None, :] - eoB[:, None, None, None] - eoB[None, None, :, None]
    emp2 = -np.sum(iajb * (2 * iajb - iajb.transpose(0, 3, 2, 1)) / den)
    return A, AB, emp2


@pytest.mark.parametrize("sizes", [(2, 3, 5, 2, 3, 5, 0), (3, 4, 6, 2, 4, 6, 1), (3, 8, 9, 4, 10, 12, 2)])
def test_size_intensivity_reduces_to_mp2(sizes):
    """P-d: a non-interacting closed-shell fragment B added to an excited
    fragment A shifts E2 by exactly the closed-shell MP2 energy of B
    -sum (ia|jb)[2(ia|jb)-(ib|ja)]/(e_a+e_b-e_i-e_j): the paper's size
    intensivity (water + distant helium atoms) in closed form."""
    A, AB, emp2 = _fragments(*sizes)
    eA = structured.solve_problem(A, tol=1e-13)["e2"]
    eAB = structured.solve_problem(AB, tol=1e-13)["e2"]
    assert abs((eAB - eA) - emp2) < 1e-13
    assert emp2 < 0
    if sizes[0] + sizes[3] <= 4 and sizes[1] + sizes[4] <= 7:
        ex = explicit.from_problem(AB)
        assert abs(ex.solve()["e2"] - eAB) < 1e-14


def test_diagonal_fock_limit_closed_form():
    """P-c: with a diagonal Fock matrix and a permutation-like C (one entry per
    row, distinct columns) the operator is diagonal: E2 is the closed form
    -sum over D, L, S determinants of b^2/D, and PCG converges in one step."""
    no, nv, na = 3, 6, 8
    p = synth.make_problem(no, nv, na, 9, fock_noise=0.0)
    C = np.zeros((no, nv))
    w = np.array([0.9, 0.4, 0.17])
    w /= np.linalg.norm(w)
    C[0, 2], C[1, 0], C[2, 4] = w
    p = synth.Problem(no, nv, na, p.F, p.B, C)
    lam, R = topbasis.top_rotation(p.F, p.C, no)
    Ft, Bt = topbasis.rotate(p.F, p.B, R)
    assert np.count_nonzero(np.abs(Ft - np.diag(np.diag(Ft))) > 1e-14) == 0
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no)
    hp = ex.h_psi0()
    closed = -sum(hp.get(d, 0.0) ** 2 / (ex.diag_fock(d) - ex.E0) for d in ex.D + ex.L + ex.S)
    r = structured.solve(Ft, Bt, lam, no, tol=1e-13)
    assert abs(r["e2"] - closed) < 1e-15
    assert r["iters"] == 1


@pytest.mark.parametrize("no,nv,seed", [(2, 3, 0), (3, 4, 1), (2, 5, 2)])
def test_reference_density_and_fock(no, nv, seed):
    """The closed-form one-body density of Psi0 equals the determinant
    expansion's (Slater-Condon), its trace is the electron count 2 n_occ, and
    the Fock operator built from it inverts the definition of the one-electron
    operator h = F - G[gamma] (both directions)."""
    p = synth.make_problem(no, nv, 7, seed)
    g = frontend.density(p.C, no)
    np.testing.assert_allclose(frontend.density_explicit(p.C, no), g, rtol=0, atol=1e-14)
    assert abs(np.trace(g) - 2 * no) < 1e-13
    h = p.F - frontend.g_matrix(g, p.B)
    np.testing.assert_allclose(frontend.fock_from_core(h, p.B, p.C, no), p.F, rtol=0, atol=1e-13)
    # G[gamma] against the four-index integrals written out
    eri = topbasis.eri_from_factor(p.B)
    Gx = np.einsum("rs,pqrs->pq", g, eri) - 0.5 * np.einsum("rs,psrq->pq", g, eri)
    np.testing.assert_allclose(frontend.g_matrix(g, p.B), Gx, rtol=0, atol=1e-13)
    # in the TOP basis the density is diagonal (2 - lam^2 on occupied l, lam^2 on l')
    lam, R = topbasis.top_rotation(p.F, p.C, no)
    gt = R.T @ g @ R
    d = np.zeros(no + nv)
    d[:no] = 2 - lam ** 2
    d[no:2 * no] = lam ** 2
    np.testing.assert_allclose(gt, np.diag(d), rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# derivatives of E2 (TOP-basis Fock matrix and factor, rotation held fixed)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("no,nv,na,seed,spin", [(3, 6, 5, 1, 0), (2, 5, 4, 3, 0), (3, 6, 5, 2, 1)])
def test_gradient_equals_full_resolve_differences(no, nv, na, seed, spin):
    """The derivative of the functional at fixed amplitudes (the adjoint of
    the symmetric first-order equation is its own solution) equals the
    central difference of E2 itself, re-solved at each displaced point, on
    entries of every Fock block and of every factor block."""
    _, lam, Ft, Bt = _rotated(no, nv, na, seed)
    L = gradient.Lagrangian(Ft, Bt, lam, no, spin=spin)
    assert abs(L.value() - L.e2) < 1e-15                       # the functional's value is E2
    n = no + nv
    h = 1e-5
    f_entries = [(0, 0), (1, 1), (0, no), (no, no), (1, no + 2), (no + 1, n - 1), (0, 1), (no + 2, no + 2)]
    for p, q in f_entries:
        E = np.zeros_like(Ft)
        E[p, q] = E[q, p] = h
        fd = (gradient.e2_of(Ft + E, Bt, lam, no, spin=spin) - gradient.e2_of(Ft - E, Bt, lam, no, spin=spin)) / (2 * h)
        fd /= 1.0 if p == q else 2.0
        g = L.grad_F(p, q)
        assert abs(g - fd) <= 1e-7 * max(abs(fd), 1e-4), (p, q, g, fd)
    b_entries = [(0, 0, no), (1, 1, no + 1), (na - 1, 0, 0), (2, no, n - 1), (0, 1, 1), (1, 0, 1), (2, no, no + 1)]
    for Q, p, q in b_entries:
        E = np.zeros_like(Bt)
        E[Q, p, q] = E[Q, q, p] = h
        fd = (gradient.e2_of(Ft, Bt + E, lam, no, spin=spin) - gradient.e2_of(Ft, Bt - E, lam, no, spin=spin)) / (2 * h)
        fd /= 1.0 if p == q else 2.0
        g = L.grad_B(Q, p, q)
        assert abs(g - fd) <= 1e-7 * max(abs(fd), 1e-4), (Q, p, q, g, fd)


def test_gradient_differences_are_exact():
    """At fixed amplitudes the functional is linear in F~ and of degree two in
    each factor entry: its second (F) and third (B) differences vanish, so
    central differences give the exact derivative for any step."""
    no = 3
    _, lam, Ft, Bt = _rotated(no, 6, 5, 4)
    L = gradient.Lagrangian(Ft, Bt, lam, no)
    E = np.zeros_like(Ft)
    E[1, 5] = E[5, 1] = 0.05
    assert abs(L.value(Ft=Ft + E) - 2 * L.value() + L.value(Ft=Ft - E)) < 1e-15
    E = np.zeros_like(Bt)
    E[2, 1, 5] = E[2, 5, 1] = 0.05
    vals = [L.value(Bt=Bt + k * E) for k in (-1, 0, 1, 2)]
    assert abs(vals[3] - 3 * vals[2] + 3 * vals[1] - vals[0]) < 1e-15
    assert abs(L.grad_B(2, 1, 5, h=1e-1) - L.grad_B(2, 1, 5, h=1e-4)) < 1e-12


def test_gradient_homogeneity():
    """H scales by s when F~ -> s F~ and B~ -> sqrt(s) B~, and E2 with it
    (b, A, D_S and b_S all scale by s), so Euler's theorem fixes
    <F~, dE2/dF~> + <B~, dE2/dB~> / 2 = E2 over the whole gradient."""
    no = 3
    _, lam, Ft, Bt = _rotated(no, 5, 4, 6)
    L = gradient.Lagrangian(Ft, Bt, lam, no)
    GF, GB = L.full_gradient()
    assert np.allclose(GF, GF.T, rtol=0, atol=0) and np.allclose(GB, GB.transpose(0, 2, 1), rtol=0, atol=0)
    euler = np.sum(Ft * GF) + 0.5 * np.sum(Bt * GB)
    assert abs(euler - L.e2) < 1e-13 * max(1.0, abs(L.e2)) + 1e-15
    # and directly: E2(s F~, sqrt(s) B~) = s E2
    s = 1.7
    assert abs(gradient.e2_of(s * Ft, np.sqrt(s) * Bt, lam, no) - s * L.e2) < 1e-14


def _costs():
    """The product's size arithmetic (a plain module, loaded by path so that the
    library itself need not be built for this CPU test)."""
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2003_12923_amd",
                        "costs.py")
    spec = importlib.util.spec_from_file_location("_esmp2_costs", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("no,nv", [(2, 2), (2, 3), (3, 3), (3, 4), (3, 5), (4, 5), (4, 6), (5, 6), (5, 8)])
def test_flop_count_equals_enumerated_nonzeros(no, nv):
    """P-l: the closed-form algorithmic work of sigma (2 x nnz of H0 - E0 on
    D + L in the representative basis, by class) equals the nonzeros of the
    explicit determinant operator with a generic Fock matrix, mapped to the
    representative rows, class by class."""
    e = opcount.rep_nnz(no, nv)
    c = _costs().sigma_nnz(no, nv)
    for k in ("diag", "vir", "occ", "ov", "total"):
        assert e[k] == c[k], (k, e[k], c[k])
    assert e["dim"] == c["diag"]
    # every stored amplitude is a row, except the redundant half of S2
    assert c["diag"] == _costs().amplitudes(no, nv) - (no * no * nv * nv - no * nv) // 2


def test_flop_count_scaling_exponents():
    """P-l: log-log regressions of the counted work over the paper's ranges
    (Sec. III.B: N_v = 100 with N_o = 30..50, N_o = 30 with N_v = 50..100)
    give the categories of Table I's H0 rows: virtual-index contractions
    N_o^2 N_v^3, occupied-index ones N_o^3 N_v^2, doubles <-> triples
    N_o^2 N_v^2; nothing in sigma grows faster than N_o^2 N_v^3 (fifth order)."""
    costs = _costs()
    O, V = np.arange(30, 51), np.arange(50, 101)
    expect = {"vir": (2, 3), "occ": (3, 2), "ov": (2, 2), "diag": (2, 2)}
    for cls, (eo, ev) in expect.items():
        so = np.polyfit(np.log(O), np.log([costs.sigma_nnz(int(o), 100)[cls] for o in O]), 1)[0]
        sv = np.polyfit(np.log(V), np.log([costs.sigma_nnz(30, int(v))[cls] for v in V]), 1)[0]
        assert abs(so - eo) < 0.1 and abs(sv - ev) < 0.1, (cls, so, sv)
    so = np.polyfit(np.log(O), np.log([costs.sigma_nnz(int(o), 100)["total"] for o in O]), 1)[0]
    sv = np.polyfit(np.log(V), np.log([costs.sigma_nnz(30, int(v))["total"] for v in V]), 1)[0]
    assert so + sv < 5.05


def _topk_case(no, nv, na, seed, k, spin):
    from oracle import topk
    p, lam, Ft, Bt = _rotated(no, nv, na, seed)
    ex = explicit.ExplicitESMP2(Ft, topbasis.eri_from_factor(Bt), lam, no, n_top=k, sign=-1 if spin else 1)
    r1 = ex.solve(dense=True)
    tk = topk.TopK(Ft, Bt, lam, no, k, spin=spin)
    return ex, r1, tk


@pytest.mark.parametrize("no,nv,na,seed,k,spin", [(2, 3, 4, 0, 2, 0), (3, 4, 6, 1, 2, 0), (3, 5, 6, 2, 3, 0),
                                                  (3, 5, 7, 3, 2, 1), (4, 5, 6, 4, 2, 0), (4, 5, 6, 4, 4, 0),
                                                  (3, 4, 6, 1, 1, 0)])
def test_topk_equals_explicit(no, nv, na, seed, k, spin):
    """TOP(k) (paper Sec. II.C: L = triples containing any large TOP, up to
    TOP(all)): the oracle's determinant-level operator, right-hand side, S-triple
    energy and E2 equal the explicit construction with k large TOPs, and the
    layout covers every determinant of D + L exactly once."""
    from oracle import topk
    ex, r1, tk = _topk_case(no, nv, na, seed, k, spin)
    dets = tk.determinants()
    live = np.where(tk.live)[0]
    idx = np.array([ex.index[dets[i]] for i in live])
    assert len(set(idx)) == len(idx)
    nons2 = [i for i in live if tk.box[i] != 1]
    assert len(live) + len(nons2) == len(ex.DL)               # own determinants + spin-flip partners
    b = tk.rhs()
    np.testing.assert_allclose(b[live], ex.b[idx], rtol=0, atol=1e-14 * max(1.0, np.abs(ex.b).max()))
    rng = np.random.default_rng(seed + 7)
    x = np.where(tk.live, rng.standard_normal(tk.dim), 0.0)
    cx = tk._coeff(x)
    c = np.zeros(len(ex.DL))
    c[idx] = cx[live]
    fh, fp = tk._flip(tk.holes), tk._flip(tk.parts)
    for i in nons2:
        d = tk.phi
        for v in fh[i]:
            if v != topk.SENT:
                d ^= 1 << int(v)
        for v in fp[i]:
            if v != topk.SENT:
                d |= 1 << int(v)
        c[ex.index[d]] = tk.sg * cx[i]
    yd = ex.A @ c
    y = tk.sigma(x)
    assert np.abs(y[live] - yd[idx]).max() <= 1e-13 * np.abs(yd).max()
    r2 = tk.solve(tol=1e-13)
    assert abs(r2["e2"] - r1["e2"]) < 1e-13 * abs(r1["e2"])
    assert abs(r2["e2_s"] - r1["e2_s"]) < 1e-13 * abs(r1["e2"])


def test_topk_one_equals_structured():
    """TOP(1) through the generic TOP(k) operator equals the seven-box oracle
    (same layout, canonical versus operator-string phase) at a size the explicit
    construction cannot reach."""
    from oracle import topk
    p, lam, Ft, Bt = _rotated(4, 12, 14, 9)
    tk = topk.TopK(Ft, Bt, lam, 4, 1)
    st = structured.Structured(Ft, lam, 4)
    x = synth.random_amplitudes(st.dim, 3)
    y = tk.phase * tk.sigma(tk.phase * x)
    ref = st.sigma(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    r = tk.solve(tol=1e-12)
    r1 = structured.solve(Ft, Bt, lam, 4, tol=1e-12)
    assert abs(r["e2"] - r1["e2"]) < 1e-12 * abs(r1["e2"])


def test_topk_more_large_tops_lower_e2_s_share():
    """Moving TOPs from S into L: with every TOP large (TOP(all)) the S-triple
    space is empty (Sec. III.B, Table II), so E2_S = 0; E2 changes with k."""
    from oracle import topk
    p, lam, Ft, Bt = _rotated(3, 5, 6, 2)
    rs = [topk.TopK(Ft, Bt, lam, 3, k).solve(tol=1e-13) for k in (1, 2, 3)]
    assert abs(rs[2]["e2_s"]) < 1e-13 * abs(rs[0]["e2_s"])
    assert abs(rs[0]["e2"] - rs[1]["e2"]) > 1e-12 and abs(rs[1]["e2"] - rs[2]["e2"]) > 1e-12
