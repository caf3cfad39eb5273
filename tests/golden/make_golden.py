"""Write the oracle's reference values for the larger workloads.

Calls only the CPU oracle (``oracle/``) on the seeded synthetic inputs
(``synth``); nothing here touches the GPU library.  The output file
``oracle_values.json`` holds, per workload, the TOP singular values, E0,
the right-hand-side and solution norms, E2 and its parts, plus a few sampled
amplitudes of b, x and of sigma(x) for a seeded random x, addressed by
their flat index in the seven-box layout.

For the batched workload ("c4": 32 independent states of uneven size) it
holds E0 and E2 with its parts per state.

Names ending in "_semican" hold sigma of the same seeded random x applied by
the operator of the pinned-semicanonical basis (``topbasis.pinned_semicanonical``:
the occupied orbitals other than t and the virtuals other than t' rotated to
diagonalise their Fock blocks), at the same sampled indices.

Names "topk_<n_occ>_<n_vir>_<n_aux>_<seed>_<k>" hold ESMP2-TOP(k) values of
``oracle.topk`` (k large TOPs): E2 and its parts, E0, and sampled elements
of b and of sigma of a seeded random vector (layout of the TOP(k) sets,
operator-string phase of the one-TOP layout), on ``synth.make_problem``.

Names ending in "_triplet" hold the same quantities for the M_s = 0 triplet
reference (beta singles with the opposite sign).

For the differentiation workload ("c5_grad", the n_occ = 8 problem) it holds
dE2/dF~ and dE2/dB~ (TOP basis, rotation held fixed) on seeded samples of
entries, from ``oracle.gradient`` (exact central differences of the
stationary functional at the oracle's own solution).

Usage:  python tests/golden/make_golden.py [c2 c3 c5 c4 c5_grad c5_triplet ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth                                   # noqa: E402
from oracle import gradient, structured, topbasis        # noqa: E402


def sample_indices(dim, offsets, seed):
    rng = np.random.default_rng(seed)
    idx = []
    for k in range(7):
        lo, hi = offsets[k], offsets[k + 1]
        if hi > lo:
            idx += list(rng.integers(lo, hi, 24))
            idx += [lo, hi - 1]
    return sorted(set(int(i) for i in idx))


def run(name, spin=0):
    p = synth.config_problem(name)
    t0 = time.time()
    lam, R = topbasis.top_rotation(p.F, p.C, p.n_occ)
    Ft, Bt = topbasis.rotate(p.F, p.B, R)
    rh = structured.RHS(Ft, Bt, lam, p.n_occ, spin=spin)
    op = rh.op
    b = rh.rhs()
    x, r, it, rel = structured.pcg(op, b, tol=1e-10, max_iter=400)
    e2_dl = op.dot(b, x) - op.dot(x, r)
    e2_s = rh.e2_s()
    from oracle.layout import box_offsets
    off = [int(v) for v in box_offsets(p.n_occ, p.n_vir)]
    xr = synth.random_amplitudes(op.dim, 1234)
    sig = op.sigma(xr)
    idx = sample_indices(op.dim, off, 99)
    out = dict(n_occ=p.n_occ, n_vir=p.n_vir, n_aux=p.n_aux, spin=spin, dim=op.dim, offsets=off,
               lam=lam.tolist(), e0=op.E0, omega=op.omega,
               b_norm_w=float(np.sqrt(op.dot(b, b))), x_norm_w=float(np.sqrt(op.dot(x, x))),
               e2=e2_dl + e2_s, e2_dl=e2_dl, e2_s=e2_s, iters=it, rel_resid=rel,
               sample_idx=idx, b_sample=b[idx].tolist(), x_sample=x[idx].tolist(),
               sigma_seed=1234, sigma_sample=sig[idx].tolist(),
               seconds=time.time() - t0)
    return out


def run_semican(name):
    p = synth.config_problem(name)
    t0 = time.time()
    lam, R = topbasis.top_rotation(p.F, p.C, p.n_occ)
    Ft, _ = topbasis.rotate(p.F, p.B, R)
    op = structured.Structured(Ft, lam, p.n_occ)
    To, Tv = topbasis.pinned_semicanonical(Ft, p.n_occ)
    T = np.zeros_like(Ft)
    T[:p.n_occ, :p.n_occ], T[p.n_occ:, p.n_occ:] = To, Tv
    op2 = structured.Structured(T.T @ Ft @ T, lam, p.n_occ, omega=op.omega)
    from oracle.layout import box_offsets
    off = [int(v) for v in box_offsets(p.n_occ, p.n_vir)]
    xr = synth.random_amplitudes(op.dim, 1234)
    sig = op2.sigma(xr)
    idx = sample_indices(op.dim, off, 99)
    return dict(n_occ=p.n_occ, n_vir=p.n_vir, dim=op.dim, sample_idx=idx, sigma_seed=1234,
                sigma_sample=sig[idx].tolist(), seconds=time.time() - t0)


def run_topk(name):
    no, nv, na, seed, k = (int(v) for v in name.split("_")[1:])
    p = synth.make_problem(no, nv, na, seed)
    t0 = time.time()
    lam, R = topbasis.top_rotation(p.F, p.C, no)
    Ft, Bt = topbasis.rotate(p.F, p.B, R)
    from oracle import topk
    tk = topk.TopK(Ft, Bt, lam, no, k)
    r = tk.solve(tol=1e-11, max_iter=400)
    xr = np.where(tk.live, synth.random_amplitudes(tk.dim, 4321), 0.0)
    sig = tk.phase * tk.sigma(tk.phase * xr)          # operator-string phase on both sides
    rng = np.random.default_rng(77)
    live = np.where(tk.live)[0]
    idx = sorted(set(int(i) for i in rng.choice(live, 400, replace=False)))
    return dict(n_occ=no, n_vir=nv, n_aux=na, seed=seed, n_top=k, dim=tk.dim, e2=r["e2"], e2_dl=r["e2_dl"],
                e2_s=r["e2_s"], e0=r["e0"], iters=r["iters"], rel_resid=r["rel"], sample_idx=idx,
                b_sample=(tk.phase * r["b"])[idx].tolist(), sigma_seed=4321, sigma_sample=sig[idx].tolist(),
                seconds=time.time() - t0)


def run_batched():
    states = []
    for (no, nv, na, seed) in synth.batched_sizes():
        t0 = time.time()
        p = synth.make_problem(no, nv, na, seed)
        r = structured.solve_problem(p, tol=1e-10, max_iter=400)
        states.append(dict(n_occ=no, n_vir=nv, n_aux=na, seed=list(seed), e0=r["e0"], e2=r["e2"],
                           e2_dl=r["e2_dl"], e2_s=r["e2_s"], iters=r["iters"], seconds=time.time() - t0))
        print("  state", len(states) - 1, no, nv, r["e2"], "%.1fs" % states[-1]["seconds"], flush=True)
    return dict(states=states)


def gradient_entries(no, nv, na, seed):
    """Seeded sample of entries: (p, q) of F~ and (Q, p, q) of B~ with p <= q;
    most of B~'s inside the blocks E2 depends on (a row or column among the
    occupied orbitals or the TOP virtuals), the rest anywhere."""
    n = no + nv
    rng = np.random.default_rng(seed)
    fe = set()
    while len(fe) < 50:
        p, q = sorted(int(v) for v in rng.integers(0, n, 2))
        fe.add((p, q))
    be = set()
    while len(be) < 35:
        p = int(rng.integers(0, 2 * no))
        q = int(rng.integers(0, n))
        be.add((int(rng.integers(0, na)),) + tuple(sorted((p, q))))
    while len(be) < 50:
        p, q = sorted(int(v) for v in rng.integers(0, n, 2))
        be.add((int(rng.integers(0, na)), p, q))
    return sorted(fe), sorted(be)


def run_gradient(name):
    p = synth.config_problem(name)
    t0 = time.time()
    lam, R = topbasis.top_rotation(p.F, p.C, p.n_occ)
    Ft, Bt = topbasis.rotate(p.F, p.B, R)
    L = gradient.Lagrangian(Ft, Bt, lam, p.n_occ, tol=1e-12, max_iter=600)
    fe, be = gradient_entries(p.n_occ, p.n_vir, p.n_aux, 2024)
    gF = [L.grad_F(a, b) for a, b in fe]
    gB = [L.grad_B(Q, a, b) for Q, a, b in be]
    return dict(workload=name, n_occ=p.n_occ, n_vir=p.n_vir, n_aux=p.n_aux, e2=L.e2, f_entries=fe, f_grad=gF,
                b_entries=be, b_grad=gB, seconds=time.time() - t0)


if __name__ == "__main__":
    names = sys.argv[1:] or ["c1", "c2", "c5", "c3"]
    path = os.path.join(HERE, "oracle_values.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    for nm in names:
        if nm.endswith("_triplet"):
            data[nm] = run(nm[:-8], spin=1)
            print(nm, data[nm]["e2"], data[nm]["iters"], data[nm]["seconds"], flush=True)
            json.dump(data, open(path, "w"), indent=1)
            continue
        if nm.startswith("topk_"):
            data[nm] = run_topk(nm)
            print(nm, data[nm]["e2"], "%.1fs" % data[nm]["seconds"], flush=True)
            json.dump(data, open(path, "w"), indent=1)
            continue
        if nm.endswith("_semican"):
            data[nm] = run_semican(nm[:-8])
            print(nm, "%.1fs" % data[nm]["seconds"], flush=True)
            json.dump(data, open(path, "w"), indent=1)
            continue
        if nm.endswith("_grad"):
            data[nm] = run_gradient(nm[:-5])
            print(nm, data[nm]["e2"], "%.1fs" % data[nm]["seconds"], flush=True)
            json.dump(data, open(path, "w"), indent=1)
            continue
        data[nm] = run_batched() if nm == "c4" else run(nm)
        if nm == "c4":
            print(nm, len(data[nm]["states"]), "states", flush=True)
            json.dump(data, open(path, "w"), indent=1)
            continue
        print(nm, data[nm]["e2"], data[nm]["iters"], data[nm]["seconds"], flush=True)
        json.dump(data, open(path, "w"), indent=1)
