"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Inputs are seeded synthetic cells (synthetic.make_cell).  Energies are
compared with the oracle's Laplace-transformed MP2 at the *same* (tau, w);
the tolerance is N_occ micro-Hartree per cell (1 uHa per occupied orbital),
and the FP64 path is additionally held to 1e-9 relative.
"""
import sys

import numpy as np
import pytest

from synthetic import make_cell, C1, CellSpec

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle(spec, m, e, c, occ=None):
    from oracle.mp2 import Problem
    return Problem(spec.L, spec.n, spec.eaux, m, e, c, spec.n_occ, occ=occ)


def _ctx(spec, m, e, c, **kw):
    from paper_1611_06797_amd import Context
    return Context(spec.L, spec.n, spec.ecut, spec.eaux, m, e, c, spec.n_occ, spec.n_tau, **kw)


def _lib_to_nat(n):
    """internal flat index (x, z, y) -> natural flat index (x, y, z)."""
    k = np.arange(n ** 3)
    x, z, y = k // (n * n), (k // n) % n, k % n
    return (x * n + y) * n + z


@pytest.fixture(scope="module")
def c1_case(torch_cuda):
    m, e, c = make_cell(C1)
    P = _oracle(C1, m, e, c)
    xmin, xmax = P.x_range()
    from oracle.quadrature import minimax_laplace
    tau, w, d = minimax_laplace(xmin, xmax, C1.n_tau)
    ref = P.energies(tau, w)
    return m, e, c, P, tau, w, ref


def test_c1_energy_fp64(c1_case):
    m, e, c, P, tau, w, ref = c1_case
    _say("C1 energy fp64 (L=8, n=12, N_occ=4)")
    with _ctx(C1, m, e, c, tau=tau, w=w) as ctx:
        ed, ex, pt, qe = ctx.energy()
    tol = C1.n_occ * 1e-6
    assert abs(ed - ref["e_d_lt"]) < tol and abs(ex - ref["e_x_lt"]) < tol
    assert abs(ed - ref["e_d_lt"]) <= 1e-9 * abs(ref["e_d_lt"])
    assert abs(ex - ref["e_x_lt"]) <= 1e-9 * abs(ref["e_x_lt"])
    assert np.allclose(pt[:, 0], ref["per_tau_d"], rtol=1e-9, atol=0)
    assert np.allclose(pt[:, 1], ref["per_tau_x"], rtol=1e-9, atol=0)


def test_c1_library_quadrature(c1_case):
    m, e, c, P, tau, w, ref = c1_case
    _say("C1 library quadrature + energy")
    with _ctx(C1, m, e, c) as ctx:
        t2, w2, d2 = ctx.get_quadrature()
        ed, ex, pt, qe = ctx.energy()
    assert np.allclose(t2, tau, rtol=1e-9) and np.allclose(w2, w, rtol=1e-9)
    assert abs(ed + ex - ref["e_d_lt"] - ref["e_x_lt"]) < C1.n_occ * 1e-6


def test_c1_green_rows(c1_case, torch_cuda):
    torch = torch_cuda
    m, e, c, P, tau, w, ref = c1_case
    n = C1.n
    nr = n ** 3
    perm = _lib_to_nat(n)
    Go, Gv = P.green(tau[2])
    with _ctx(C1, m, e, c, tau=tau, w=w) as ctx:
        for row0, nrows in [(0, 64), (1000, 77), (nr - 5, 5)]:
            _say("C1 green rows", row0, nrows)
            go = torch.zeros((nrows, nr), dtype=torch.float64, device="cuda")
            gv = torch.zeros((nrows, nr), dtype=torch.float64, device="cuda")
            ctx.green(2, row0, nrows, go, gv)
            rows = perm[row0:row0 + nrows]
            ref_o = Go[rows][:, perm]
            ref_v = Gv[rows][:, perm]
            assert np.abs(ref_o.imag).max() < 1e-12
            assert np.abs(go.cpu().numpy() - ref_o.real).max() < 1e-12 * np.abs(ref_o).max()
            assert np.abs(gv.cpu().numpy() - ref_v.real).max() < 1e-11 * np.abs(ref_v).max()


def test_c1_chi_GG(c1_case, torch_cuda):
    torch = torch_cuda
    m, e, c, P, tau, w, ref = c1_case
    _say("C1 chi(G,G')")
    with _ctx(C1, m, e, c, tau=tau, w=w) as ctx:
        ng = ctx.info.n_g
        out = torch.zeros((ng, ng), dtype=torch.complex128, device="cuda")
        edt = ctx.chi(3, out)
        aux = ctx.aux_miller()
    pos = {tuple(v): k for k, v in enumerate(P.aux.tolist())}
    idx = np.array([pos[tuple(v)] for v in aux.tolist()])
    Cref = P.chi_GG(tau[3])[np.ix_(idx, idx)]
    Cg = out.cpu().numpy()
    assert np.abs(Cg - Cref).max() <= 1e-11 * np.abs(Cref).max()
    assert abs(edt - ref["per_tau_d"][3]) <= 1e-10 * abs(ref["per_tau_d"][3])


def test_c1_exchange_sharded_sum(c1_case):
    # emulated sharding of the outer G' loop: disjoint ranges add up
    m, e, c, P, tau, w, ref = c1_case
    _say("C1 exchange by G' ranges")
    with _ctx(C1, m, e, c, tau=tau, w=w) as ctx:
        nh = ctx.info.n_h
        full = ctx.exchange(5)
        parts = [ctx.exchange(5, a, b - a) for a, b in [(0, 7), (7, 50), (50, nh)]]
    assert abs(sum(parts) - full) <= 1e-12 * abs(full)
    assert abs(full - ref["per_tau_x"][5]) <= 1e-10 * abs(full)


@pytest.mark.parametrize("seed,L,ecut,eaux,no,nt", [(1, 6.0, 3.0, 2.0, 1, 4),
                                                    (2, 7.0, 4.0, 2.5, 3, 1),
                                                    (3, 9.0, 3.0, 2.0, 7, 6)])
def test_small_cells(torch_cuda, seed, L, ecut, eaux, no, nt):
    # edge cases: a single occupied orbital (E_x = -E_d/2), one Laplace point,
    # an odd occupied count; basis and auxiliary sets of ragged size
    spec = CellSpec(L=L, n=12, ecut=ecut, eaux=eaux, n_occ=no, n_tau=nt, seed=seed)
    m, e, c = make_cell(spec)
    _say("small cell", spec)
    P = _oracle(spec, m, e, c)
    from oracle.quadrature import minimax_laplace
    tau, w, d = minimax_laplace(*P.x_range(), nt)
    ref = P.energies(tau, w)
    with _ctx(spec, m, e, c, tau=tau, w=w) as ctx:
        ed, ex, pt, qe = ctx.energy()
    assert abs(ed - ref["e_d_lt"]) <= 1e-9 * abs(ref["e_d_lt"])
    assert abs(ex - ref["e_x_lt"]) <= 1e-9 * abs(ref["e_x_lt"])
    if no == 1:
        assert abs(ex + 0.5 * ed) <= 1e-9 * abs(ed)


@pytest.mark.parametrize("prec,name", [(1, "fp32"), (2, "bf16x3")])
def test_c1_energy_mixed(c1_case, prec, name):
    # grown precision forms: FP32 storage / transforms / GEMMs (bf16x3: the
    # Green's-function GEMMs on split-BF16 MFMA), FP64 accumulation of the
    # traces and Laplace sums; bar: N_occ uHa per cell against the FP64 oracle
    m, e, c, P, tau, w, ref = c1_case
    _say("C1 energy", name)
    with _ctx(C1, m, e, c, tau=tau, w=w, prec=prec) as ctx:
        ed, ex, pt, qe = ctx.energy()
    dd, dx = ed - ref["e_d_lt"], ex - ref["e_x_lt"]
    print(f"[{name}] dE_d={dd:.3e} dE_x={dx:.3e} per-tau max "
          f"{np.abs(pt[:, 0] - ref['per_tau_d']).max():.3e} "
          f"{np.abs(pt[:, 1] - ref['per_tau_x']).max():.3e}", flush=True)
    tol = C1.n_occ * 1e-6
    assert abs(dd) < tol and abs(dx) < tol


def test_c1_green_rows_fp32(c1_case, torch_cuda):
    torch = torch_cuda
    m, e, c, P, tau, w, ref = c1_case
    n = C1.n
    nr = n ** 3
    perm = _lib_to_nat(n)
    Go, Gv = P.green(tau[1])
    _say("C1 green rows fp32")
    with _ctx(C1, m, e, c, tau=tau, w=w, prec=1) as ctx:
        go = torch.zeros((100, nr), dtype=torch.float64, device="cuda")
        gv = torch.zeros((100, nr), dtype=torch.float64, device="cuda")
        ctx.green(1, 300, 100, go, gv)
    rows = perm[300:400]
    ro = Go[rows][:, perm].real
    rv = Gv[rows][:, perm].real
    assert np.abs(go.cpu().numpy() - ro).max() < 2e-5 * np.abs(ro).max()
    assert np.abs(gv.cpu().numpy() - rv).max() < 2e-5 * np.abs(rv).max()


@pytest.fixture(scope="module")
def c2_cell(torch_cuda):
    from synthetic import C2
    m, e, c = make_cell(C2)
    return C2, m, e, c


def test_c2_occupied_subset_vs_oracle(c2_cell):
    # full 32^3 grid, all 3895 virtuals, occupied subset I = {58, 61, 62, 63}:
    # the energy restricted to i, j in I against the oracle (same tau, w)
    spec, m, e, c = c2_cell
    occ = np.array([58, 61, 62, 63])
    _say("C2 occupied subset", occ.tolist())
    from oracle.mp2 import Problem
    from oracle.quadrature import minimax_laplace
    P = Problem(spec.L, spec.n, spec.eaux, m, e, c, spec.n_occ, occ=occ)
    tau, w, _ = minimax_laplace(*P.x_range(), spec.n_tau)
    ref = P.energies(tau, w)
    sel = np.concatenate([occ, np.arange(spec.n_occ, len(e))])
    sub = CellSpec(L=spec.L, n=spec.n, ecut=spec.ecut, eaux=spec.eaux, n_occ=len(occ),
                   n_tau=spec.n_tau, seed=spec.seed)
    for prec in (0, 1, 2):
        with _ctx(sub, m, e[sel], c[sel], tau=tau, w=w, prec=prec) as ctx:
            ed, ex, pt, qe = ctx.energy()
        dd, dx = ed - ref["e_d_lt"], ex - ref["e_x_lt"]
        print(f"[c2-subset prec={prec}] E_d={ed:.10f} dE_d={dd:.3e} E_x={ex:.10f} dE_x={dx:.3e}",
              flush=True)
        assert abs(dd) < len(occ) * 1e-6 and abs(dx) < len(occ) * 1e-6
        if prec == 0:
            assert abs(dd) <= 1e-9 * abs(ref["e_d_lt"]) and abs(dx) <= 1e-9 * abs(ref["e_x_lt"])


def test_c2_full_precision_forms(c2_cell):
    # full throughput workload (64 occupied): FP32 and BF16x3 against FP64 GPU
    # within N_occ uHa; E_d(tau) <= 0 and E_x(tau) >= 0 at every point
    spec, m, e, c = c2_cell
    res = {}
    for prec in (0, 1, 2):
        _say("C2 full, prec", prec)
        with _ctx(spec, m, e, c, prec=prec) as ctx:
            res[prec] = ctx.energy()
    ed0, ex0, pt0, _ = res[0]
    assert np.all(pt0[:, 0] < 0) and np.all(pt0[:, 1] > 0)
    for prec in (1, 2):
        ed, ex, pt, _ = res[prec]
        print(f"[c2 prec={prec}] dE_d={ed - ed0:.3e} dE_x={ex - ex0:.3e}", flush=True)
        assert abs(ed - ed0) < spec.n_occ * 1e-6 and abs(ex - ex0) < spec.n_occ * 1e-6


def test_c3_occupied_subset_vs_oracle(torch_cuda):
    # the large mixed-precision cell (40^3 grid, 7649 virtuals) restricted to the
    # occupied subset I = {156, 157, 158, 159}, every precision against the
    # oracle (stored by tests/golden/make_c3_subset.py: minutes of CPU time)
    import json
    import os
    from synthetic import C3
    with open(os.path.join(os.path.dirname(__file__), "golden", "c3_subset.json")) as f:
        ref = json.load(f)
    m, e, c = make_cell(C3)
    occ = np.array(ref["occ"])
    _say("C3 occupied subset", occ.tolist())
    tau, w = np.array(ref["tau"]), np.array(ref["w"])
    sel = np.concatenate([occ, np.arange(C3.n_occ, len(e))])
    sub = CellSpec(L=C3.L, n=C3.n, ecut=C3.ecut, eaux=C3.eaux, n_occ=len(occ),
                   n_tau=C3.n_tau, seed=C3.seed)
    for prec in (0, 1, 2):
        with _ctx(sub, m, e[sel], c[sel], tau=tau, w=w, prec=prec) as ctx:
            ed, ex, pt, qe = ctx.energy()
        dd, dx = ed - ref["e_d_lt"], ex - ref["e_x_lt"]
        print(f"[c3-subset prec={prec}] E_d={ed:.10f} dE_d={dd:.3e} E_x={ex:.10f} dE_x={dx:.3e}",
              flush=True)
        assert abs(dd) < len(occ) * 1e-6 and abs(dx) < len(occ) * 1e-6
        if prec == 0:
            assert abs(dd) <= 1e-9 * abs(ref["e_d_lt"]) and abs(dx) <= 1e-9 * abs(ref["e_x_lt"])
            assert np.allclose(pt[:, 0], ref["per_tau_d"], rtol=1e-9, atol=0)
            assert np.allclose(pt[:, 1], ref["per_tau_x"], rtol=1e-9, atol=0)


def test_c3_subset_cutoff_extrapolation_paths(torch_cuda):
    # the per-shell split on the 36^3 pair forms (FP64: 256 threads x 17
    # outputs; FP32 and BF16x3: the two-per-CU 17-output form): the first
    # cutoff is the plain energy (stored oracle value for FP64), every
    # cutoff's energy agrees between the precision forms, and the nested
    # energies shrink in magnitude with the cutoff.  A context without the
    # split runs the pair instance without that epilogue (FP32: z lines read
    # through buffer resources instead of global loads): the same sums, up
    # to FP32 rounding where the two compiled instances fuse operations
    # differently (measured 1e-10 relative; bar 1e-8)
    import json
    import os
    from synthetic import C3
    with open(os.path.join(os.path.dirname(__file__), "golden", "c3_subset.json")) as f:
        ref = json.load(f)
    m, e, c = make_cell(C3)
    occ = np.array(ref["occ"])
    tau, w = np.array(ref["tau"]), np.array(ref["w"])
    sel = np.concatenate([occ, np.arange(C3.n_occ, len(e))])
    sub = CellSpec(L=C3.L, n=C3.n, ecut=C3.ecut, eaux=C3.eaux, n_occ=len(occ),
                   n_tau=C3.n_tau, seed=C3.seed)
    out = {}
    for prec in (0, 1, 2):
        _say("C3 subset cutoff extrapolation, prec", prec)
        with _ctx(sub, m, e[sel], c[sel], tau=tau, w=w, prec=prec, n_extrap=8) as ctx:
            ed, ex, pt, qe = ctx.energy()
            ea, edn, exn, einf = ctx.extrapolation(8)
        out[prec] = (edn, exn)
        assert abs(edn[0] - ed) <= 1e-12 * abs(ed) and abs(exn[0] - ex) <= 1e-12 * abs(ex)
        with _ctx(sub, m, e[sel], c[sel], tau=tau, w=w, prec=prec) as ctx:
            ed0, ex0, _, _ = ctx.energy()
        print(f"[c3 extrap prec={prec}] split - plain: dE_d={ed - ed0:.3e} dE_x={ex - ex0:.3e}",
              flush=True)
        rel = 1e-12 if prec == 0 else 1e-8
        assert abs(ed0 - ed) <= rel * abs(ed) and abs(ex0 - ex) <= rel * abs(ex)
        assert np.all(np.diff(np.abs(edn)) < 0)
        print(f"[c3 extrap prec={prec}] E_d[n]={np.round(edn, 8).tolist()} E_inf={einf[0]:.8f}",
              flush=True)
    assert abs(out[0][0][0] - ref["e_d_lt"]) <= 1e-9 * abs(ref["e_d_lt"])
    assert abs(out[0][1][0] - ref["e_x_lt"]) <= 1e-9 * abs(ref["e_x_lt"])
    for prec in (1, 2):
        assert np.abs(out[prec][0] - out[0][0]).max() < len(occ) * 1e-6
        assert np.abs(out[prec][1] - out[0][1]).max() < len(occ) * 1e-6


def test_c3_runtime_kept_set_forms(torch_cuda):
    # an auxiliary cutoff whose kept set (k_max 9) is neither of the two
    # compiled windows of the 36^3 grid, with more than 9 x 256 vectors: the
    # FP32 and BF16x3 pair transforms take the 512-thread two-field form and
    # the FP64 ones the 256-thread runtime form; the three agree to the
    # mixed-precision bar, and the FP64 energy is real and negative / positive
    from synthetic import C3
    m, e, c = make_cell(C3)
    occ = np.array([150, 153, 157, 159])
    sel = np.concatenate([occ, np.arange(C3.n_occ, len(e))])
    sub = CellSpec(L=C3.L, n=C3.n, ecut=C3.ecut, eaux=4.5, n_occ=len(occ), n_tau=6,
                   seed=C3.seed)
    res = {}
    for prec in (0, 1, 2):
        _say("C3 subset, runtime kept set, prec", prec)
        with _ctx(sub, m, e[sel], c[sel], prec=prec) as ctx:
            info = ctx.info
            res[prec] = ctx.energy()
        assert info.n_grid == 36 and info.n_g > 9 * 256
    ed0, ex0 = res[0][0], res[0][1]
    assert ed0 < 0 < ex0
    for prec in (1, 2):
        print(f"[c3 runtime kmax prec={prec}] dE_d={res[prec][0] - ed0:.3e} "
              f"dE_x={res[prec][1] - ex0:.3e}", flush=True)
        assert abs(res[prec][0] - ed0) < len(occ) * 1e-6
        assert abs(res[prec][1] - ex0) < len(occ) * 1e-6


@pytest.mark.parametrize("prec", [0, 2])
def test_c1_phased_inputs(torch_cuda, prec):
    # orbitals from a plain complex eigensolver with seeded random phases:
    # real on the grid only up to a phase each.  The library brings them to
    # real form at setup; the energy is phase invariant, and the oracle works
    # with the phased orbitals as given.
    from synthetic import make_cell_complex
    m, e, c = make_cell_complex(C1, phase_seed=7)
    _say("C1 phased inputs, prec", prec)
    P = _oracle(C1, m, e, c)
    from oracle.quadrature import minimax_laplace
    tau, w, _ = minimax_laplace(*P.x_range(), C1.n_tau)
    ref = P.energies(tau, w)
    with _ctx(C1, m, e, c, tau=tau, w=w, prec=prec) as ctx:
        ed, ex, pt, qe = ctx.energy()
    dd, dx = ed - ref["e_d_lt"], ex - ref["e_x_lt"]
    print(f"[phased prec={prec}] dE_d={dd:.3e} dE_x={dx:.3e}", flush=True)
    assert abs(dd) < C1.n_occ * 1e-6 and abs(dx) < C1.n_occ * 1e-6
    if prec == 0:
        assert abs(dd) <= 1e-9 * abs(ref["e_d_lt"]) and abs(dx) <= 1e-9 * abs(ref["e_x_lt"])
        assert np.allclose(pt[:, 0], ref["per_tau_d"], rtol=1e-9, atol=0)
        assert np.allclose(pt[:, 1], ref["per_tau_x"], rtol=1e-9, atol=0)


def test_c1_multi_block_exchange(torch_cuda):
    # 12 occupied orbitals (two 8 x 8 blocks of occupied pairs, one ragged) and
    # a workspace cap that cuts the outer G' loop into several
    # transformed-state blocks; per-tau values against the oracle
    spec = CellSpec(L=8.0, n=12, ecut=6.0, eaux=4.0, n_occ=12, n_tau=6, seed=0)
    m, e, c = make_cell(spec)
    P = _oracle(spec, m, e, c)
    from oracle.quadrature import minimax_laplace
    tau, w, _ = minimax_laplace(*P.x_range(), spec.n_tau)
    ref = P.energies(tau, w)
    with _ctx(spec, m, e, c, tau=tau, w=w) as ctx:
        full_bytes, nh = ctx.info.device_bytes, ctx.info.n_h
        assert ctx.info.g_block == nh
    cap, blocks = full_bytes, 1
    for frac in (0.9, 0.8, 0.7, 0.65, 0.6, 0.55):
        cap = int(full_bytes * frac)
        try:
            with _ctx(spec, m, e, c, tau=tau, w=w, workspace_cap=cap) as ctx:
                gb = ctx.info.g_block
        except Exception:
            break
        if gb * 3 <= nh:
            break
    _say("C1 multi-block exchange: n_h", nh, "cap", cap)
    with _ctx(spec, m, e, c, tau=tau, w=w, workspace_cap=cap) as ctx:
        gb = ctx.info.g_block
        ed, ex, pt, qe = ctx.energy()
    print(f"[multi-block] n_h={nh} g_block={gb} dE_d={ed - ref['e_d_lt']:.3e} "
          f"dE_x={ex - ref['e_x_lt']:.3e}", flush=True)
    assert gb * 2 <= nh
    assert np.allclose(pt[:, 0], ref["per_tau_d"], rtol=1e-9, atol=0)
    assert np.allclose(pt[:, 1], ref["per_tau_x"], rtol=1e-9, atol=0)


@pytest.mark.parametrize("prec,tol", [(1, 1e-5), (2, 1e-4)])
def test_c1_chi_GG_mixed(c1_case, torch_cuda, prec, tol):
    # chi(G, G') element by element in the FP32 and split-BF16x3 forms against
    # the FP64 oracle; bound relative to the largest element
    torch = torch_cuda
    m, e, c, P, tau, w, ref = c1_case
    _say("C1 chi(G,G') prec", prec)
    with _ctx(C1, m, e, c, tau=tau, w=w, prec=prec) as ctx:
        ng = ctx.info.n_g
        out = torch.zeros((ng, ng), dtype=torch.complex128, device="cuda")
        edt = ctx.chi(3, out)
        aux = ctx.aux_miller()
    pos = {tuple(v): k for k, v in enumerate(P.aux.tolist())}
    idx = np.array([pos[tuple(v)] for v in aux.tolist()])
    Cref = P.chi_GG(tau[3])[np.ix_(idx, idx)]
    err = np.abs(out.cpu().numpy() - Cref).max() / np.abs(Cref).max()
    print(f"[chi prec={prec}] max |dchi| / max |chi| = {err:.3e}; "
          f"E_d(tau) rel {abs(edt / ref['per_tau_d'][3] - 1):.3e}", flush=True)
    assert err <= tol


def test_c1_green_rows_bf16x3(c1_case, torch_cuda):
    # G_occ / G_vir rows of a split-BF16x3 context come from its split
    # operands (hi*hi + hi*lo + lo*hi, FP32 accumulation): against the oracle
    torch = torch_cuda
    m, e, c, P, tau, w, ref = c1_case
    n = C1.n
    nr = n ** 3
    perm = _lib_to_nat(n)
    Go, Gv = P.green(tau[4])
    _say("C1 green rows bf16x3")
    with _ctx(C1, m, e, c, tau=tau, w=w, prec=2) as ctx:
        for row0, nrows in [(0, 64), (300, 100), (nr - 5, 5)]:
            go = torch.zeros((nrows, nr), dtype=torch.float64, device="cuda")
            gv = torch.zeros((nrows, nr), dtype=torch.float64, device="cuda")
            ctx.green(4, row0, nrows, go, gv)
            rows = perm[row0:row0 + nrows]
            ro = Go[rows][:, perm].real
            rv = Gv[rows][:, perm].real
            eo = np.abs(go.cpu().numpy() - ro).max() / np.abs(Go).max()
            ev = np.abs(gv.cpu().numpy() - rv).max() / np.abs(Gv).max()
            print(f"[green bf16x3 rows {row0}+{nrows}] occ {eo:.3e} vir {ev:.3e}", flush=True)
            assert eo < 1e-4 and ev < 1e-4


def _subset16(name, spec):
    """Oracle energy of a 16-orbital occupied subset (stored by
    tests/golden/make_subsets.py) against every precision form: two 8 x 8
    blocks of occupied pairs on the full transform grid, all virtuals."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"{name}_subset16.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet")
    with open(path) as f:
        ref = json.load(f)
    m, e, c = make_cell(spec)
    occ = np.array(ref["occ"])
    tau, w = np.array(ref["tau"]), np.array(ref["w"])
    sel = np.concatenate([occ, np.arange(spec.n_occ, len(e))])
    sub = CellSpec(L=spec.L, n=spec.n, ecut=spec.ecut, eaux=spec.eaux, n_occ=len(occ),
                   n_tau=spec.n_tau, seed=spec.seed)
    for prec in (0, 1, 2):
        _say(f"{name} 16-orbital subset, prec {prec}")
        with _ctx(sub, m, e[sel], c[sel], tau=tau, w=w, prec=prec) as ctx:
            ed, ex, pt, qe = ctx.energy()
            gb, nh = ctx.info.g_block, ctx.info.n_h
        dd, dx = ed - ref["e_d_lt"], ex - ref["e_x_lt"]
        print(f"[{name}-subset16 prec={prec}] g_block={gb}/{nh} E_d={ed:.10f} dE_d={dd:.3e} "
              f"E_x={ex:.10f} dE_x={dx:.3e}", flush=True)
        assert abs(dd) < len(occ) * 1e-6 and abs(dx) < len(occ) * 1e-6
        if prec == 0:
            assert abs(dd) <= 1e-9 * abs(ref["e_d_lt"]) and abs(dx) <= 1e-9 * abs(ref["e_x_lt"])
            assert np.allclose(pt[:, 0], ref["per_tau_d"], rtol=1e-9, atol=0)
            assert np.allclose(pt[:, 1], ref["per_tau_x"], rtol=1e-9, atol=0)


def test_c2_subset16_vs_oracle(torch_cuda):
    from synthetic import C2
    _subset16("c2", C2)


def test_c3_subset16_vs_oracle(torch_cuda):
    from synthetic import C3
    _subset16("c3", C3)


@pytest.mark.parametrize("prec", [0, 2])
def test_c1_cutoff_extrapolation(c1_case, prec):
    # internal cutoff extrapolation: the energies of the eight nested
    # auxiliary cutoffs E_aux / 1.05^(n-1), taken from one pass of the path,
    # against eight independent oracle evaluations with those auxiliary sets,
    # and the intercepts of the E_aux^(-3/2) fit against the oracle's
    from oracle.extrapolation import energies_at_cutoffs, extrapolate, cutoffs
    m, e, c, P, tau, w, ref = c1_case
    _say("C1 cutoff extrapolation, prec", prec)
    ed_o, ex_o = energies_at_cutoffs(C1.L, C1.n, C1.eaux, m, e, c, C1.n_occ, tau, w)
    with _ctx(C1, m, e, c, tau=tau, w=w, prec=prec, n_extrap=8) as ctx:
        ed, ex, pt, qe = ctx.energy()
        ea, edn, exn, einf = ctx.extrapolation(8)
    assert np.allclose(ea, cutoffs(C1.eaux), rtol=1e-15)
    assert abs(edn[0] - ed) <= 1e-12 * abs(ed) and abs(exn[0] - ex) <= 1e-12 * abs(ex)
    ref_inf = [extrapolate(ea, ed_o + ex_o)[0], extrapolate(ea, ed_o)[0], extrapolate(ea, ex_o)[0]]
    print(f"[extrap prec={prec}] max dE_d[n]={np.abs(edn - ed_o).max():.3e} "
          f"max dE_x[n]={np.abs(exn - ex_o).max():.3e} E_inf={einf[0]:.10f} "
          f"(oracle {ref_inf[0]:.10f})", flush=True)
    if prec == 0:
        assert np.allclose(edn, ed_o, rtol=1e-9, atol=0) and np.allclose(exn, ex_o, rtol=1e-9, atol=0)
        assert np.allclose(einf, ref_inf, rtol=1e-8, atol=0)
    else:
        tol = C1.n_occ * 1e-6
        assert np.abs(edn - ed_o).max() < tol and np.abs(exn - ex_o).max() < tol


def test_c2_subset_cutoff_extrapolation(torch_cuda):
    # the same on the 32^3 cell (two occupied orbitals, all virtuals) against
    # stored oracle energies (tests/golden/make_extrapolation.py)
    import json
    import os
    from synthetic import C2
    path = os.path.join(os.path.dirname(__file__), "golden", "c2_extrapolation.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet")
    ref = json.load(open(path))
    m, e, c = make_cell(C2)
    occ = np.array(ref["occ"])
    sel = np.concatenate([occ, np.arange(C2.n_occ, len(e))])
    sub = CellSpec(L=C2.L, n=C2.n, ecut=C2.ecut, eaux=C2.eaux, n_occ=len(occ), n_tau=C2.n_tau,
                   seed=C2.seed)
    for prec in (0, 2):
        _say("C2 subset cutoff extrapolation, prec", prec)
        with _ctx(sub, m, e[sel], c[sel], tau=np.array(ref["tau"]), w=np.array(ref["w"]),
                  prec=prec, n_extrap=8) as ctx:
            ctx.energy()
            ea, edn, exn, einf = ctx.extrapolation(8)
        dd = np.abs(edn - np.array(ref["e_d"])).max()
        dx = np.abs(exn - np.array(ref["e_x"])).max()
        print(f"[c2 extrap prec={prec}] max dE_d[n]={dd:.3e} max dE_x[n]={dx:.3e} "
              f"E_inf={einf[0]:.10f} (oracle {ref['e_inf'][0]:.10f})", flush=True)
        if prec == 0:
            assert np.allclose(edn, ref["e_d"], rtol=1e-9, atol=0)
            assert np.allclose(exn, ref["e_x"], rtol=1e-9, atol=0)
            assert np.allclose(einf, ref["e_inf"], rtol=1e-8, atol=0)
        else:
            assert dd < len(occ) * 1e-6 and dx < len(occ) * 1e-6


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_c1_direct_term_two_routes(c1_case, prec):
    # the direct term by the Hartree-like step (transformed states, h =
    # sum_i psi_i w_i, its transform and Coulomb sum) against the
    # Green's-function chi route and the oracle; the two routes share no kernel
    m, e, c, P, tau, w, ref = c1_case
    _say("C1 direct term, Hartree-like route, prec", prec)
    with _ctx(C1, m, e, c, tau=tau, w=w, prec=prec) as ctx:
        for it in (0, 4, C1.n_tau - 1):
            eh = ctx.direct_hartree(it)
            ec = ctx.chi(it)
            r = ref["per_tau_d"][it]
            print(f"[hartree prec={prec} tau {it}] route diff {abs(eh - ec) / abs(r):.3e} "
                  f"vs oracle {abs(eh - r) / abs(r):.3e}", flush=True)
            if prec == 0:
                assert abs(eh - ec) <= 1e-11 * abs(r) and abs(eh - r) <= 1e-10 * abs(r)
            else:
                assert abs(eh - r) <= 1e-4 * abs(r)


def test_c1_direct_term_two_routes_blocked(torch_cuda):
    # the Hartree-like route with the outer G' loop cut into blocks
    spec = CellSpec(L=8.0, n=12, ecut=6.0, eaux=4.0, n_occ=12, n_tau=6, seed=0)
    m, e, c = make_cell(spec)
    _say("Hartree-like route, several G' blocks")
    with _ctx(spec, m, e, c) as ctx:
        full = ctx.info.device_bytes
    with _ctx(spec, m, e, c, workspace_cap=int(full * 0.6)) as ctx:
        assert ctx.info.g_block < ctx.info.n_h
        for it in (1, 5):
            eh, ec = ctx.direct_hartree(it), ctx.chi(it)
            assert abs(eh - ec) <= 1e-11 * abs(ec)
