"""GPU parity of spin-unrestricted cells (ltmp2_setup_unrestricted) against
the CPU oracle (oracle.unrestricted), through the C ABI.

Inputs: the small workload's cell with two spin channels split by a second
seeded potential (synthetic.make_cell_spin), 4 and 3 occupied states.
Energies are compared at the same (tau, w); FP64 to 1e-9 relative, the
mixed forms to 1 micro-Hartree per occupied state of both channels.
"""
import sys

import numpy as np
import pytest

from synthetic import make_cell, make_cell_spin, C1

pytestmark = pytest.mark.gpu

N_OCC_B = 3


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(spec, m, e, c, n_occ=None, **kw):
    from paper_1611_06797_amd import Context
    n_tau = len(kw["tau"]) if kw.get("tau") is not None else spec.n_tau
    return Context(spec.L, spec.n, spec.ecut, spec.eaux, m, e, c,
                   spec.n_occ if n_occ is None else n_occ, n_tau, **kw)


@pytest.fixture(scope="module")
def spin_case(torch_cuda):
    from oracle.unrestricted import UProblem
    from oracle.quadrature import minimax_laplace
    m, e1, c1, e2, c2 = make_cell_spin(C1, n_occ_b=N_OCC_B)
    U = UProblem(C1.L, C1.n, C1.eaux, m, e1, c1, C1.n_occ, e2, c2, N_OCC_B)
    tau, w, _ = minimax_laplace(*U.x_range(), C1.n_tau)
    ref = U.energies(tau, w)
    return m, e1, c1, e2, c2, U, tau, w, ref


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_spin_energy(spin_case, prec):
    m, e1, c1, e2, c2, U, tau, w, ref = spin_case
    _say("C1 spin-unrestricted energy, prec", prec)
    with _ctx(C1, m, e1, c1, tau=tau, w=w, prec=prec,
              second_spin=(e2, c2, N_OCC_B)) as ctx:
        ed, ex, pt, qe = ctx.energy()
        info = ctx.info
    assert info.n_spin == 2 and info.n_occ_b == N_OCC_B and info.n_occ == C1.n_occ
    dd, dx = abs(ed - ref["e_d_lt"]), abs(ex - ref["e_x_lt"])
    print(f"[spin prec={prec}] dE_d={dd:.3e} dE_x={dx:.3e}")
    tol = (C1.n_occ + N_OCC_B) * 1e-6
    assert dd < tol and dx < tol
    if prec == 0:
        assert dd <= 1e-9 * abs(ref["e_d_lt"]) and dx <= 1e-9 * abs(ref["e_x_lt"])
        assert np.allclose(pt[:, 0], ref["per_tau_d"], rtol=1e-9, atol=0)
        assert np.allclose(pt[:, 1], ref["per_tau_x"], rtol=1e-9, atol=0)


def test_spin_library_quadrature(spin_case):
    # one quadrature fitted on the range of both channels
    m, e1, c1, e2, c2, U, tau, w, ref = spin_case
    _say("C1 spin-unrestricted library quadrature")
    with _ctx(C1, m, e1, c1, second_spin=(e2, c2, N_OCC_B)) as ctx:
        t2, w2, d2 = ctx.get_quadrature()
        xmin, xmax = ctx.info.x_min, ctx.info.x_max
    lo, hi = U.x_range()
    assert abs(xmin - lo) <= 1e-14 * hi and abs(xmax - hi) <= 1e-14 * hi
    assert np.allclose(t2, tau, rtol=1e-9) and np.allclose(w2, w, rtol=1e-9)


def test_spin_chi_sum_and_exchange(spin_case, torch_cuda):
    # ltmp2_chi returns the transform of chi_1 + chi_2; per-tau values are
    # spin-summed; disjoint G' ranges of the exchange add up
    torch = torch_cuda
    m, e1, c1, e2, c2, U, tau, w, ref = spin_case
    _say("C1 spin-unrestricted chi(G,G') and exchange ranges")
    with _ctx(C1, m, e1, c1, tau=tau, w=w, second_spin=(e2, c2, N_OCC_B)) as ctx:
        ng, nh = ctx.info.n_g, ctx.info.n_h
        out = torch.zeros((ng, ng), dtype=torch.complex128, device="cuda")
        edt = ctx.chi(3, out)
        aux = ctx.aux_miller()
        full = ctx.exchange(5)
        parts = [ctx.exchange(5, a, b - a) for a, b in [(0, 9), (9, 60), (60, nh)]]
    pos = {tuple(v): k for k, v in enumerate(U.ch[0].aux.tolist())}
    idx = np.array([pos[tuple(v)] for v in aux.tolist()])
    Cref = U.chi_GG(tau[3])[np.ix_(idx, idx)]
    assert np.abs(out.cpu().numpy() - Cref).max() <= 1e-11 * np.abs(Cref).max()
    assert abs(edt - ref["per_tau_d"][3]) <= 1e-10 * abs(ref["per_tau_d"][3])
    assert abs(sum(parts) - full) <= 1e-12 * abs(full)
    assert abs(full - ref["per_tau_x"][5]) <= 1e-10 * abs(full)


@pytest.mark.parametrize("prec", [0, 2])
def test_identical_channels_equal_restricted(torch_cuda, prec):
    m, e, c = make_cell(C1)
    _say("C1 identical spin channels vs restricted, prec", prec)
    with _ctx(C1, m, e, c, prec=prec) as ctx:
        r = ctx.energy()
        tq = ctx.get_quadrature()[0]
    with _ctx(C1, m, e, c, prec=prec, second_spin=(e, c, C1.n_occ)) as ctx:
        u = ctx.energy()
        tu = ctx.get_quadrature()[0]
        with pytest.raises(Exception):
            ctx.direct_hartree(0)   # the Hartree-like route is spin-restricted only
    assert np.allclose(tq, tu, rtol=1e-13)
    rt = 1e-12 if prec == 0 else 1e-6
    assert abs(u[0] - r[0]) <= rt * abs(r[0]) and abs(u[1] - r[1]) <= rt * abs(r[1])


def _cap_for_blocks(m, e, c, n_occ, tau, w, g_max):
    """Largest workspace cap (within 1 KiB) at which a cell of this channel
    runs its exchange in blocks of at most g_max outer G'."""
    with _ctx(C1, m, e, c, n_occ=n_occ, tau=tau, w=w) as ctx:
        hi = ctx.info.device_bytes
    lo = 0
    while hi - lo > 1024:
        mid = (lo + hi) // 2
        try:
            with _ctx(C1, m, e, c, n_occ=n_occ, tau=tau, w=w, workspace_cap=mid) as ctx:
                gb = ctx.info.g_block
        except Exception:
            lo = mid
            continue
        if gb <= g_max:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("n_occ_1,n_occ_2,g_max", [(4, 3, 30), (2, 5, 2)])
def test_spin_multi_block_exchange(torch_cuda, n_occ_1, n_occ_2, g_max):
    # a workspace cap that splits the exchange into several G' blocks; with
    # (2, 5) and at most 2 G' per block channel 2 does not fit one G' of its
    # own into channel 1's transformed-state buffers and takes its own
    from oracle.unrestricted import UProblem
    from oracle.quadrature import minimax_laplace
    m, e1, c1, e2, c2 = make_cell_spin(C1, n_occ_b=n_occ_2)
    U = UProblem(C1.L, C1.n, C1.eaux, m, e1, c1, n_occ_1, e2, c2, n_occ_2)
    tau, w, _ = minimax_laplace(*U.x_range(), 4)
    ref = U.energies(tau, w)
    _say("C1 spin multi-block exchange", n_occ_1, n_occ_2)
    cap = _cap_for_blocks(m, e1, c1, n_occ_1, tau, w, g_max)
    with _ctx(C1, m, e1, c1, n_occ=n_occ_1, tau=tau, w=w, workspace_cap=cap,
              second_spin=(e2, c2, n_occ_2)) as ctx:
        gb, nh = ctx.info.g_block, ctx.info.n_h
        ed, ex, pt, qe = ctx.energy()
    print(f"[spin blocks {n_occ_1},{n_occ_2}] cap={cap} g_block={gb} n_h={nh}")
    assert 1 <= gb <= g_max
    assert abs(ed - ref["e_d_lt"]) <= 1e-9 * abs(ref["e_d_lt"])
    assert abs(ex - ref["e_x_lt"]) <= 1e-9 * abs(ref["e_x_lt"])


def test_spin_cutoff_extrapolation(spin_case):
    # spin-summed energies of the nested auxiliary cutoffs against the oracle
    # evaluated with each cutoff's auxiliary set
    from oracle.unrestricted import UProblem
    from oracle.extrapolation import cutoffs, extrapolate
    m, e1, c1, e2, c2, U, tau, w, ref = spin_case
    _say("C1 spin-unrestricted cutoff extrapolation")
    with _ctx(C1, m, e1, c1, tau=tau, w=w, n_extrap=8,
              second_spin=(e2, c2, N_OCC_B)) as ctx:
        ed, ex, pt, qe = ctx.energy()
        ea, edn, exn, einf = ctx.extrapolation(8)
    assert np.allclose(ea, cutoffs(C1.eaux), rtol=1e-15)
    edo, exo = [], []
    for e_n in ea:
        r = UProblem(C1.L, C1.n, e_n, m, e1, c1, C1.n_occ, e2, c2, N_OCC_B).energies(tau, w)
        edo.append(r["e_d_lt"])
        exo.append(r["e_x_lt"])
    edo, exo = np.array(edo), np.array(exo)
    assert np.allclose(edn, edo, rtol=1e-9, atol=0) and np.allclose(exn, exo, rtol=1e-9, atol=0)
    assert abs(edn[0] - ed) <= 1e-12 * abs(ed) and abs(exn[0] - ex) <= 1e-12 * abs(ex)
    assert abs(einf[0] - extrapolate(ea, edo + exo)[0]) <= 1e-9 * abs(einf[0])
