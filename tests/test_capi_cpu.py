"""C-ABI checks that need no GPU: symbol export, host symbolic parity with the
oracle (bit-exact), structural patterns, argument and call-order errors."""
import ctypes as C

import numpy as np
import pytest

from paper_2606_04725_amd import capi
from paper_2606_04725_amd import nmpc as N
from oracle import symbolic as S
from oracle.distillation import DistillationOCP


def test_library_exports_every_declared_symbol():
    L = capi.lib()
    declared = capi.declared_symbols()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(capi.SIGNATURES)


def _symbolic_parity(Ntr, H, alpha=2.5, ordering=N.capi.NMPC_ORDER_NESTED_DISSECTION, Hc=0):
    p = N.Problem(N.distillation_structure(Ntr, H, 0.1, alpha, ordering=ordering, control_horizon=Hc))
    p.analyze()
    lib = p.export_symbolic()
    m = DistillationOCP(Ntr, H, 0.1, alpha, Hc=Hc)
    assert p.m_c == m.m_c
    r, c = S.kkt_lower_pattern(m)
    if ordering == N.capi.NMPC_ORDER_NESTED_DISSECTION:
        a = S.analyze(m.n, r, c, graph_stages=(m.H, m.ns, m.nx))
    elif ordering == N.capi.NMPC_ORDER_FAMILY_DISSECTION:
        a = S.analyze(m.n, r, c, stages=(m.H, m.ns))
    else:
        a = S.analyze(m.n, r, c)
    assert np.array_equal(lib["perm"], a["perm"])
    assert np.array_equal(lib["parent"], a["parent"])
    assert np.array_equal(lib["colcount"], a["colcount"])
    assert np.array_equal(lib["snode_ptr"], a["snode_ptr"])
    rp = lib["snode_rows_ptr"]
    assert len(a["snode_rows"]) == lib["n_supernodes"]
    for s, rows in enumerate(a["snode_rows"]):
        assert np.array_equal(lib["snode_rows"][rp[s]:rp[s + 1]], rows)
    assert lib["nnz_l"] == a["nnz_L"] and lib["flops"] == a["flops"]
    pat = p.patterns()
    assert set(zip(pat["k_rows"], pat["k_cols"])) == set(zip(r, c))
    assert p.nnz_k == len(r)
    mj = len(m.jc_rows)
    assert set(zip(pat["j_rows"][:mj], pat["j_cols"][:mj])) == set(zip(m.jc_rows, m.jc_cols))
    assert set(zip(pat["j_rows"][mj:] - m.m_c, pat["j_cols"][mj:])) == set(zip(m.jd_rows, m.jd_cols))
    assert set(zip(pat["w_rows"], pat["w_cols"])) == set(zip(m.h_rows, m.h_cols))
    return lib


@pytest.mark.parametrize("Ntr,H", [(2, 1), (3, 4), (10, 20), (7, 13), (40, 100)])
def test_symbolic_bit_exact_vs_oracle(Ntr, H):
    _symbolic_parity(Ntr, H)


@pytest.mark.parametrize("Ntr,H,Hc", [(3, 4, 1), (10, 20, 5), (40, 100, 30)])
def test_control_horizon_patterns_and_symbolic_vs_oracle(Ntr, H, Hc):
    """Hold rows u_k - u_{k-1} (k >= Hc) join the equality rows; their products
    lie inside the move penalty's pattern, so the analysis matches the oracle's
    and equals the unheld problem's."""
    lib = _symbolic_parity(Ntr, H, Hc=Hc)
    free = _symbolic_parity(Ntr, H)
    for key in ("perm", "parent", "colcount", "snode_ptr", "snode_rows"):
        assert np.array_equal(lib[key], free[key]), key


@pytest.mark.parametrize("Ntr,H", [(2, 1), (3, 4), (10, 20), (40, 100)])
def test_symbolic_bit_exact_vs_oracle_min_degree(Ntr, H):
    _symbolic_parity(Ntr, H, ordering=N.capi.NMPC_ORDER_MIN_DEGREE)


@pytest.mark.parametrize("Ntr,H", [(2, 1), (3, 4), (10, 20), (40, 100)])
def test_symbolic_bit_exact_vs_oracle_family_dissection(Ntr, H):
    _symbolic_parity(Ntr, H, ordering=N.capi.NMPC_ORDER_FAMILY_DISSECTION)


@pytest.mark.slow
def test_symbolic_bit_exact_batch_instance_sizes():
    from workloads.generators import batch_distillation_workloads
    ws = batch_distillation_workloads(64)
    big = max(ws, key=lambda w: w.N * w.H)
    _symbolic_parity(big.N, big.H, big.alpha)


@pytest.mark.parametrize("family", [False, True], ids=["nested_dissection", "family_dissection"])
@pytest.mark.parametrize("G,H", [(4, 3), (8, 4), (12, 7), (16, 10)])
def test_plate_symbolic_bit_exact_vs_oracle(G, H, family):
    from oracle.plate import PlateOCP
    o = N.capi.NMPC_ORDER_FAMILY_DISSECTION if family else N.capi.NMPC_ORDER_NESTED_DISSECTION
    p = N.Problem(N.plate_structure(G, H, 0.01, ordering=o))
    p.analyze()
    lib = p.export_symbolic()
    m = PlateOCP(G, H, 0.01)
    r, c = S.kkt_lower_pattern(m)
    if family:
        a = S.analyze(m.n, r, c, lattice=(H, G, m.ns))
    else:
        a = S.analyze(m.n, r, c, graph_stages=(H, m.ns, m.nx))
    for key in ("perm", "parent", "colcount", "snode_ptr"):
        assert np.array_equal(lib[key], a[key if key != "snode_ptr" else "snode_ptr"]), key
    rp = lib["snode_rows_ptr"]
    for s_, rows in enumerate(a["snode_rows"]):
        assert np.array_equal(lib["snode_rows"][rp[s_]:rp[s_ + 1]], rows)
    pat = p.patterns()
    assert set(zip(pat["k_rows"], pat["k_cols"])) == set(zip(r, c))
    assert set(zip(pat["j_rows"], pat["j_cols"])) == set(zip(m.jc_rows, m.jc_cols))
    assert set(zip(pat["w_rows"], pat["w_cols"])) == set(zip(m.h_rows, m.h_cols))


def test_plate_symbolic_bit_exact_full_size():
    """The 32 x 32 x 50 plate workload (n = 52,000): the whole analysis
    under the family (lattice) dissection, and the permutation under the
    default one (the oracle's column structures in that order take three
    minutes of host time; its permutation a few seconds)."""
    from oracle.plate import PlateOCP
    G, H = 32, 50
    m = PlateOCP(G, H, 0.01)
    r, c = S.kkt_lower_pattern(m)
    p = N.Problem(N.plate_structure(G, H, 0.01))
    p.analyze()
    assert np.array_equal(p.export_symbolic()["perm"],
                          S.final_permutation(m.n, r, c, graph_stages=(H, m.ns, m.nx)))
    p = N.Problem(N.plate_structure(G, H, 0.01, ordering=N.capi.NMPC_ORDER_FAMILY_DISSECTION))
    p.analyze()
    lib = p.export_symbolic()
    a = S.analyze(m.n, r, c, lattice=(H, G, m.ns))
    for key in ("perm", "parent", "colcount", "snode_ptr"):
        assert np.array_equal(lib[key], a[key]), key
    rp = lib["snode_rows_ptr"]
    assert len(a["snode_rows"]) == lib["n_supernodes"]
    for s_, rows in enumerate(a["snode_rows"]):
        assert np.array_equal(lib["snode_rows"][rp[s_]:rp[s_ + 1]], rows)
    assert lib["nnz_l"] == a["nnz_L"] and lib["flops"] == a["flops"]


def test_plate_permutation_bit_exact_differentiated_size():
    """The 64 x 64 x 100 plate (n = 411,200): the column structures of L
    (6e8 entries) are out of reach of the oracle, so the contract there is the
    permutation (ordering and elimination-tree postorder, from the pattern
    alone) and its determinism across analyses."""
    from oracle.plate import PlateOCP
    G, H = 64, 100
    p = N.Problem(N.plate_structure(G, H, 0.01))
    p.analyze()
    perm = p.export_symbolic()["perm"]
    q = N.Problem(N.plate_structure(G, H, 0.01))
    q.analyze()
    assert np.array_equal(q.export_symbolic()["perm"], perm)
    m = PlateOCP(G, H, 0.01)
    r, c = S.kkt_lower_pattern(m)
    assert np.array_equal(perm, S.final_permutation(m.n, r, c, graph_stages=(H, m.ns, m.nx)))


def test_create_rejects_bad_structures():
    s = N.distillation_structure(10, 20, 0.1, 2.5)
    s.horizon = 0
    with pytest.raises(N.NMPCError) as e:
        N.Problem(s)
    assert e.value.code == capi.NMPC_ERR_INVALID_ARG
    s = N.distillation_structure(10, 20, 0.1, 0.5)     # alpha must exceed 1
    with pytest.raises(N.NMPCError):
        N.Problem(s)
    s = N.distillation_structure(10, 20, 0.1, 2.5)
    s.family = 99
    with pytest.raises(N.NMPCError) as e:
        N.Problem(s)
    assert e.value.code == capi.NMPC_ERR_UNSUPPORTED
    h = C.c_void_p()
    assert capi.lib().nmpc_create_problem(None, C.byref(h)) == capi.NMPC_ERR_INVALID_ARG
    assert b"NULL" in capi.lib().nmpc_last_error()


def test_call_order_and_argument_errors():
    p = N.Problem(N.distillation_structure(4, 3, 0.1, 2.5))
    with pytest.raises(N.NMPCError) as e:
        p.symbolic_sizes()
    assert e.value.code == capi.NMPC_ERR_BAD_ORDER
    with pytest.raises(N.NMPCError) as e:
        p.solve()
    assert e.value.code == capi.NMPC_ERR_BAD_ORDER
    x0 = np.full(p.nx, 0.5)
    x0[2] = np.nan
    with pytest.raises(N.NMPCError) as e:
        p.set_parameters(x0)
    assert e.value.code == capi.NMPC_ERR_INVALID_ARG
    p.analyze()
    p.analyze()     # idempotent
    if not N.device_available():
        with pytest.raises(N.NMPCError) as e:
            p.solve()
        assert e.value.code == capi.NMPC_ERR_NO_DEVICE
    with pytest.raises(N.NMPCError) as e:
        p.solve(warm=True)
    assert e.value.code in (capi.NMPC_ERR_BAD_ORDER, capi.NMPC_ERR_NO_DEVICE)
    capi.lib().nmpc_destroy(None)    # no-op


def test_default_options_match_oracle():
    from oracle.ipm import IPMOptions
    o = N.default_options()
    ref = IPMOptions()
    for name in ("tol", "gamma", "mu0_cold", "mu0_warm", "mu_min", "kappa_eps", "kappa_mu", "theta_mu",
                 "tau_min", "armijo", "ls_max", "max_iter", "kappa_sigma", "eta_first", "eta_min", "eta_max",
                 "kp_first", "kp", "km", "bound_push", "slack_push", "filter_gamma_theta", "filter_gamma_phi",
                 "filter_s_theta", "filter_s_phi", "filter_delta", "alpha_min_frac", "theta_max_fact",
                 "theta_min_fact", "filter_cap", "soc_max", "soc_kappa", "merit_fallback"):
        assert getattr(o, name) == pytest.approx(getattr(ref, name), rel=0, abs=0), name


def test_batch_create_argument_errors():
    from paper_2606_04725_amd import capi
    L = capi.lib()
    import ctypes as C
    p = N.Problem(N.distillation_structure(4, 3, 0.1, 2.5))
    h = C.c_void_p()
    arr = (C.c_void_p * 2)(p._h.value, p._h.value)
    assert L.nmpc_batch_create(arr, 2, C.byref(h)) == capi.NMPC_ERR_INVALID_ARG
    assert L.nmpc_batch_create(arr, 0, C.byref(h)) == capi.NMPC_ERR_INVALID_ARG
    assert L.nmpc_batch_create(arr, 1, C.byref(h)) == capi.NMPC_ERR_BAD_ORDER
    assert L.nmpc_batch_solve(None, 0, None, None) == capi.NMPC_ERR_INVALID_ARG
    L.nmpc_batch_destroy(None)
