"""GPU parity of the probes, the objective and the checkpointed discrete adjoint
against the oracle (store-all adjoint in serial C, same derivative
conventions), and properties of the checkpointed reversal.

Both sides evaluate the same discrete step map in double precision with
different summation orders; the forward states agree to ~1e-15 relative and the
gradients to ~1e-12, so the tests compare J, T_N, dJ/dW and dJ/dT_0 to 1e-9
relative (relative to the largest component for vectors)."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import need_gpu, rel_errors, sim_for

pytestmark = pytest.mark.gpu


def _off_kinks(prob):
    """The seeded law's first breakpoint is the ambient temperature, so cold
    Gauss points sit on a kink of k and c_p where the one-sided slope follows
    the last bit of the interpolated T, which the two sides round differently
    (both slopes are valid derivatives).  Parity inputs move that breakpoint
    below ambient."""
    T_bp = np.array(prob.T_bp, dtype=np.float64).copy()
    T_bp[0] = 250.0
    return prob.replace(T_bp=T_bp)


def _case(kind, degree=2):
    """(problem, dt, steps): the oracle's adjoint cases (3 short tracks, all
    scanned within the run, melt and consolidation reached), or a ragged
    multi-tile mesh."""
    if kind == "ragged":
        prob = W.small_nonlinear(nx=20, ny=18, nz=10, steps=0, n_tracks=3, track_length=0.03e-3,
                                 hatch=60e-6)
        prob = W.with_probes(_off_kinks(prob).replace(degree=degree), 12, seed=5, t_hi=900.0)
        return prob, 2.0e-6, 70
    prob = _off_kinks(W.small_nonlinear(nx=8, ny=6, nz=4, steps=0, n_tracks=3, track_length=0.06e-3,
                                        hatch=50e-6))
    if kind == "linear":
        prob = prob.replace(T_bp=np.array([0.0, 1e4]), k_bp=np.array([25.0, 25.0]),
                            cp_bp=np.array([600.0, 600.0]), latent=0.0, powder_k_factor=1.0,
                            powder_depth=0.0)
    prob = W.with_probes(prob.replace(degree=degree), 6, seed=3, t_hi=900.0)
    return prob, 2.5e-6, 100


def _gpu_gradient(prob, dt, n, n_snaps, T0=None, powers=None):
    sim = sim_for(prob)
    if powers is not None:
        sim.set_track_powers(powers, prob.absorptivity)
    sim.set_probes(prob.probes, prob.targets)
    T, rc = sim.init_state(prob.T0)
    if T0 is not None:
        T = torch.tensor(T0, device="cuda")
    work = sim.gradient_work(n_snaps)
    TN, J = sim.gradient_forward(T, rc, 0.0, dt, n, work)
    g = sim.gradient_backward(0.0, dt, n, work, with_lam0=True)
    torch.cuda.synchronize()
    return dict(J=J.item(), TN=TN.cpu().numpy(), dJdW=g["dJdW"].cpu().numpy(),
                dJdP=g["dJdP"].cpu().numpy(), dJdA=g["dJdA"].item(), lam0=g["lam0"].cpu().numpy(),
                n_advances=g["n_advances"])


def _oracle_gradient(prob, dt, n, T0=None, powers=None):
    o = oracle.Oracle(prob, track_power=powers)
    if T0 is None:
        T0 = o.init_T()
    J, dW, TN, lam0 = o.adjoint(T0, 0.0, dt, n, prob.probes, prob.targets, with_lam0=True)
    return dict(J=J, dJdW=dW, TN=TN, lam0=lam0)


def _vec_close(a, b, tol, what):
    mx = np.abs(a - b).max() / np.abs(b).max()
    print(f"{what}: max diff / max = {mx:.2e}")
    assert mx <= tol, what


def test_probes_and_objective_vs_oracle():
    need_gpu()
    prob, dt, _ = _case("ragged")
    o = oracle.Oracle(prob)
    T = o.init_T() + 300.0 * (1.0 + W.seeded_vector(o.N, 8))
    sim = sim_for(prob)
    sim.set_probes(prob.probes, prob.targets)
    Td = torch.tensor(T, device="cuda")
    vals = sim.probe(Td).cpu().numpy()
    np.testing.assert_allclose(vals, o.probe(T, prob.probes), rtol=1e-14, atol=0)
    J, lam = sim.objective(Td)
    Jo, _, _, lamo = o.adjoint(T, 0.0, dt, 0, prob.probes, prob.targets, with_lam0=True)
    assert abs(J.item() - Jo) <= 1e-13 * Jo
    np.testing.assert_allclose(lam.cpu().numpy(), lamo, rtol=0, atol=1e-13 * np.abs(lamo).max())


@pytest.mark.parametrize("kind,degree", [("full", 2), ("full", 1), ("linear", 2), ("ragged", 2)])
def test_gradient_vs_oracle(kind, degree):
    need_gpu()
    prob, dt, n = _case(kind, degree)
    P0 = prob.tracks[:, 7] * (1.0 + 0.1 * np.arange(len(prob.tracks)))
    g = _gpu_gradient(prob, dt, n, n_snaps=4, powers=P0)
    r = _oracle_gradient(prob, dt, n, powers=P0)
    if kind != "linear":
        assert r["TN"].max() > prob.T_l
    assert np.all(r["dJdW"] != 0)
    print(f"{kind} Q{degree}: J gpu {g['J']:.15e} oracle {r['J']:.15e}")
    assert abs(g["J"] - r["J"]) <= 1e-11 * abs(r["J"])
    mx, _ = rel_errors(g["TN"], r["TN"])
    assert mx <= 1e-13
    np.testing.assert_allclose(g["dJdW"], r["dJdW"], rtol=1e-9, atol=0)
    _vec_close(g["lam0"], r["lam0"], 1e-9, "dJ/dT0")
    # parameter gradients: dJ/dP_k = A dJ/dW_k, dJ/dA = sum_k P_k dJ/dW_k
    A = prob.absorptivity
    np.testing.assert_allclose(g["dJdP"], A * g["dJdW"], rtol=1e-15, atol=0)
    assert abs(g["dJdA"] - np.dot(P0, g["dJdW"])) <= 1e-12 * abs(g["dJdA"])


def test_surface_flux_gradient_vs_oracle():
    """Q1, constant law, Gaussian surface flux (the first configuration's physics)."""
    need_gpu()
    prob = W.with_probes(W.cfg1(), 8, seed=9, t_hi=1500.0)
    o = oracle.Oracle(prob)
    lam = o.stability_lambda(W.seeded_vector(o.N, 1), 100)
    dt = 0.5 * 2.0 / lam
    n = 40
    g = _gpu_gradient(prob, dt, n, n_snaps=5)
    r = _oracle_gradient(prob, dt, n)
    assert abs(g["J"] - r["J"]) <= 1e-11 * abs(r["J"])
    np.testing.assert_allclose(g["dJdW"], r["dJdW"], rtol=1e-9, atol=0)
    _vec_close(g["lam0"], r["lam0"], 1e-9, "dJ/dT0")


def test_checkpointing_matches_store_all_bitwise():
    """Replays are bitwise reproducible (fixed summation orders), so every
    schedule gives the same gradient bit for bit; the forward-step count is the
    binomial optimum."""
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    prob, dt, n = _case("full")
    a = _gpu_gradient(prob, dt, n, n_snaps=n)
    for s in (1, 3, 10):
        b = _gpu_gradient(prob, dt, n, n_snaps=s)
        assert b["J"] == a["J"]
        assert np.array_equal(b["dJdW"], a["dJdW"])
        assert np.array_equal(b["lam0"], a["lam0"])
        assert b["n_advances"] == pbftherm.revolve_schedule(n, s, with_actions=False)[1]
    assert a["n_advances"] == n - 1


def test_autograd_function():
    need_gpu()
    from paper_2302_05164_amd.scan_adjoint import scan_objective
    prob, dt, n = _case("full")
    sim = sim_for(prob)
    sim.set_probes(prob.probes, prob.targets)
    T0, rc0 = sim.init_state(prob.T0)
    P = torch.tensor(prob.tracks[:, 7] * 1.05, dtype=torch.float64, requires_grad=True)
    A = torch.tensor(prob.absorptivity, dtype=torch.float64, requires_grad=True)
    J = scan_objective(P, A, sim, T0, rc0, 0.0, dt, n, n_snaps=7)
    (2.0 * J).backward()
    r = _oracle_gradient(prob, dt, n, powers=P.detach().numpy())
    assert abs(J.item() - r["J"]) <= 1e-11 * r["J"]
    np.testing.assert_allclose(P.grad.numpy(), 2.0 * prob.absorptivity * r["dJdW"], rtol=1e-9)
    # dJ/dA = (1/A) sum_k P_k dJ/dP_k
    assert abs(A.grad.item() - np.dot(P.detach().numpy(), P.grad.numpy()) / prob.absorptivity) \
        <= 1e-12 * abs(A.grad.item())


def test_backward_without_forward_is_rejected():
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    prob, dt, n = _case("full")
    sim = sim_for(prob)
    sim.set_probes(prob.probes, prob.targets)
    work = sim.gradient_work(3)
    with pytest.raises(pbftherm.PbfError):
        sim.gradient_backward(0.0, dt, n, work)


# ---------------------------------------------------------------------------
# full size: the 48x48x24 Q2 box, 3000 steps, 64 probes, 10 tracks, 30 slots
# ---------------------------------------------------------------------------
def _full_size(linear=False, latent=True):
    prob = W.cfg5()
    if not latent:
        prob = prob.replace(latent=0.0)
    if linear:
        prob = prob.replace(T_bp=np.array([0.0, 1e4]), k_bp=np.array([25.0, 25.0]),
                            cp_bp=np.array([600.0, 600.0]), latent=0.0, powder_k_factor=1.0,
                            powder_depth=0.0)
    sim = sim_for(prob)
    info = sim.info()
    v0 = torch.tensor(W.seeded_vector(info["n_dofs"], 1), device="cuda")
    dt = prob.dt_factor * sim.stability_dt(v0, 100)
    sim.set_probes(prob.probes, prob.targets)
    return prob, sim, dt


def _full_gradient(sim, prob, dt, n_snaps, powers=None):
    if powers is not None:
        sim.set_track_powers(powers, prob.absorptivity)
    T0, rc0 = sim.init_state(prob.T0)
    work = sim.gradient_work(n_snaps)
    _, J = sim.gradient_forward(T0, rc0, 0.0, dt, prob.steps, work)
    g = sim.gradient_backward(0.0, dt, prob.steps, work, with_lam0=True)
    torch.cuda.synchronize()
    return J.item(), g


def test_full_size_checkpointing_matches_store_all_bitwise():
    need_gpu()
    prob, sim, dt = _full_size()
    J30, g30 = _full_gradient(sim, prob, dt, 30)
    assert g30["n_advances"] == 8472
    Jall, gall = _full_gradient(sim, prob, dt, prob.steps)
    assert gall["n_advances"] == prob.steps - 1
    assert J30 == Jall
    assert torch.equal(g30["dJdW"], gall["dJdW"]) and torch.equal(g30["lam0"], gall["lam0"])
    assert torch.isfinite(g30["lam0"]).all() and (g30["dJdW"] != 0).all()


def test_full_size_constant_law_central_differences():
    """Constant coefficients: T_N is affine in the powers, J quadratic, so central
    differences equal the derivative up to round-off at any step size."""
    need_gpu()
    prob, sim, dt = _full_size(linear=True)
    P0 = prob.tracks[:, 7].copy()
    J, g = _full_gradient(sim, prob, dt, 30, powers=P0)
    for k in (0, 5, 9):
        Js = []
        for sgn in (1.0, -1.0):
            P = P0.copy()
            P[k] += sgn * 10.0
            Js.append(_full_gradient(sim, prob, dt, 30, powers=P)[0])
        fd = (Js[0] - Js[1]) / 20.0
        dJdP = g["dJdP"][k].item()
        print(f"track {k}: adjoint {dJdP:.12e} central difference {fd:.12e}")
        assert abs(dJdP - fd) <= 1e-7 * abs(fd)


def test_backward_rejects_a_changed_problem():
    """The reversal replays forward steps and forms dJ/dP = A dJ/dW: it must run
    on the problem its forward sweep saw.  Changing the track powers, the
    absorptivity or the law in between is refused; restoring them is accepted
    and gives the unchanged gradient."""
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    prob, dt, n = _case("full")
    ref = _gpu_gradient(prob, dt, n, n_snaps=4)
    sim = sim_for(prob)
    sim.set_probes(prob.probes, prob.targets)
    T0, rc0 = sim.init_state(prob.T0)
    work = sim.gradient_work(4)
    P0 = prob.tracks[:, 7].copy()
    for change in ("powers", "absorptivity", "law"):
        sim.gradient_forward(T0, rc0, 0.0, dt, n, work)
        if change == "powers":
            sim.set_track_powers(P0 * 1.01, prob.absorptivity)
        elif change == "absorptivity":
            sim.set_track_powers(P0, prob.absorptivity * 1.01)
        else:
            sim.set_material(prob.T_bp, prob.k_bp * 1.01, prob.cp_bp, prob.rho, prob.T_s, prob.T_l,
                             prob.latent, prob.powder_k_factor, prob.powder_depth)
        with pytest.raises(pbftherm.PbfError, match="changed"):
            sim.gradient_backward(0.0, dt, n, work)
        sim.set_track_powers(P0, prob.absorptivity)
        sim.set_material(prob.T_bp, prob.k_bp, prob.cp_bp, prob.rho, prob.T_s, prob.T_l,
                         prob.latent, prob.powder_k_factor, prob.powder_depth)
        g = sim.gradient_backward(0.0, dt, n, work)
        torch.cuda.synchronize()
        assert np.array_equal(g["dJdW"].cpu().numpy(), ref["dJdW"])


# the seeded law unchanged (first breakpoint at the ambient temperature), the
# full 48x48x24 mesh, 64 probes, 10 tracks; steps 170..219 of the scan from the
# ambient state (the end of the first track and the start of the second), a
# fixed step below the stability limit (7.66e-6 s)
FULL_DT = 3.8e-6
FULL_N0, FULL_N = 170, 50


@pytest.mark.timeout(900)
def test_full_size_real_law_gradient_vs_oracle():
    """dJ/dW, dJ/dP, dJ/dA and dJ/dT_0 on the full differentiation mesh with the
    unmodified nonlinear law, against the oracle's store-all adjoint, to 1e-5
    relative (cold points sit exactly on the law's first breakpoint: both
    one-sided slopes are valid there and the sides may pick different ones)."""
    need_gpu()
    prob = W.cfg5()
    t0 = FULL_N0 * FULL_DT
    sim = sim_for(prob)
    sim.set_probes(prob.probes, prob.targets)
    T0, rc0 = sim.init_state(prob.T0)
    work = sim.gradient_work(8)
    TN, J = sim.gradient_forward(T0, rc0, t0, FULL_DT, FULL_N, work)
    g = sim.gradient_backward(t0, FULL_DT, FULL_N, work, with_lam0=True)
    torch.cuda.synchronize()
    o = oracle.Oracle(prob)
    Jo, dWo, TNo, lam0o = o.adjoint(o.init_T(), t0, FULL_DT, FULL_N, prob.probes, prob.targets, with_lam0=True)
    assert TNo.max() > prob.T_l
    active = np.nonzero(dWo)[0]
    assert len(active) >= 2  # two tracks inside the window
    dW = g["dJdW"].cpu().numpy()
    print(f"cfg5 real law, steps {FULL_N0}..{FULL_N0 + FULL_N - 1}: J gpu {J.item():.12e} oracle {Jo:.12e}")
    for k in active:
        print(f"  track {k}: dJ/dW gpu {dW[k]:.12e} oracle {dWo[k]:.12e} rel {abs(dW[k] / dWo[k] - 1):.2e}")
    assert abs(J.item() - Jo) <= 1e-11 * abs(Jo)
    mx, _ = rel_errors(TN.cpu().numpy(), TNo)
    assert mx <= 1e-13
    np.testing.assert_allclose(dW, dWo, rtol=1e-5, atol=1e-5 * np.abs(dWo).max())
    A = prob.absorptivity
    P = prob.tracks[:, 7]
    np.testing.assert_allclose(g["dJdP"].cpu().numpy(), A * dWo, rtol=1e-5, atol=1e-5 * A * np.abs(dWo).max())
    dA = g["dJdA"].item()
    dAo = float(np.dot(P, dWo))
    print(f"  dJ/dA gpu {dA:.12e} oracle {dAo:.12e}")
    assert abs(dA - dAo) <= 1e-5 * abs(dAo)
    _vec_close(g["lam0"].cpu().numpy(), lam0o, 1e-5, "dJ/dT0")


@pytest.mark.timeout(900)
def test_full_size_central_differences_without_latent_heat():
    """The 3000-step run of the differentiation workload with the seeded k(T)
    and c_p(T) tables, the powder history and the moving source, but no latent
    heat: central differences of J against the adjoint for three tracks and the
    absorptivity.  (With latent heat the apparent capacity jumps at T_s and
    T_l, so J itself jumps wherever a node's temperature crosses those values
    one step earlier or later: central differences at any h then measure the
    jumps, not the derivative, and the gradient is checked against the oracle's
    adjoint instead.)  Without latent heat J is continuous but only piecewise
    smooth: the tables are piecewise linear in T and the consolidated fraction
    is a running maximum, so a perturbation moves Gauss points across kinks and
    a central difference carries an error of first order in h.  At the
    workload's h = 1e-4 (relative) the agreement is bounded by 1e-3 (measured
    0.9e-4 .. 2.5e-4); it tightens as h shrinks, and at h = 1e-7 central
    differences agree with the adjoint to the 1e-5 bar (measured 3e-8 .. 4e-7;
    J ~ 4e7 is deterministic, so round-off stays near 1e-7 there)."""
    need_gpu()
    prob, sim, dt = _full_size(latent=False)
    P0 = prob.tracks[:, 7].copy()
    A0 = prob.absorptivity
    J, g = _full_gradient(sim, prob, dt, 30, powers=P0)
    work = sim.gradient_work(1)

    def J_at(P, A):
        sim.set_track_powers(P, A)
        T0, rc0 = sim.init_state(prob.T0)
        _, Jv = sim.gradient_forward(T0, rc0, 0.0, dt, prob.steps, work)
        torch.cuda.synchronize()
        return Jv.item()

    for name, k in [("P0", 0), ("P5", 5), ("P9", 9), ("A", None)]:
        ad = g["dJdP"][k].item() if k is not None else g["dJdA"].item()
        for hrel, bound in ((1e-4, 1e-3), (1e-7, 1e-5)):
            Js = []
            for sgn in (1.0, -1.0):
                P, A = P0.copy(), A0
                if k is None:
                    A = A0 * (1.0 + sgn * hrel)
                    step = A0 * hrel
                else:
                    P[k] = P0[k] * (1.0 + sgn * hrel)
                    step = P0[k] * hrel
                Js.append(J_at(P, A))
            fd = (Js[0] - Js[1]) / (2.0 * step)
            err = abs(fd - ad) / abs(ad)
            print(f"{name}: adjoint {ad:.10e} central difference (h = {hrel:g} rel) {fd:.10e} rel diff {err:.2e}")
            assert err <= bound, (name, hrel)
    sim.set_track_powers(P0, A0)
