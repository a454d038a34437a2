"""GPU parity of the collision operators other than BGK (reading R29: two relaxation times, the
regularised operator and multiple relaxation times) against the FP64 oracle, through the C ABI,
for the step and for the hand-written adjoint (against autograd through the oracle, and against
finite differences of the GPU forward at C4's full size).

FP64 storage matches to 1e-10 (max-norm per state group, as for BGK); FP32 and FP16 storage use
the bounds stated at the test.  tau = 0.7 so that the TRT even rate differs from the odd one
(Lambda = 1/4: tau_plus = 1.75; Lambda = 1/12: tau_plus = 0.917).
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import lbm_oracle as O
from test_gpu_parity import TOL64, comp_errors, oracle_state, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2201_05473_amd import load_library
    load_library()


COLLISIONS = {
    "trt_quarter": dict(collision=wl.TRT, trt_magic=0.25),
    "trt_twelfth": dict(collision=wl.TRT, trt_magic=1.0 / 12.0),
    "regularised": dict(collision=wl.REG),
    # rates of energy, energy square, heat flux and stress all away from 1/tau and from each other
    "mrt": dict(collision=wl.MRT, mrt_se=1.3, mrt_seps=0.6, mrt_sq=1.7, mrt_spi=1.2),
}
VARIANTS = {
    "window": dict(moving_window=1),
    "periodic_z": dict(periodic=1),
    "periodic_zr_cartesian": dict(periodic=3, fields_on=0, cyl_on=0),
    "tanh_window": dict(ramp_kind=2, ramp_start=3.0, ramp_len=2.0, moving_window=1),
    "linear_vacuum_floor": dict(ramp_kind=1, ramp_start=4.5, ramp_len=1.5, moving_window=1, n_floor=1e-8),
}


@pytest.mark.parametrize("var", list(VARIANTS))
@pytest.mark.parametrize("coll", list(COLLISIONS))
def test_fp64_parity(coll, var):
    """150 x 13 (three 64-wide tiles with a ragged tail, four 4-row tiles with a ragged tail),
    27 steps, driver, noise and random initial momentum: every state value."""
    cfg = wl.config(None, nz=150, nr=13, dz=0.05, dr=0.05, nb=0.3, sigma_z=0.4, sigma_r=0.3,
                    zd0=5.0, noise_amp=1e-3, seed=11, storage=wl.F64, tau=0.7,
                    **COLLISIONS[coll], **VARIANTS[var])
    pert = wl.density_perturbation(cfg)
    pinit = wl.random_momentum(cfg, 0.05, seed=3)
    print(f"[collision fp64 parity] {coll} {var} 150x13, 27 steps", flush=True)
    lat = run_gpu(cfg, 27, pert, pinit)
    st, k, s = lat.state()
    S, P = O.run(cfg, 27, pert, pinit)
    assert (k, s) == (S.k, S.s)
    errs = comp_errors(st, oracle_state(S, P))
    assert errs.max() < TOL64, (errs.argmax(), errs.max())
    lat.close()


@pytest.mark.parametrize("coll", ["trt_quarter", "regularised", "mrt"])
def test_reduced_precision_parity_c2_copy(coll):
    """C2's 512 x 128 copy with the plasma already around the driver, 400 steps: FP32 and FP16
    storage against the FP64 oracle (max-norm relative error of n, E_z, E_r).

    Bounds.  Density: those of the BGK test (1e-5 with FP32 arithmetic, 1e-7 with FP64
    arithmetic).  Fields: with plain FP32 storage of E_r and B_theta the E_z error sat near 1e-5
    here (FP64 arithmetic on FP32 storage: BGK 9.9e-6, TRT 1.1e-5, regularised 1.7e-5); with the
    compensated fields it is below 1e-6 (TRT: FP32 arithmetic E_z 8.5e-7, E_r 4.0e-7; FP64
    arithmetic 5.8e-7, 1.8e-7).  So, as for BGK: every FP32 quantity within the target's 1e-5, the
    fields within 3e-6 (a third of the uncompensated level), and with FP64 arithmetic within
    2e-6.  FP16: 5e-3, FP16N: 5e-4 (fields) and 5e-5 (density), as for BGK."""
    cfg64 = wl.config("C2s", **COLLISIONS[coll])
    cfg64.update(ramp_start=cfg64["zd0"] - 3.0, ramp_len=1.0)
    S, P = O.run(cfg64, 400)
    ref = {"n": S.M[0].numpy(), "Ez": S.Ez.numpy(), "Er": S.Er.numpy()}
    errs = {}
    for (storage, m64) in ((wl.F32, 0), (wl.F32, 1), (wl.F16, 0), (wl.F16N, 0)):
        print(f"[collision reduced precision] {coll} C2s storage={storage} fp64_math={m64}", flush=True)
        lat = run_gpu(dict(cfg64, storage=storage, fp64_math=m64), 400)
        st, _, _ = lat.state()
        errs[(storage, m64)] = {"n": O.rel_err(st[27], ref["n"]), "Ez": O.rel_err(st[30], ref["Ez"]),
                                "Er": O.rel_err(st[31], ref["Er"])}
        print(coll, storage, m64, errs[(storage, m64)], flush=True)
        lat.close()
    f32, floor, f16 = errs[(wl.F32, 0)], errs[(wl.F32, 1)], errs[(wl.F16, 0)]
    assert max(f32.values()) < 1e-5 and floor["n"] < 1e-7, errs
    for q in ("Ez", "Er"):
        assert f32[q] < 3e-6 and floor[q] < 2e-6, (q, errs)
    assert max(f16.values()) < 5e-3, errs
    f16n = errs[(wl.F16N, 0)]
    assert f16n["n"] < 5e-5 and f16n["Ez"] < 5e-4 and f16n["Er"] < 5e-4, errs


@pytest.mark.parametrize("coll", ["trt_quarter", "regularised", "mrt"])
def test_full_size_c2_single_step(coll):
    """C2 at full size (2048 x 512, the benchmark's launch configuration), one step from the
    initial state with a seeded density perturbation and momentum, so that the populations leave
    equilibrium: FP64 to 1e-10, FP32 moments to 1e-6."""
    from paper_2201_05473_amd import Lattice
    cfg = wl.config("C2", storage=wl.F64, noise_amp=1e-2, seed=7, **COLLISIONS[coll])
    pert = wl.density_perturbation(cfg)
    pinit = wl.random_momentum(cfg, 0.05, seed=9)
    S, P = O.run(cfg, 1, pert, pinit)
    ref = oracle_state(S, P)
    for storage, tol in ((wl.F64, TOL64), (wl.F32, 1e-6)):
        print(f"[collision full size] {coll} C2 storage={storage}", flush=True)
        lat = Lattice(dict(cfg, storage=storage), pert, pinit)
        lat.step(1)
        st, k, s = lat.state()
        assert (k, s) == (S.k, S.s)
        errs = comp_errors(st, ref)
        if storage == wl.F64:
            assert errs.max() < tol, (errs.argmax(), errs.max())
        else:
            assert errs[27:].max() < tol, errs[27:]
        lat.close()


@pytest.mark.parametrize("var", ["window", "periodic_zr_cartesian", "tanh_window", "linear_vacuum_floor"])
@pytest.mark.parametrize("coll", list(COLLISIONS))
def test_vjp_step_matches_oracle_autograd(coll, var):
    """One reverse step (the window-shift step k = 4 where the window is on) on 150 x 13 at a
    state with noise and random momentum: lambda^k and the theta partials match the FP64 CPU
    adjoint to 1e-10."""
    from paper_2201_05473_amd import Lattice
    from test_gpu_adjoint import group_errors, oracle_vjp_step
    cfg = wl.config(None, nz=150, nr=13, dz=0.05, dr=0.05, nb=0.3, sigma_z=0.4, sigma_r=0.3,
                    zd0=5.0, noise_amp=1e-3, seed=11, storage=wl.F64, tau=0.7,
                    **COLLISIONS[coll], **VARIANTS[var])
    pert = wl.density_perturbation(cfg)
    pinit = wl.random_momentum(cfg, 0.05, seed=3)
    lam_next = np.random.default_rng(104).standard_normal((33, cfg["nr"], cfg["nz"]))
    print(f"[collision vjp step] {coll} {var} k=4", flush=True)
    lat = Lattice(cfg, pert, pinit)
    lat.step(4)
    lam, grad = lat.vjp_step(lam_next)
    lam_ref, grad_ref = oracle_vjp_step(cfg, 4, lam_next, pert, pinit)
    errs = group_errors(lam, lam_ref)
    assert errs.max() < 1e-10, (errs.argmax(), errs.max())
    scale = max(np.abs(grad_ref).max(), 1e-300)
    assert np.abs(grad - grad_ref).max() < 1e-10 * scale, (grad, grad_ref)
    lat.close()


def adjoint_wake_cfg(coll, storage=wl.F64):
    from test_gpu_adjoint import wake_cfg
    return dict(wake_cfg(storage), tau=0.7, **COLLISIONS[coll])


@pytest.mark.parametrize("coll", list(COLLISIONS))
def test_adjoint_gradient_matches_oracle_autograd(coll):
    """lbm_adjoint on C4's 128 x 32 copy (witness in the wake, window shifts), 60 steps with a
    checkpoint every 7 and a ragged last segment, against autograd through the FP64 oracle;
    and the FP32-storage adjoint against it (FP32 arithmetic: bound 1e-4 of the largest
    partial)."""
    from paper_2201_05473_amd import Lattice
    from test_gpu_adjoint import NAMES, theta_of
    cfg = adjoint_wake_cfg(coll)
    n, ck = 60, 7
    print(f"[collision adjoint] {coll} 128x32 {n} steps", flush=True)
    J, grad = Lattice(cfg).adjoint(n, ck, z_behind=cfg["z_behind"], row=0)
    th = theta_of(cfg)
    P = O.Params(cfg, th)
    S = O.initial_state(P)
    for _ in range(n):
        S = O.step(S, P)
    Jref = O.objective(S, P, cfg["z_behind"])
    Jref.backward()
    gref = np.array([float(th[nm].grad) for nm in NAMES])
    J32, g32 = Lattice(dict(cfg, storage=wl.F32)).adjoint(n, ck, z_behind=cfg["z_behind"], row=0)
    print(coll, "J", J, float(Jref.detach()), "grad", grad, gref, "fp32", g32, flush=True)
    assert abs(J - float(Jref.detach())) < 1e-12 * abs(float(Jref.detach()))
    assert np.abs(grad - gref).max() < 1e-9 * np.abs(gref).max(), (grad, gref)
    assert np.abs(g32 - gref).max() < 1e-4 * np.abs(gref).max(), (g32, gref)


@pytest.mark.parametrize("coll", ["trt_quarter", "regularised", "mrt"])
def test_revolve_matches_uniform_checkpointing(coll):
    """Binomial checkpointing with 3 snapshots gives the gradient of the uniform schedule (37
    steps on the 128 x 32 copy, window shifts included) and leaves the lattice at step 0."""
    from paper_2201_05473_amd import Lattice
    cfg = adjoint_wake_cfg(coll)
    n = 37
    J0, g0 = Lattice(cfg).adjoint(n, 6, z_behind=cfg["z_behind"])
    lat = Lattice(cfg)
    J, g, adv = lat.adjoint_revolve(n, 3, z_behind=cfg["z_behind"])
    print(f"[collision revolve] {coll} forward steps {adv}", flush=True)
    assert lat.counters() == (0, 0)
    assert abs(J - J0) <= 1e-13 * abs(J0)
    assert np.abs(g - g0).max() <= 1e-11 * np.abs(g0).max(), (g, g0)


@pytest.mark.parametrize("coll", list(COLLISIONS))
def test_adjoint_fd_c4(coll):
    """C4 at full size (1024 x 256, 2,000 steps, FP32 storage, checkpoints every 45 steps) with
    each operator at tau = 0.7: the adjoint gradient against central finite differences
    (h = 1e-4) of FP64 forward runs, to 1e-4 (the BGK bound)."""
    from paper_2201_05473_amd import Lattice
    from test_gpu_adjoint import NAMES, gpu_objective
    cfg = wl.config("C4", tau=0.7, **COLLISIONS[coll])
    n, ck, zb = cfg["nsteps"], 45, cfg["z_behind"]
    print(f"[collision adjoint fd] {coll} C4", flush=True)
    J, grad = Lattice(cfg).adjoint(n, ck, z_behind=zb)
    cfg64 = dict(cfg, storage=wl.F64)
    J64 = gpu_objective(cfg64, n, zb)
    fd = np.zeros(4)
    hstep = 1e-4
    for a, nm in enumerate(NAMES):
        cp, cm = dict(cfg64), dict(cfg64)
        cp[nm] += hstep
        cm[nm] -= hstep
        fd[a] = (gpu_objective(cp, n, zb) - gpu_objective(cm, n, zb)) / (2 * hstep)
    rel = np.abs(grad - fd) / np.abs(fd)
    print(coll, "C4 J32", J, "J64", J64, "adjoint", grad, "fd", fd, "rel", rel, flush=True)
    assert abs(J - J64) < 1e-4 * abs(J64)
    assert rel.max() < 1e-4, rel


def test_adjoint_rejections():
    """The adjoint refuses FP64 arithmetic on reduced storage (FP32, FP16, FP16N) for operators
    other than BGK: the forward recompute it needs exists for BGK only there."""
    from paper_2201_05473_amd import LBM_EINVAL, LbmError, Lattice
    base = wl.config(None, nz=64, nr=8, nb=0.3, zd0=2.0, sigma_z=0.3, sigma_r=0.3, tau=0.7)
    for extra, why in ((dict(collision=wl.TRT, storage=wl.F32, fp64_math=1), "fp64_math"),
                       (dict(collision=wl.MRT, storage=wl.F16, fp64_math=1), "fp64_math"),
                       (dict(collision=wl.REG, storage=wl.F16N, fp64_math=1), "fp64_math")):
        lat = Lattice(dict(base, **extra))
        with pytest.raises(LbmError) as ei:
            lat.adjoint(4, 2, z_behind=1.0)
        assert ei.value.code == LBM_EINVAL and why in str(ei.value), str(ei.value)
        with pytest.raises(LbmError) as ei:
            lat.vjp_step(np.zeros((33, 8, 64)))
        assert ei.value.code == LBM_EINVAL and why in str(ei.value), str(ei.value)
        lat.close()
    lat = Lattice(dict(base, collision=wl.BGK, storage=wl.F32, fp64_math=1))
    J, g = lat.adjoint(4, 2, z_behind=1.0)
    assert np.isfinite(J) and np.all(np.isfinite(g))
    lat.close()


def test_regularised_operator_tames_the_nonlinear_wake():
    """The paper attributes the rise of the smallest usable D in the nonlinear regime to BGK.
    Nonlinear wake (n_b = 2, Q~ = 3.9; 2048 x 256, dz = 0.02, FP32, 6,000 steps) at tau = 0.55
    (D = 0.0017, below BGK's usable range): BGK's most negative density is about -1e-2, the
    regularised operator's about -5e-5.  The test asks for a hundredfold smaller excursion.  BGK's
    excursion grows from rounding noise, so its size depends on the field precision: -0.04 with
    plain FP32 fields, -0.0099 with the compensated E_r and B_theta; the bound on BGK only asks that
    it is clearly negative."""
    import math

    from paper_2201_05473_amd import Lattice
    nmin = {}
    for coll in (wl.BGK, wl.REG):
        cfg = wl.config(None, nz=2048, nr=256, dz=0.02, dr=0.02, c_dt_over_dz=0.2, tau=0.55, storage=wl.F32,
                        moving_window=1, n0=1.0, ramp_kind=2, nb=2.0, sigma_z=0.5, sigma_r=0.5, n_floor=1e-6,
                        collision=coll)
        zd0 = cfg["nz"] * cfg["dz"] - 4.0
        cfg.update(zd0=zd0, ramp_start=zd0 + 2.0, ramp_len=2.0)
        lat = Lattice(cfg)
        lat.step(6000)
        n = lat.moments()[0]
        assert lat.diagnostics()["nonfinite"] == 0
        nmin[coll] = float(n.min())
        print(f"[nonlinear wake] collision={coll} tau=0.55 n_min={nmin[coll]:.3e}", flush=True)
        lat.close()
    assert nmin[wl.BGK] < -5e-3, nmin
    assert math.isfinite(nmin[wl.REG]) and abs(min(nmin[wl.REG], 0.0)) < 1e-2 * abs(nmin[wl.BGK]), nmin
