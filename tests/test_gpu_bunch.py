"""GPU parity of the particle driver (reading R30: the bunch of Sec. II, Eq. (1), as macroparticles
coupled through their projected current) against the FP64 oracle, through the C ABI.

FP64: every state value to 1e-10 (max-norm per group, as for the rigid driver) and every particle
coordinate to 1e-10 relative to its scale; lost particles (w = 0) identical.  The deposit uses
atomic additions, so the GPU sums over particles in no fixed order: the agreement is to
round-off, not bit for bit.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import lbm_oracle as O
from test_gpu_parity import TOL64, comp_errors, oracle_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2201_05473_amd import load_library
    load_library()


def lattice(cfg, bunch, n_pert=None):
    from paper_2201_05473_amd import Lattice
    lat = Lattice(cfg, n_pert)
    lat.set_bunch(bunch, True)
    return lat


def bunch_errors(b, ref):
    """Max relative error of positions (scale: max |position|), momenta (max |p|) and weights."""
    ref = ref.numpy() if hasattr(ref, "numpy") else ref
    out = []
    for rows in ((0, 1, 2), (3, 4, 5), (6,)):
        den = max(np.abs(ref[list(rows)]).max(), 1e-300)
        out.append(np.abs(b[list(rows)] - ref[list(rows)]).max() / den)
    return out


CASES = {
    # gamma = 5000, the paper's bunch shape: nearly rigid, moving window
    "relativistic_window": dict(cfg=dict(moving_window=1), gamma=5000.0, emittance=0.05, spread=1e-4, steps=40),
    # gamma = 3 with a transverse spread: the push deflects the particles, some leave radially and
    # through the rear of the window (lost), and the deposit carries a radial current
    "slow_deflected": dict(cfg=dict(moving_window=1), gamma=3.0, emittance=0.4, spread=0.05, steps=60),
    # fixed window, TRT collision
    "fixed_trt": dict(cfg=dict(collision=wl.TRT, trt_magic=0.25), gamma=20.0, emittance=0.1, spread=0.01,
                      steps=30),
    # periodic z (the step variant with the wrap code; non-periodic grids take the one without)
    "periodic_z": dict(cfg=dict(periodic=1), gamma=20.0, emittance=0.1, spread=0.01, steps=30),
    # the deflected bunch again with non-temporal bunch accesses in the push and move
    "slow_deflected_streaming": dict(cfg=dict(moving_window=1, bunch_streaming=1), gamma=3.0, emittance=0.4,
                                     spread=0.05, steps=60),
    # moving window with the regularised and the MRT collision operators
    "window_regularised": dict(cfg=dict(moving_window=1, collision=wl.REG), gamma=20.0, emittance=0.1,
                               spread=0.01, steps=30),
    "window_mrt": dict(cfg=dict(moving_window=1, collision=wl.MRT, mrt_se=1.3, mrt_seps=0.6, mrt_sq=1.7,
                                mrt_spi=1.2), gamma=20.0, emittance=0.1, spread=0.01, steps=30),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_parity(name):
    c = CASES[name]
    cfg = wl.config(None, nz=130, nr=21, dz=0.05, dr=0.05, nb=0.4, sigma_z=0.35, sigma_r=0.25, zd0=4.0,
                    driver=wl.PARTICLES, max_particles=6000, storage=wl.F64, noise_amp=1e-3, seed=4,
                    tau=0.7, **c["cfg"])
    b = wl.bunch(cfg, 5000, gamma=c["gamma"], emittance=c["emittance"], energy_spread=c["spread"], seed=8)
    pert = wl.density_perturbation(cfg)
    print(f"[bunch fp64 parity] {name} 130x21, {c['steps']} steps, 5000 particles", flush=True)
    lat = lattice(cfg, b, pert)
    lat.step(c["steps"])
    st, k, s = lat.state()
    bg = lat.bunch()
    S, P = O.run(cfg, c["steps"], pert, bunch=b)
    assert (k, s) == (S.k, S.s)
    errs = comp_errors(st, oracle_state(S, P))
    assert errs.max() < TOL64, (errs.argmax(), errs.max())
    ref = S.bunch.numpy()
    assert np.array_equal(bg[6] == 0.0, ref[6] == 0.0)
    be = bunch_errors(bg, ref)
    print(name, "lost", int((ref[6] == 0.0).sum()), "bunch errors", be, flush=True)
    assert max(be) < 1e-10, be
    if name.startswith("slow_deflected"):
        assert 0 < int((ref[6] == 0.0).sum()) < 5000     # the loss path ran
    lat.close()


def test_call_splits_and_checks_agree():
    """Within one lbm_step call the push of a step and the move of the next run as one launch; a
    call boundary, a diagnostic check or a re-sort of the bunch splits them.  One call of 45 steps,
    45 calls of one step, calls of 13 + 32 steps with a check every 7 steps, and re-sorts every 4
    steps (with and without checks every 7) all give the oracle's state and bunch (FP64, 1e-10,
    bunch in the caller's order), with the deflected slow bunch (losses included)."""
    c = CASES["slow_deflected"]
    base = wl.config(None, nz=130, nr=21, dz=0.05, dr=0.05, nb=0.4, sigma_z=0.35, sigma_r=0.25, zd0=4.0,
                     driver=wl.PARTICLES, max_particles=6000, storage=wl.F64, noise_amp=1e-3, seed=4,
                     tau=0.7, **c["cfg"])
    b = wl.bunch(base, 5000, gamma=c["gamma"], emittance=c["emittance"], energy_spread=c["spread"], seed=8)
    pert = wl.density_perturbation(base)
    S, P = O.run(base, 45, pert, bunch=b)
    ref_state, ref_b = oracle_state(S, P), S.bunch.numpy()
    for label, cfg, calls in (("one call", base, [45]), ("single steps", base, [1] * 45),
                              ("checks", dict(base, check_every=7), [13, 32]),
                              ("re-sorts", dict(base, resort_every=4), [45]),
                              ("re-sorts every step", dict(base, resort_every=1), [45]),
                              ("re-sorts and checks", dict(base, resort_every=4, check_every=7), [13, 1, 31])):
        print(f"[bunch calls] {label}", flush=True)
        lat = lattice(cfg, b, pert)
        for n in calls:
            lat.step(n)
        st, k, s = lat.state()
        assert (k, s) == (S.k, S.s)
        assert comp_errors(st, ref_state).max() < TOL64, label
        bg = lat.bunch()
        assert np.array_equal(bg[6] == 0.0, ref_b[6] == 0.0), label
        assert max(bunch_errors(bg, ref_b)) < 1e-10, label
        lat.close()


def test_bunch_replaced_mid_run():
    """lbm_set_bunch(init_fields = 0) after 20 steps replaces a bunch near the window's front with
    one centred 3 k_p^-1 (60 cells) further back; 100 more steps match the oracle with the same swap
    (FP64, 1e-10).  The step reads and clears J_b only near the current bunch (its extent widened by
    c dt per step since it was taken), and that region grows over about 20 cells of the first
    bunch's last deposit within those steps: that current must not survive there."""
    cfg = wl.config(None, nz=130, nr=21, dz=0.05, dr=0.05, nb=0.4, sigma_z=0.35, sigma_r=0.25, zd0=5.0,
                    driver=wl.PARTICLES, max_particles=6000, storage=wl.F64, noise_amp=1e-3, seed=4,
                    tau=0.7, moving_window=1)
    a = wl.bunch(cfg, 5000, gamma=5000.0, emittance=0.05, energy_spread=1e-4, seed=8)
    b = wl.bunch(dict(cfg, zd0=2.0), 3000, gamma=5000.0, emittance=0.05, energy_spread=1e-4, seed=9)
    pert = wl.density_perturbation(cfg)
    S, P = O.run(cfg, 20, pert, bunch=a)
    b[2] += S.k * P.dt                                   # the second bunch's positions at t_19
    S.bunch = torch.as_tensor(b.copy(), dtype=torch.float64)
    for _ in range(100):
        S = O.step(S, P)
    print("[bunch swap] 20 + 100 steps", flush=True)
    lat = lattice(cfg, a, pert)
    lat.step(20)
    lat.set_bunch(b, False)
    lat.step(100)
    st, k, s = lat.state()
    assert (k, s) == (S.k, S.s)
    assert comp_errors(st, oracle_state(S, P)).max() < TOL64
    ref = S.bunch.numpy()
    bg = lat.bunch()
    assert np.array_equal(bg[6] == 0.0, ref[6] == 0.0)
    assert max(bunch_errors(bg, ref)) < 1e-10
    lat.close()


def test_checkpoint_resumes_particle_run():
    """lbm_save / lbm_load carry the bunch (its stored order after re-sorts, the caller's indices and
    the extent that bounds J_b): 13 steps with re-sorts every 4, a checkpoint in host and in device
    memory, and 32 more steps through another context (which held another bunch and had stepped,
    so that its J_b buffers hold current elsewhere) match the oracle's 45 steps (FP64, 1e-10, the
    deflected slow bunch with its losses).  The checkpoint is 24 + 60 n bytes longer than a
    rigid-driver one.  Checkpoints of the other driver, of more particles than the context holds or
    with a damaged index array are rejected and leave the context as it was."""
    from paper_2201_05473_amd import LBM_EINVAL, LbmError, Lattice, lbm_checkpoint_bytes
    c = CASES["slow_deflected"]
    cfg = wl.config(None, nz=130, nr=21, dz=0.05, dr=0.05, nb=0.4, sigma_z=0.35, sigma_r=0.25, zd0=4.0,
                    driver=wl.PARTICLES, max_particles=6000, storage=wl.F64, noise_amp=1e-3, seed=4,
                    tau=0.7, resort_every=4, **c["cfg"])
    b = wl.bunch(cfg, 5000, gamma=c["gamma"], emittance=c["emittance"], energy_spread=c["spread"], seed=8)
    other = wl.bunch(dict(cfg, zd0=2.0), 3000, gamma=5000.0, emittance=0.05, energy_spread=1e-4, seed=9)
    pert = wl.density_perturbation(cfg)
    S, P = O.run(cfg, 45, pert, bunch=b)
    ref_state, ref_b = oracle_state(S, P), S.bunch.numpy()
    print("[bunch checkpoint] 13 + 32 steps, re-sorts every 4", flush=True)
    lat = lattice(cfg, b, pert)
    lat.step(13)
    rigid = Lattice(dict(cfg, driver=wl.RIGID))
    assert lbm_checkpoint_bytes(lat.ctx) == lbm_checkpoint_bytes(rigid.ctx) + 24 + 60 * 5000
    for on_device in (False, True):
        ck = lat.save(on_device)
        res = lattice(cfg, other, pert)
        res.step(6)
        res.load(ck)
        res.step(32)
        st, k, s = res.state()
        assert (k, s) == (S.k, S.s)
        assert comp_errors(st, ref_state).max() < TOL64, on_device
        bg = res.bunch()
        assert np.array_equal(bg[6] == 0.0, ref_b[6] == 0.0), on_device
        assert max(bunch_errors(bg, ref_b)) < 1e-10, on_device
        res.close()
    ck = lat.save(False)
    bad_pid = ck.copy()
    pid = bad_pid[-4 * 5000:].view(np.int32)
    pid[0] = pid[1]
    small = lattice(dict(cfg, max_particles=4000), other, pert)
    small.step(3)
    before = small.state(), small.bunch()
    for target, buf in ((small, ck), (small, rigid.save(False)), (small, bad_pid), (rigid, ck)):
        with pytest.raises(LbmError) as ei:
            target.load(buf)
        assert ei.value.code == LBM_EINVAL
    with pytest.raises(LbmError) as ei:
        lattice(cfg, other, pert).load(bad_pid)
    assert ei.value.code == LBM_EINVAL
    after = small.state(), small.bunch()
    assert all(np.array_equal(x, y) for x, y in zip(before[0], after[0]))
    assert np.array_equal(before[1], after[1])
    small.step(1)
    for x in (lat, rigid, small):
        x.close()


@pytest.mark.parametrize("resort,m64,nt", [(0, 0, 0), (3, 0, 0), (3, 1, 0), (3, 0, 1)])
def test_fp32_particle_run(resort, m64, nt):
    """FP32 storage with the particle driver over 60 steps of the deflected slow bunch (losses
    included), with the default re-sort interval and with a re-sort every 3 steps, in FP32 and in
    FP64 arithmetic (fp64_math), and with non-temporal bunch accesses (bunch_streaming): the FP32
    tile deposit (shares summed within runs of lanes in FP32) and the J_b bound against the FP64
    oracle.  Moments and fields within 1e-5 of their group's scale, particle coordinates within
    1e-6 of theirs, and the same particles lost."""
    c = CASES["slow_deflected"]
    cfg = wl.config(None, nz=130, nr=21, dz=0.05, dr=0.05, nb=0.4, sigma_z=0.35, sigma_r=0.25, zd0=4.0,
                    driver=wl.PARTICLES, max_particles=6000, storage=wl.F32, noise_amp=1e-3, seed=4,
                    tau=0.7, resort_every=resort, fp64_math=m64, bunch_streaming=nt, **c["cfg"])
    b = wl.bunch(cfg, 5000, gamma=c["gamma"], emittance=c["emittance"], energy_spread=c["spread"], seed=8)
    pert = wl.density_perturbation(cfg)
    S, P = O.run(dict(cfg, storage=wl.F64, fp64_math=0), 60, pert, bunch=b)
    print(f"[bunch fp32] resort_every={resort} fp64_math={m64} bunch_streaming={nt}", flush=True)
    lat = lattice(cfg, b, pert)
    lat.step(60)
    st, k, s = lat.state()
    assert (k, s) == (S.k, S.s)
    errs = comp_errors(st, oracle_state(S, P))
    ref = S.bunch.numpy()
    bg = lat.bunch()
    be = bunch_errors(bg, ref)
    print("moments/fields", errs[27:].max(), "bunch", be, flush=True)
    assert errs[27:].max() < 1e-5, errs[27:]
    assert np.array_equal(bg[6] == 0.0, ref[6] == 0.0)
    assert max(be) < 1e-6, be
    lat.close()


def test_empty_bunch():
    """A particle-driven context with no particles (and one whose bunch was never set) evolves as
    the plasma with no driver: the oracle's state for an empty bunch, FP64 to 1e-10, over 12
    steps with two window shifts, also when resumed from a checkpoint (host and device memory)
    taken after 5 steps."""
    cfg = wl.config(None, nz=70, nr=9, dz=0.05, dr=0.05, driver=wl.PARTICLES, max_particles=10,
                    storage=wl.F64, noise_amp=1e-3, seed=3, moving_window=1, tau=0.7)
    pert = wl.density_perturbation(cfg)
    S, P = O.run(cfg, 12, pert, bunch=np.zeros((7, 0)))
    ref = oracle_state(S, P)
    from paper_2201_05473_amd import Lattice
    for set_empty in (True, False):
        print(f"[empty bunch] set_bunch(empty)={set_empty}", flush=True)
        lat = Lattice(cfg, pert)
        if set_empty:
            lat.set_bunch(np.zeros((7, 0)), True)
        lat.step(5)
        cks = [lat.save(False), lat.save(True)]
        lat.step(7)
        for x in [lat] + cks:
            if x is not lat:
                res = Lattice(cfg)
                res.load(x)
                res.step(7)
            else:
                res = lat
            st, k, s = res.state()
            assert (k, s) == (S.k, S.s)
            assert comp_errors(st, ref).max() < TOL64
            assert res.bunch().shape == (7, 0)
            res.close()


def test_initial_gauss_law_from_the_bunch():
    """Right after lbm_set_bunch the discrete Gauss residual (driver density from the deposited
    bunch) vanishes, and the initial field matches the oracle's."""
    cfg = wl.config("C2s", driver=wl.PARTICLES, max_particles=20000, storage=wl.F64)
    b = wl.bunch(cfg, 20000, seed=3)
    lat = lattice(cfg, b)
    d = lat.diagnostics()
    assert d["gauss_max"] < 1e-13, d
    st, _, _ = lat.state()
    S = O.initial_state(O.Params(cfg), None, None, b)
    assert comp_errors(st, oracle_state(S, O.Params(cfg))).max() < 1e-12
    lat.close()


def test_full_size_c2_single_step_with_paper_sized_bunch():
    """C2 at full size (2048 x 512) driven by a 200,000-particle bunch of the paper's shape
    (gamma = 5000): one step, FP64 to 1e-10 with the oracle (state and bunch), FP32, FP16N and
    FP16 moments and fields to 1e-6 (measured 1.0e-7 for all three)."""
    cfg = wl.config("C2", driver=wl.PARTICLES, max_particles=200000, storage=wl.F64)
    b = wl.bunch(cfg, 200000, gamma=5000.0, emittance=0.05, energy_spread=1e-4, seed=6)
    S, P = O.run(cfg, 1, bunch=b)
    ref = oracle_state(S, P)
    for storage, tol in ((wl.F64, TOL64), (wl.F32, 1e-6), (wl.F16N, 1e-6), (wl.F16, 1e-6)):
        print(f"[bunch full size] C2 storage={storage}", flush=True)
        lat = lattice(dict(cfg, storage=storage), b)
        lat.step(1)
        st, k, s = lat.state()
        errs = comp_errors(st, ref)
        if storage == wl.F64:
            assert errs.max() < tol, (errs.argmax(), errs.max())
            assert max(bunch_errors(lat.bunch(), S.bunch)) < 1e-10
        else:
            print(f"storage {storage}: moments/fields {errs[27:].max():.3g}", flush=True)
            assert errs[27:].max() < tol, errs[27:]
        lat.close()


def test_bunch_interface_errors():
    from paper_2201_05473_amd import LBM_EINVAL, LbmError, Lattice
    rigid = Lattice(wl.config(None, nz=64, nr=8))
    with pytest.raises(LbmError) as ei:
        rigid.set_bunch(np.zeros((7, 1)))
    assert ei.value.code == LBM_EINVAL
    rigid.close()
    cfg = wl.config(None, nz=64, nr=8, nb=0.3, zd0=2.0, sigma_z=0.3, sigma_r=0.2, driver=wl.PARTICLES,
                    max_particles=10)
    lat = Lattice(cfg)
    with pytest.raises(LbmError) as ei:
        lat.set_bunch(np.zeros((7, 11)))                 # over capacity
    assert ei.value.code == LBM_EINVAL
    b = wl.bunch(cfg, 10, seed=1)
    for bad in (np.nan, np.inf):
        nb = b.copy()
        nb[2, 3] = bad
        with pytest.raises(LbmError) as ei:
            lat.set_bunch(nb)                            # non-finite coordinate
        assert ei.value.code == LBM_EINVAL
    nb = b.copy()
    nb[6, 0] = -1.0
    with pytest.raises(LbmError) as ei:
        lat.set_bunch(nb)                                # negative weight
    assert ei.value.code == LBM_EINVAL
    lat.set_bunch(b)
    assert np.array_equal(lat.bunch(), b)
    lat.step(2)
    with pytest.raises(LbmError) as ei:
        lat.set_bunch(b, True)                           # initial field only at step 0
    assert ei.value.code == LBM_EINVAL
    lat.set_bunch(b, False)                              # resuming keeps the fields
    lat.close()
    fresh = Lattice(cfg)
    with pytest.raises(LbmError) as ei:
        fresh.adjoint(4, 2)                              # the adjoint covers the rigid driver
    assert ei.value.code == LBM_EINVAL
    fresh.close()
