"""GPU parity of remove_fa = 2 against the FP64 oracle, through the C ABI.
In this mode the correction -F_a = D u uses a rate taken from the data:
D = (rho^n - rho^(n-1)) + div(rho u_o), with u_o the uncorrected velocity
(Eq. 12 with a backward difference in time), instead of Eq. 5.  The kernel
keeps phi^(n-1) in one more float plane of each state copy."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

PHI_TOL = 1e-5
U_TOL = 1e-4


@pytest.fixture(scope="module")
def hip():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1110_5004_amd as P
    P.lib()
    return P


def oracle_run(case, steps):
    s = O.Sim(case.params, case.phi0, case.u0, case.p0)
    s.step(steps)
    return s


def errors(got, want):
    dphi = float(np.abs(got["phi"].astype(np.float64) - want["phi"]).max())
    du = float(np.linalg.norm(got["u"].astype(np.float64) - want["u"]) /
               np.linalg.norm(want["u"]))
    return dphi, du


def moving_droplet(nx, ny, wall, seed, rf=2):
    prm = W.base_params(W.D2Q9, nx, ny, 1, wall, sigma=0.01, gravity=2e-5, remove_fa=rf,
                        tau_g=0.7, mu_ratio=4.0)
    rng = np.random.default_rng(seed)
    phi, u, p = W.droplet_fields(prm, (nx * 0.45, ny * 0.55), min(nx, ny) * 0.28,
                                 impact_u=0.03, noise=rng.normal(0, 1e-3, (2, nx * ny)))
    return W.Case(prm, phi, u, p)


def test_droplet128_1000_steps(hip):
    """The resting 128^2 droplet (R = 25, ratio 10, velocity noise), 1000
    steps, at the FP32 bounds."""
    case = W.stationary_droplet(seed=0, remove_fa=2)
    sim = hip.Simulation([case])
    sim.step(1000)
    dphi, du = errors(sim.moments(), oracle_run(case, 1000).fields())
    print(f"correction from data, droplet128: max|dphi|={dphi:.2e} relL2(u)={du:.2e}")
    assert dphi <= PHI_TOL and du <= U_TOL


def test_translating_droplet128_drift_as_eq5(hip):
    """The same droplet translating at (0.02, -0.01) for 1000 steps, under the
    Eq. 5 correction and the correction from data.  A moving interface turns
    the FP32 velocity difference (~5e-5 relative) into a displacement that
    grows with time: |grad phi| <= 1/W = 0.25 times ~1e-3 l.u. gives the
    measured max|dphi| ~1.6e-4 for both.  The correction from data must add
    no drift of its own."""
    res = {}
    for rf in (1, 2):
        c = W.stationary_droplet(seed=0, remove_fa=rf)
        u0 = c.u0.copy()
        u0[0] += 0.02
        u0[1] -= 0.01
        case = W.Case(c.params, c.phi0, u0, c.p0)
        sim = hip.Simulation([case])
        sim.step(1000)
        res[rf] = errors(sim.moments(), oracle_run(case, 1000).fields())
        sim.close()
    print(f"translating droplet128: Eq. 5 max|dphi|={res[1][0]:.2e} relL2(u)={res[1][1]:.2e}; "
          f"from data max|dphi|={res[2][0]:.2e} relL2(u)={res[2][1]:.2e}")
    for rf in (1, 2):
        assert res[rf][1] <= U_TOL and res[rf][0] <= 4e-4
    assert res[2][0] <= 1.2 * res[1][0] and res[2][1] <= 1.2 * res[1][1]


@pytest.mark.parametrize("shape,wall", [((70, 45), (0, 1, 0)), ((37, 53), (1, 1, 0)),
                                        ((66, 18), (0, 0, 0))])
def test_ragged_every_variant(hip, shape, wall):
    """Moving droplet with gravity and walls, ragged tiles, 300 steps; every
    launch variant, full-grid and persistent, gives the same bits."""
    case = moving_droplet(shape[0], shape[1], wall, seed=shape[0])
    first = None
    for variant in range(len(hip.variants())):
        for grid in (0, 8):
            sim = hip.Simulation([case])
            sim.set_launch(variant, grid, 16)
            sim.step(300)
            if first is None:
                want = oracle_run(case, 300).fields()
                dphi, du = errors(sim.moments(), want)
                print(f"correction from data {shape} {wall}: max|dphi|={dphi:.2e} "
                      f"relL2(u)={du:.2e}")
                assert dphi <= PHI_TOL and du <= U_TOL
                first = sim.get_state()
            else:
                assert np.array_equal(sim.get_state(), first), \
                    f"variant {variant} grid {grid} differs"
            sim.close()


def test_first_steps_and_dump(hip):
    """The first step (phi^(n-1) = phi0, only the divergence acts) and the
    field dump after 1, 2 and 7 steps: phi, u, p, mu and the Eq. 5 F_a."""
    case = moving_droplet(64, 48, (0, 1, 0), seed=5)
    sim = hip.Simulation([case])
    ref = O.Sim(case.params, case.phi0, case.u0, case.p0)
    for steps in (0, 1, 1, 5):
        if steps:
            sim.step(steps)
            ref.step(steps)
        got, want = sim.moments(), ref.fields()
        dphi, du = errors(got, want)
        assert dphi <= 1e-6 and du <= 1e-5, (sim.time, dphi, du)
        assert np.abs(got["p"] - want["p"]).max() <= 1e-4 * np.abs(want["p"]).max()
        assert np.abs(got["mu"] - want["mu"]).max() <= 1e-4 * np.abs(want["mu"]).max()
        assert np.abs(got["fa"] - want["fa"]).max() <= 2e-3 * np.abs(want["fa"]).max()


def test_checkpoint_resume_bitwise(hip):
    """The state bytes include the phi plane: 200 steps = 90 + save + load +
    110, to the last bit."""
    case = moving_droplet(64, 64, (0, 0, 0), seed=9)
    a = hip.Simulation([case])
    a.step(200)
    b = hip.Simulation([case])
    b.step(90)
    st = b.get_state()
    b.close()
    c = hip.Simulation([case])
    c.set_state(st, step=90)
    c.step(110)
    assert np.array_equal(a.get_state(), c.get_state())


def test_fixed_point_bitwise(hip):
    n = 32
    prm = W.base_params(W.D2Q9, n, n, 1, (0, 1, 0), sigma=0.01, remove_fa=2)
    for phi in (0.0, 1.0):
        sim = hip.Simulation([W.Case(prm, np.full(n * n, phi), np.zeros((2, n * n)),
                                     np.zeros(n * n))])
        s0 = sim.get_state()
        sim.step(7)
        assert np.array_equal(sim.get_state(), s0)


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_16bit_storage(hip, storage):
    case = moving_droplet(96, 64, (0, 1, 0), seed=13)
    sim = hip.Simulation([case], storage=storage)
    sim.step(300)
    got = sim.moments()
    d = sim.diagnostics()
    want = oracle_run(case, 300).fields()
    dphi, du = errors(got, want)
    print(f"correction from data {storage}: max|dphi|={dphi:.2e} relL2(u)={du:.2e} "
          f"drift {d['mass_drift_rel']:.2e}")
    assert d["nonfinite"] == 0 and d["mass_drift_rel"] <= 1e-5
    # measured 1.2e-4 / 3.2e-4 (FP16) and 1.0e-3 / 2.6e-3 (BF16)
    assert dphi <= (1e-3 if storage == "fp16" else 1e-2)
    assert du <= (1e-3 if storage == "fp16" else 1e-2)


def test_three_models_on_the_falling_droplet(hip):
    """The paper's falling droplet (150 x 450, Eo = 17) to t = 1.9e4 under the
    original model, the Eq. 5 correction and the correction from data: the
    GPU centroid and spread radius of each, against the oracle at t = 500
    (printed at 1.9e4: how far the data-based correction moves the result
    from the Eq. 5 one)."""
    res = {}
    for rf in (0, 1, 2):
        case = W.paper_falling(remove_fa=rf)
        sim = hip.Simulation([case])
        sim.step(500)
        if rf == 2:
            ref = oracle_run(case, 500).fields()
            dphi, du = errors(sim.moments(), ref)
            assert dphi <= PHI_TOL and du <= U_TOL, (dphi, du)
        sim.step(18500)
        d = sim.diagnostics()
        assert d["nonfinite"] == 0
        res[rf] = (d["centroid"][1], sim.spread_radius())
        sim.close()
    print("falling droplet t=1.9e4 (centroid y, spread radius): original "
          f"{res[0][0]:.3f} {res[0][1]:.3f}; Eq. 5 correction {res[1][0]:.3f} {res[1][1]:.3f}; "
          f"correction from data {res[2][0]:.3f} {res[2][1]:.3f}")


def droplet3d(dims, wall, seed):
    nx, ny, nz = dims
    prm = W.base_params(W.D3Q19, nx, ny, nz, wall, sigma=0.01, gravity=2e-5, remove_fa=2,
                        tau_g=0.7, mu_ratio=4.0)
    rng = np.random.default_rng(seed)
    phi, u, p = W.droplet_fields(prm, (nx * 0.45, ny * 0.5, nz * 0.55), min(dims) * 0.3,
                                 impact_u=0.02, noise=rng.normal(0, 1e-3, (3, nx * ny * nz)))
    return W.Case(prm, phi, u, p)


@pytest.mark.parametrize("dims,wall", [((20, 18, 16), (0, 0, 1)), ((17, 21, 19), (1, 1, 1))])
def test_d3q19_parity_every_variant(hip, dims, wall):
    """D3Q19, moving droplet with gravity and walls, 120 steps, at the FP32
    bounds; every fields-tile shape gives the same bits."""
    case = droplet3d(dims, wall, seed=sum(dims))
    sim = hip.Simulation([case])
    sim.step(120)
    dphi, du = errors(sim.moments(), oracle_run(case, 120).fields())
    print(f"correction from data d3q19 {dims} {wall}: max|dphi|={dphi:.2e} relL2(u)={du:.2e}")
    assert dphi <= PHI_TOL and du <= U_TOL
    first = sim.get_state()
    sim.close()
    for variant in range(1, len(hip.variants(hip.D3Q19))):
        other = hip.Simulation([case])
        other.set_launch(variant, 0, 16)
        other.step(120)
        assert np.array_equal(other.get_state(), first), f"variant {variant} differs"
        other.close()


def test_d3q19_first_steps_and_dump(hip):
    """D3Q19: dumps at steps 0, 1, 2 and 7 (phi^(n-1) = phi0 at the first),
    and a checkpoint that carries the phi plane."""
    case = droplet3d((16, 14, 12), (0, 1, 1), seed=2)
    sim = hip.Simulation([case])
    ref = O.Sim(case.params, case.phi0, case.u0, case.p0)
    for steps in (0, 1, 1, 5):
        if steps:
            sim.step(steps)
            ref.step(steps)
        got, want = sim.moments(), ref.fields()
        dphi, du = errors(got, want)
        assert dphi <= 1e-6 and du <= 1e-5, (sim.time, dphi, du)
        assert np.abs(got["mu"] - want["mu"]).max() <= 1e-4 * np.abs(want["mu"]).max()
        assert np.abs(got["fa"] - want["fa"]).max() <= 2e-3 * np.abs(want["fa"]).max()
    st = sim.get_state()
    sim.step(20)
    other = hip.Simulation([case])
    other.set_state(st, step=7)
    other.step(20)
    assert np.array_equal(other.get_state(), sim.get_state())
