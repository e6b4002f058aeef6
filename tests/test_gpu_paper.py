"""The paper's two experiments at their own sizes, on the GPU path: the
falling-droplet series (centroid, spread radius) of both models against the
FP64 oracle, the paper's qualitative claims about the two models, and the
splash test's Reynolds-number dependence of the model difference.

The paper's own numbers (Fig. 5: a 4.1 l.u. spread-radius difference at
t = 1.9e4) depend on the exact original model of its Ref. [9], which the paper
does not print; only the signs are compared with the paper ("parity unpinned"
for the magnitudes, which are printed)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "paper_falling150x450_oracle.npz")


@pytest.fixture(scope="module")
def hip():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1110_5004_amd as P
    P.lib()
    return P


def test_spread_radius_definition(hip):
    """The GPU diagnostic applies the oracle's definition to the GPU field
    (same crossings, same interpolation), and agrees with the oracle's value
    on the oracle's own field after 300 steps."""
    case = W.paper_falling(remove_fa=1)
    dims = (case.params["nx"], case.params["ny"])
    sim = hip.Simulation([case])
    sim.step(300)
    got = sim.spread_radius()
    phi_gpu = sim.moments()["phi"].astype(np.float64)
    assert abs(got - O.spread_radius(phi_gpu, dims)) < 1e-9
    assert abs(sim.spread_radius(level=0.3) - O.spread_radius(phi_gpu, dims, 0.3)) < 1e-9
    ref = O.Sim(case.params, case.phi0, case.u0, case.p0)
    ref.step(300)
    want = O.spread_radius(ref.fields()["phi"], dims)
    print(f"spread radius after 300 steps: gpu {got:.6f} oracle {want:.6f}")
    assert abs(got - want) < 1e-3
    sim.close()


def _series(hip, remove_fa, steps, every):
    case = W.paper_falling(remove_fa=remove_fa)
    sim = hip.Simulation([case])
    out = dict(t=[], cy=[], spread=[], mass=[])
    for k in range(steps // every + 1):
        if k:
            sim.step(every)
        d = sim.diagnostics()
        out["t"].append(k * every)
        out["cy"].append(d["centroid"][1])
        out["spread"].append(sim.spread_radius())
        out["mass"].append(d["mass"])
    sim.close()
    return {k: np.array(v) for k, v in out.items()}


def test_paper_falling_both_models(hip):
    """20k steps of the falling droplet (150 x 450, Eo = 17), original and
    corrected model: centroid and spread radius within 0.05 l.u. of the
    oracle's at every 500 steps, mass conserved; then the paper's claims
    (its Fig. 4 and 5 discussion): the original model falls faster (lower
    centroid) and spreads less, with the difference growing after t = 1e4."""
    ref = np.load(GOLDEN)
    runs = {m: _series(hip, m, 20000, 500) for m in (0, 1)}
    for m in (0, 1):
        r = runs[m]
        assert np.array_equal(r["t"], ref["t"])
        dy = np.abs(r["cy"] - ref[f"centroid_y_{m}"]).max()
        ds = np.abs(r["spread"] - ref[f"spread_{m}"]).max()
        drift = np.abs(r["mass"] - r["mass"][0]).max() / r["mass"][0]
        print(f"remove_fa={m}: max|d centroid_y|={dy:.4f} max|d spread|={ds:.4f} "
              f"mass drift={drift:.2e}")
        assert dy < 0.05 and ds < 0.05 and drift < 1e-6
    k = int(np.searchsorted(runs[0]["t"], 19000))
    dcy = runs[0]["cy"][k] - runs[1]["cy"][k]
    dsp = runs[0]["spread"][k] - runs[1]["spread"][k]
    rcy = ref["centroid_y_0"][k] - ref["centroid_y_1"][k]
    rsp = ref["spread_0"][k] - ref["spread_1"][k]
    print(f"t=1.9e4, original - corrected: centroid {dcy:+.3f} (oracle {rcy:+.3f}), "
          f"spread radius {dsp:+.3f} (oracle {rsp:+.3f}; the paper reports 4.1 in "
          f"magnitude for its original model)")
    assert dcy < 0 and dsp < 0                       # falls faster, spreads less
    assert abs(dcy - rcy) < 0.3 * abs(rcy) and abs(dsp - rsp) < 0.3 * abs(rsp)
    early = int(np.searchsorted(runs[0]["t"], 5000))
    assert abs(runs[0]["cy"][early] - runs[1]["cy"][early]) < 0.1 * abs(dcy)


def test_paper_splash_re48(hip):
    """The splash test (300 x 150, We = 960, Re = 48): the GPU fields of both
    models against the oracle at t* = tU/D = 1, and the paper's observation
    for Re = 48 (its Fig. 1) that the two models give nearly the same
    result: the mean |phi_original - phi_corrected| stays below 1e-3 through
    t* = 2 while the interface moves by tens of cells."""
    fields, refs = [], []
    for m in (0, 1):
        case = W.paper_splash(re=48, remove_fa=m)
        t1 = int(round(case.meta["t_unit"]))
        sim = hip.Simulation([case])
        sim.step(t1)
        got = sim.moments()
        ref = O.Sim(case.params, case.phi0, case.u0, case.p0)
        ref.step(t1)
        want = ref.fields()
        dphi = float(np.abs(got["phi"] - want["phi"]).max())
        du = float(np.linalg.norm(got["u"] - want["u"]) / np.linalg.norm(want["u"]))
        print(f"paper splash Re 48 remove_fa={m}, t*=1: max|dphi|={dphi:.2e} relL2(u)={du:.2e}")
        # an impact that deforms the interface by tens of cells over 1500
        # steps; FP32 rounding accumulates to a few 1e-4 in phi here (the
        # 1e-5 bound of the 1000-step resting droplet does not transfer)
        assert dphi < 1e-3 and du < 1e-3
        sim.step(t1)
        assert sim.diagnostics()["nonfinite"] == 0
        fields.append(sim.moments()["phi"].astype(np.float64))
        sim.close()
    diff = float(np.abs(fields[0] - fields[1]).mean())
    moved = float(np.abs(fields[0] - W.paper_splash(re=48).phi0).mean())
    print(f"t*=2: mean |phi_orig - phi_corr| = {diff:.2e} (mean change since t=0: {moved:.2e})")
    assert diff < 1e-3 and moved > 20 * diff


def test_fa_discrete_against_oracle_and_eq5(hip):
    """F_a of Eq. 12 from discrete data, -u [(rho^n - rho^(n-1)) + div(rho u)],
    on the falling droplet (original model, t = 4000 -> 4001): GPU against
    the oracle's definition on the oracle's fields, and the comparison the
    paper's Eq. 5 reading rests on -- d_t rho + div(rho u) ~ drho theta_M
    lap mu, so the discrete F_a should follow the F_a the step evaluates
    (printed: relative L2 difference and the cosine between the two fields)."""
    import torch
    case = W.paper_falling(remove_fa=0)
    steps = 4000
    sim = hip.Simulation([case])
    sim.step(steps)
    phi_prev = sim.moments_device()["phi"].clone()
    sim.step(1)
    got = sim.fa_discrete(phi_prev).cpu().numpy().astype(np.float64)
    eq5 = sim.moments()["fa"].astype(np.float64)
    sim.close()
    ref = O.Sim(case.params, case.phi0, case.u0, case.p0)
    ref.step(steps)
    prev = ref.fields()["phi"]
    ref.step(1)
    fl = ref.fields()
    want = O.fa_discrete(case.params, prev, fl["phi"], fl["u"])
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    rel5 = np.linalg.norm(got - eq5) / np.linalg.norm(eq5)
    cos = float((got * eq5).sum() / (np.linalg.norm(got) * np.linalg.norm(eq5)))
    print(f"discrete F_a: GPU vs oracle rel-L2 {rel:.2e}; against the Eq. 5 F_a of the step: "
          f"rel-L2 {rel5:.2e}, cosine {cos:.3f}; max|F| {np.abs(want).max():.2e}")
    assert rel < 5e-2
    assert np.isfinite(rel5) and np.isfinite(cos)


@pytest.mark.parametrize("lattice,dims,wall,well", [
    (W.D2Q9, (70, 45, 1), (0, 1, 0), 0), (W.D2Q9, (37, 53, 1), (1, 1, 0), 1),
    (W.D3Q19, (20, 18, 16), (0, 0, 1), 0), (W.D3Q19, (17, 15, 19), (1, 1, 1), 1)])
def test_fa_leelin_against_oracle(hip, lattice, dims, wall, well):
    """F_a in Lee and Lin's form, -u div[lambda (grad P - grad p)] (Eq. 11 in
    Eq. 12), on a moving droplet with gravity and walls after 150 steps of the
    original model: GPU on its fields against the oracle's definition on the
    oracle's fields, both wells, both lattices, ragged sizes."""
    nx, ny, nz = dims
    ps = 0.8
    prm = W.base_params(lattice, nx, ny, nz, wall, sigma=0.01, gravity=2e-5, remove_fa=0,
                        tau_g=0.7, mu_ratio=4.0, theta_m=0.1 * ((2 * ps) ** 2 if well else 1.0),
                        well=well, phi_star=ps)
    dim = 2 if lattice == W.D2Q9 else 3
    rng = np.random.default_rng(nx * ny * nz)
    centre = (nx * 0.45, ny * 0.55, nz * 0.5)[:dim]
    phi, u, p = W.droplet_fields(prm, centre, min(dims[:dim]) * 0.28, impact_u=0.03,
                                 noise=rng.normal(0, 1e-3, (dim, nx * ny * nz)))
    case = W.Case(prm, phi, u, p)
    sim = hip.Simulation([case])
    sim.step(150)
    got = sim.fa_leelin().cpu().numpy().astype(np.float64)
    sim.close()
    ref = O.Sim(case.params, case.phi0, case.u0, case.p0)
    ref.step(150)
    fl = ref.fields()
    want = O.fa_leelin(case.params, fl["phi"], fl["u"], fl["p"])
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    eq5 = fl["fa"]
    cos = float((want * eq5).sum() / (np.linalg.norm(want) * np.linalg.norm(eq5)))
    print(f"Lee-Lin F_a {dims} {wall} well={well}: GPU vs oracle rel-L2 {rel:.2e}, "
          f"max|F| {np.abs(want).max():.2e}; oracle: |F_LL| / |F_Eq5| "
          f"{np.linalg.norm(want) / np.linalg.norm(eq5):.3f}, cosine {cos:.3f}")
    # measured 3e-6 .. 1.3e-5: the FP32 fields' differences, through two
    # derivatives of P - p
    assert rel < 1e-3
    assert np.abs(want).max() > 0.0
