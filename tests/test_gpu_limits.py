"""Edge cases of the grid size on the GPU path, through the C ABI.

Largest: a D2Q9 grid whose state copy is just under the 4 GiB that 32-bit
byte offsets address (8192 x 7000 nodes at 74 B each; 8192 x 6700 at 78 B
with the phi plane of the correction from data).  A droplet near the far
end of the node range must evolve to the same bits as the same droplet in a
small grid: a step reads a node's neighbourhood within 4 nodes, so after k
steps nothing beyond 4k nodes of the droplet has changed, and every node is
computed by the same arithmetic from the same inputs.

The same for D3Q19 (256 x 256 x 425 nodes at 154 B; 256 x 256 x 414 at 158
B with the phi plane), for the three-kernel and the fused step.

Smallest: 4 x 4 (and 5 x 4, 4 x 4 x 4) grids, where every tile shape is larger
than the grid and most of each tile lies outside it, against the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hip():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1110_5004_amd as P
    P.lib()
    return P


def droplet_case(nx, ny, centre, rf):
    """Periodic grid, droplet of radius 20 moving down at 0.03."""
    prm = W.base_params(W.D2Q9, nx, ny, 1, (0, 0, 0), sigma=0.01, remove_fa=rf)
    phi, u, p = W.droplet_fields(prm, centre, 20.0, impact_u=0.03)
    return W.Case(prm, phi, u, p)


def _largest(hip, rf):
    import torch
    # 74 B per node, 78 B with the phi plane of the correction from data
    big_n = (8192, 7000 if rf == 1 else 6700)
    steps = 12
    # the same fractional centre, so that both grids see bit-identical inputs
    cb = (4000.3, 6450.6)
    small = 256
    cs = (128.3, 128.6)
    sim = hip.Simulation([droplet_case(*big_n, cb, rf)])
    per_copy = sim.state_bytes()
    print(f"largest rf={rf}: {big_n[0]} x {big_n[1]}, {per_copy} B per state copy")
    assert 0.98 * 2**32 < per_copy < 2**32
    sim.step(steps)
    d = sim.diagnostics()
    m = sim.moments_device()
    x0, y0 = int(cb[0]) - 128, int(cb[1]) - 128
    assert y0 + small <= big_n[1] and x0 + small <= big_n[0]
    win = (slice(y0, y0 + small), slice(x0, x0 + small))
    phi_b = m["phi"].view(big_n[1], big_n[0])[win].cpu().numpy()
    u_b = m["u"].view(2, big_n[1], big_n[0])[(slice(None),) + win].cpu().numpy()
    p_b = m["p"].view(big_n[1], big_n[0])[win].cpu().numpy()
    del m
    sim.close()
    torch.cuda.empty_cache()
    ref = hip.Simulation([droplet_case(small, small, cs, rf)])
    ref.step(steps)
    r = ref.moments()
    ref.close()
    assert d["nonfinite"] == 0 and d["mass_drift_rel"] <= 1e-6
    assert np.array_equal(phi_b, r["phi"].reshape(small, small))
    assert np.array_equal(u_b, r["u"].reshape(2, small, small))
    assert np.array_equal(p_b, r["p"].reshape(small, small))


@pytest.mark.parametrize("rf", [1, 2])
def test_largest_copy_matches_small_grid(hip, rf):
    """A state copy just under 4 GiB (8192 x 7000 nodes; 8192 x 6700 with the
    phi plane), droplet at (4000.3, 6450.6), 12 steps: the window around it
    equals a 256 x 256 grid's run bit for bit."""
    _largest(hip, rf)


@pytest.mark.parametrize("dims,wall", [((4, 4, 1), (0, 0, 0)), ((4, 4, 1), (1, 1, 0)),
                                       ((5, 4, 1), (0, 1, 0)), ((4, 4, 4), (0, 0, 1))])
@pytest.mark.parametrize("rf", [0, 1])
def test_smallest_grids(hip, dims, wall, rf):
    nx, ny, nz = dims
    lat = W.D2Q9 if nz == 1 else W.D3Q19
    n = nx * ny * nz
    prm = W.base_params(lat, nx, ny, nz, wall, sigma=0.01, remove_fa=rf, width=2.0)
    x = np.tile(np.arange(nx, dtype=float), ny * nz)
    y = np.repeat(np.tile(np.arange(ny, dtype=float), nz), nx)
    phi = 0.5 + 0.3 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny)
    rng = np.random.default_rng(n + rf)
    dim = 2 if nz == 1 else 3
    u = rng.normal(0, 2e-3, (dim, n))
    case = W.Case(prm, phi, u, np.zeros(n))
    steps = 50
    ref = O.Sim(case.params, case.phi0, case.u0, case.p0)
    ref.step(steps)
    want = ref.fields()
    first = None
    for v in range(len(hip.variants(lat))):
        sim = hip.Simulation([case])
        sim.set_launch(v, 0, 16)
        sim.step(steps)
        if first is None:
            got = sim.moments()
            dphi = float(np.abs(got["phi"].astype(np.float64) - want["phi"]).max())
            du = float(np.linalg.norm(got["u"].astype(np.float64) - want["u"]) /
                       np.linalg.norm(want["u"]))
            print(f"smallest {dims} {wall} rf={rf}: max|dphi|={dphi:.2e} relL2(u)={du:.2e}")
            assert dphi <= 1e-5 and du <= 1e-4
            first = sim.get_state()
        else:
            assert np.array_equal(sim.get_state(), first), f"variant {v} differs"
        sim.close()


def _largest_3d(hip, rf, variant):
    import torch
    # 154 B per node, 158 with the phi plane of the correction from data
    nz = 425 if rf != 2 else 414
    big = (256, 256, nz)
    steps = 8
    # exactly representable fractions: both grids start from the same bits;
    # far along z, so the window holds the highest node indices
    cb = (128.25, 128.5, nz - 70 + 0.25)
    n_s = 128
    cs = (64.25, 64.5, 64.25)
    prm = W.base_params(W.D3Q19, *big, (0, 0, 0), sigma=0.01, remove_fa=rf)
    phi, u, p = W.droplet_fields(prm, cb, 10.0, impact_u=0.03)
    sim = hip.Simulation([W.Case(prm, phi, u, p)])
    del phi, u, p
    per_copy = sim.state_bytes()
    print(f"largest d3q19 rf={rf} variant {variant}: {big}, {per_copy} B per state copy")
    assert 0.98 * 2**32 < per_copy < 2**32
    sim.set_launch(variant, 0, 16)
    sim.step(steps)
    d = sim.diagnostics()
    m = sim.moments_device()
    x0, y0, z0 = (int(cb[k]) - n_s // 2 for k in range(3))
    assert z0 + n_s <= nz
    win = (slice(z0, z0 + n_s), slice(y0, y0 + n_s), slice(x0, x0 + n_s))
    phi_b = m["phi"].view(nz, 256, 256)[win].cpu().numpy()
    u_b = m["u"].view(3, nz, 256, 256)[(slice(None),) + win].cpu().numpy()
    p_b = m["p"].view(nz, 256, 256)[win].cpu().numpy()
    del m
    sim.close()
    torch.cuda.empty_cache()
    prm_s = W.base_params(W.D3Q19, n_s, n_s, n_s, (0, 0, 0), sigma=0.01, remove_fa=rf)
    ref = hip.Simulation([W.Case(prm_s, *W.droplet_fields(prm_s, cs, 10.0, impact_u=0.03))])
    ref.set_launch(variant, 0, 16)
    ref.step(steps)
    r = ref.moments()
    ref.close()
    assert d["nonfinite"] == 0 and d["mass_drift_rel"] <= 1e-6
    # a step reads within 4 nodes, so after k steps a node within 63 - 4k of
    # the centre depends only on initial values within 63 of it, which the two
    # grids share (the small grid wraps at 64); farther out the droplet's FP32
    # tails (~1e-32) meet the small grid's periodic image
    h = 63 - 4 * steps
    core = (slice(n_s // 2 - h, n_s // 2 + h + 1),) * 3
    assert np.array_equal(phi_b[core], r["phi"].reshape(n_s, n_s, n_s)[core])
    assert np.array_equal(u_b[(slice(None),) + core],
                          r["u"].reshape(3, n_s, n_s, n_s)[(slice(None),) + core])
    assert np.array_equal(p_b[core], r["p"].reshape(n_s, n_s, n_s)[core])


@pytest.mark.parametrize("rf,variant", [(1, 0), (1, 10), (0, 12), (2, 1), (2, 9)])
def test_largest_copy_matches_small_grid_d3q19(hip, rf, variant):
    """D3Q19 state copies just under 4 GiB (256 x 256 x 425 nodes at 154 B;
    256 x 256 x 414 at 158 B with the phi plane), the three-kernel and the
    fused step (also the fused step without the Eq. 5 term), droplet far
    along z, 8 steps: the 63^3 core of the window around it (all nodes whose
    8-step dependency cone the two grids share) equals a 128^3 grid's run
    bit for bit."""
    _largest_3d(hip, rf, variant)


@pytest.mark.parametrize("rf", [1, 0])
def test_largest_copy_fp16_fused_equals_three_kernel(hip, rf):
    """A 16-bit D3Q19 state copy just under 4 GiB (256 x 256 x 840 nodes at
    78 B), droplet far along z, 6 steps: the fused 16-bit step (k3_march,
    variant 12) equals the three-kernel step (variant 1) bit for bit over the
    whole grid, so its 32-bit buffer offsets hold up to the end of a copy.
    (The stochastic rounding draws from the node index, so a smaller grid's
    run is not a bitwise reference here; the other form on the same grid
    is.)"""
    import torch
    nz = 840
    prm = W.base_params(W.D3Q19, 256, 256, nz, (0, 0, 1), sigma=0.01, remove_fa=rf)
    phi, u, p = W.droplet_fields(prm, (128.25, 128.5, nz - 40.25), 10.0, impact_u=0.03)
    states = []
    for variant in (1, 12):
        sim = hip.Simulation([W.Case(prm, phi, u, p)], storage="fp16")
        per_copy = sim.state_bytes()
        assert 0.98 * 2**32 < per_copy < 2**32
        sim.set_launch(variant, 0, 16)
        sim.step(6)
        d = sim.diagnostics()
        assert d["nonfinite"] == 0 and d["mass_drift_rel"] <= 1e-6
        states.append(torch.from_numpy(sim.get_state()))
        sim.close()
        torch.cuda.empty_cache()
    assert torch.equal(states[0], states[1])
