"""FP64 diagnostics on the GPU (lbm_field_diagnostics, and lbm_diagnostics
which runs the same kernels on a case's own fields) against the oracle's
definition of them (orc_field_diag), on the same float32 fields.

The GPU sums in a fixed tree order and the oracle left to right, so sums
agree to rounding (relative 1e-12 with the magnitudes here); |u|max and
the non-finite count are exact."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

KEYS = ("mass", "wsum", "momentum", "centroid", "centroid_vel", "second_moment")


@pytest.fixture(scope="module")
def hip():
    import torch
    assert torch.cuda.is_available()
    import paper_1110_5004_amd as P
    return P


def droplet_fields(dims, seed, phi_g=0.0, phi_l=1.0, radius_frac=0.3):
    """A tanh droplet off the grid centre with a random velocity field."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    axes = np.meshgrid(*[np.arange(d, dtype=np.float64) for d in reversed(dims)], indexing="ij")
    pos = [a.ravel() for a in reversed(axes)]  # x fastest
    centre = [0.37 * d + 1.3 for d in dims]
    r = np.sqrt(sum((p - c) ** 2 for p, c in zip(pos, centre)))
    s = 0.5 + 0.5 * np.tanh(2.0 * (radius_frac * min(dims) - r) / 4.0)
    phi = (phi_g + (phi_l - phi_g) * s + 1e-3 * rng.standard_normal(n)).astype(np.float32)
    u = (0.02 * rng.standard_normal((len(dims), n))).astype(np.float32)
    return phi, u


def compare(d_gpu, ref, dim):
    for k in KEYS:
        g = np.atleast_1d(d_gpu[k])[:dim] if np.ndim(ref[k]) else d_gpu[k]
        r = np.atleast_1d(ref[k])[:dim] if np.ndim(ref[k]) else ref[k]
        assert np.allclose(g, r, rtol=1e-12, atol=1e-12 * max(1.0, abs(ref["mass"]))), (k, g, r)
    assert d_gpu["umax"] == pytest.approx(ref["umax"], rel=1e-15)
    assert d_gpu["nonfinite"] == ref["nonfinite"]


def slots_dict(s):
    s = np.asarray(s, dtype=np.float64)
    return dict(mass=s[0], momentum=s[1:4], wsum=s[4], centroid=s[5:8], centroid_vel=s[8:11],
                second_moment=s[11:14], umax=s[14], nonfinite=int(s[15]))


@pytest.mark.parametrize("dims,well", [((37, 29, 11), 0), ((64, 48), 0), ((3, 5, 7), 1),
                                       ((1, 1), 0), ((256, 256, 128), 0)])
def test_field_diagnostics_vs_oracle(hip, dims, well):
    import torch
    phi_g, phi_l = (-0.5, 0.5) if well else (0.0, 1.0)
    phi, u = droplet_fields(dims, seed=sum(dims), phi_g=phi_g, phi_l=phi_l)
    ref = O.field_diag(phi.astype(np.float64), u.astype(np.float64), dims, phi_g, phi_l, 0.1, 1.0)
    out = hip.field_diagnostics(torch.from_numpy(phi).cuda(), torch.from_numpy(u).cuda(), dims,
                                phi_g, phi_l, 0.1, 1.0)
    torch.cuda.synchronize()
    s = out.cpu().numpy()
    compare(slots_dict(s), ref, len(dims))
    assert np.all(s[1 + len(dims):4] == 0.0) and np.all(s[5 + len(dims):8] == 0.0)
    # fixed reduction order: a second call gives the same bits
    again = hip.field_diagnostics(torch.from_numpy(phi).cuda(), torch.from_numpy(u).cuda(), dims,
                                  phi_g, phi_l, 0.1, 1.0)
    assert np.array_equal(again.cpu().numpy(), s)


def test_field_diagnostics_nonfinite_and_empty_weight(hip):
    import torch
    dims = (40, 30)
    phi = np.zeros(1200, dtype=np.float32)  # all gas: no weight
    u = np.zeros((2, 1200), dtype=np.float32)
    u[0, 17] = np.inf
    u[1, 1100] = np.nan
    run = lambda ph: hip.field_diagnostics(torch.from_numpy(ph).cuda(), torch.from_numpy(u).cuda(),
                                           dims, 0.0, 1.0, 0.1, 1.0).cpu().numpy()
    out = run(phi)
    assert out[15] == 2.0
    assert out[4] == 0.0 and np.all(out[5:14] == 0.0)
    phi[5] = np.nan  # a non-finite phi is counted once with its node
    u[:, 17] = 0.0
    assert run(phi)[15] == 2.0


def test_handle_diagnostics_vs_oracle(hip):
    """lbm_diagnostics of a moving droplet against orc_field_diag of the
    fields lbm_moments returns, and the centred second moment against the
    oracle simulation's own."""
    case = W.stationary_droplet(seed=5, n=96, radius=20.0, centre_jitter=3.0)
    sim = hip.Simulation([case], storage="fp32")
    sim.step(20)
    m = sim.moments()
    d = sim.diagnostics()
    sim.close()
    ref = O.field_diag(m["phi"].astype(np.float64), m["u"].astype(np.float64), (96, 96), 0.0, 1.0,
                       case.params["rho_g"], case.params["rho_l"])
    compare(d, ref, 2)
    orc = O.Sim(case.params, case.phi0, case.u0, case.p0)
    orc.step(20)
    od = orc.diag()
    assert np.allclose(d["second_moment"][:2], od["second_moment"][:2], rtol=1e-5)
