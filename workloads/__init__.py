"""Seeded synthetic workloads: case parameters and initial fields.

This module is the only code shared by the HIP path and the CPU oracle.  It
holds none of the method's arithmetic: it draws the physical parameters and
builds the FP64 initial fields phi0, u0, p0 (droplet and film tanh profiles,
velocity noise, the Laplace pressure jump of a resting droplet).  Each side
derives beta, kappa, relaxation rates and equilibria on its own.

The paper publishes no input data.  Its two experiments (droplet splash on a
thin film, Fig. 1-3; falling droplet, Fig. 4-5) shape these generators; the
grids, radii and physical numbers of the benchmark workloads are listed in
WORKLOADS.  Draw order with numpy.random.default_rng(seed) (PCG64) is fixed:
scalar jitters first, in the order each builder lists them, then per-node
noise as one normal array of shape (dim, N) (all x components, then y, then z;
nodes in index order x + nx*(y + ny*z)).
"""
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

D2Q9, D3Q19 = 0, 1
PERIODIC, WALL = 0, 1


@dataclass
class Case:
    """One simulation case: parameters (plain dict) + FP64 initial fields."""
    params: Dict
    phi0: np.ndarray            # [N]
    u0: np.ndarray              # [dim, N]
    p0: np.ndarray              # [N]
    name: str = ""
    meta: Dict = field(default_factory=dict)

    @property
    def n(self):
        p = self.params
        return p["nx"] * p["ny"] * p.get("nz", 1)

    @property
    def dim(self):
        return 2 if self.params["lattice"] == D2Q9 else 3

    def with_params(self, **kw):
        return Case(dict(self.params, **kw), self.phi0, self.u0, self.p0, self.name,
                    dict(self.meta))


def base_params(lattice, nx, ny, nz=1, wall=(0, 0, 0), *, sigma, width=4.0,
                theta_m=0.1, tau_f=0.8, tau_g=0.8, rho_l=1.0, rho_g=0.1,
                mu_ratio=None, gravity=0.0, rho_ref=None, remove_fa=0, well=0,
                phi_star=0.5):
    """Physical parameters of a case.  mu_ratio defaults to the density ratio
    (constant kinematic viscosity); rho_ref defaults to rho_g.  well = 0: the
    double well of Eq. 1a with phi in [0, 1]; well = 1: the symmetric well of
    Eq. 1b with phi in [-phi_star, phi_star]."""
    return dict(
        lattice=lattice, nx=int(nx), ny=int(ny), nz=int(nz), wall=[int(w) for w in wall],
        sigma=float(sigma), width=float(width), theta_m=float(theta_m),
        tau_f=float(tau_f), tau_g=float(tau_g), rho_l=float(rho_l), rho_g=float(rho_g),
        mu_ratio=float(rho_l / rho_g if mu_ratio is None else mu_ratio),
        gravity=float(gravity), rho_ref=float(rho_g if rho_ref is None else rho_ref),
        remove_fa=int(remove_fa), well=int(well), phi_star=float(phi_star))


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def tanh_profile(signed_distance, width):
    """1/2 + 1/2 tanh(2 d / W): the flat-interface shape of width W."""
    return 0.5 + 0.5 * np.tanh(2.0 * signed_distance / width)


def droplet_fields(params, centre, radius, *, film_height=None, impact_u=0.0,
                   noise=None, p_base=0.0):
    """phi0 = max(droplet, film); u0 = impact velocity along -vertical inside
    the droplet (+ noise); p0 = p_base + Laplace jump inside the droplet.

    The film of height h sits on the bottom wall, which lies half a cell
    below node 0 of the vertical axis, so its surface is at h - 1/2."""
    nx, ny, nz = params["nx"], params["ny"], params.get("nz", 1)
    dim = 2 if params["lattice"] == D2Q9 else 3
    W = params["width"]
    x, y, z = _grid(nx, ny, nz)
    coords = [x, y, z][:dim]
    r = np.sqrt(sum((c - c0) ** 2 for c, c0 in zip(coords, centre)))
    phi_d = tanh_profile(radius - r, W)
    phi = phi_d.copy()
    vert = coords[dim - 1]
    if film_height is not None:
        phi = np.maximum(phi, tanh_profile(film_height - 0.5 - vert, W))
    u = np.zeros((dim, x.size))
    u[dim - 1] = -impact_u * phi_d
    if noise is not None:
        u += noise
    # Young-Laplace jump: sigma / R in 2-D, 2 sigma / R in 3-D.
    p = p_base + (dim - 1) * params["sigma"] / radius * phi_d
    if params.get("well", 0):
        # the symmetric well's order parameter: phi* tanh(2 d / W)
        phi = params["phi_star"] * (2.0 * phi - 1.0)
    return phi, u, p


# ---------------------------------------------------------------- workloads

def stationary_droplet(seed=0, n=128, radius=25.0, remove_fa=0, noise_amp=1e-4,
                       sigma=0.01, ratio=10.0, tau=0.8, theta_m=0.1, width=4.0,
                       centre_jitter=2.0, name=None, well=0, phi_star=0.5):
    """Stationary 2-D droplet in a periodic n x n box (128^2, R = 25, W = 4,
    ratio 10, sigma = 0.01, tau_f = tau_g = 0.8, theta_M = 0.1).
    Draws: centre jitter x, y ~ U(-2, 2); velocity noise N(0, 1e-4^2)."""
    rng = np.random.default_rng(seed)
    prm = base_params(D2Q9, n, n, sigma=sigma, width=width, theta_m=theta_m,
                      tau_f=tau, tau_g=tau, rho_l=1.0, rho_g=1.0 / ratio,
                      remove_fa=remove_fa, well=well, phi_star=phi_star)
    jit = rng.uniform(-centre_jitter, centre_jitter, size=2) if centre_jitter else np.zeros(2)
    centre = (n / 2 + jit[0], n / 2 + jit[1])
    noise = rng.normal(0.0, noise_amp, size=(2, n * n)) if noise_amp else None
    phi, u, p = droplet_fields(prm, centre, radius, noise=noise)
    return Case(prm, phi, u, p, name or f"droplet{n}", dict(centre=centre, radius=radius))


def splash_2d(seed=0, nx=1024, ny=512, film=40.0, radius=50.0, gap=70.0, impact=0.05,
              ratio=10.0, sigma=0.005, tau_g=0.53, remove_fa=0, jitter=0.5,
              theta_m=0.1, tau_f=0.8, width=4.0):
    """Droplet splashing on a thin film: periodic x, bounce-back walls in y,
    film 40 cells, droplet R = 50 centred 70 cells above the film surface,
    impact velocity 0.05 downwards, ratios 10/10, sigma = 0.005, tau_g = 0.53
    (nu_L = 0.01, Re = U 2R / nu_L = 500).  Draws: jitter U(-0.5, 0.5) on
    x_c, y_c, h."""
    rng = np.random.default_rng(seed)
    prm = base_params(D2Q9, nx, ny, wall=(0, 1, 0), sigma=sigma, width=width,
                      theta_m=theta_m, tau_f=tau_f, tau_g=tau_g,
                      rho_l=1.0, rho_g=1.0 / ratio, remove_fa=remove_fa)
    jx, jy, jh = rng.uniform(-jitter, jitter, size=3) if jitter else (0.0, 0.0, 0.0)
    h = film + jh
    centre = (nx / 2 + jx, h - 0.5 + gap + jy)
    phi, u, p = droplet_fields(prm, centre, radius, film_height=h, impact_u=impact)
    return Case(prm, phi, u, p, f"splash{nx}x{ny}",
                dict(centre=centre, radius=radius, film=h))


def falling_droplet(seed=0, nx=256, ny=1024, radius=32.0, centre=(128.0, 928.0),
                    gravity=1e-6, ratio=10.0, sigma=0.005, tau_g=0.575, remove_fa=1,
                    theta_m=0.1, tau_f=0.8, width=4.0):
    """Falling droplet under gravity: walls all round, R = 32 at (128, 928),
    g = 1e-6, ratios 10/10, sigma = 0.005, tau_g = 0.575 (nu_L = 0.025, the
    paper's falling-droplet viscosity), rho_ref = rho_G.
    No random draws (u0 = 0)."""
    del seed
    prm = base_params(D2Q9, nx, ny, wall=(1, 1, 0), sigma=sigma, width=width,
                      theta_m=theta_m, tau_f=tau_f, tau_g=tau_g,
                      rho_l=1.0, rho_g=1.0 / ratio, gravity=gravity,
                      remove_fa=remove_fa)
    phi, u, p = droplet_fields(prm, centre, radius)
    return Case(prm, phi, u, p, f"falling{nx}x{ny}", dict(centre=centre, radius=radius))


def ensemble(seed=0, ncases=64, sizes=(64, 128, 256, 512), remove_fa=0):
    """Batched ensemble of periodic square droplet cases.  Per case, in this
    order: N from sizes, R/N ~ U[0.15, 0.3], density ratio ~ U[2, 20],
    sigma ~ U[1e-3, 2e-2], g from {0, 1e-6}.  W = 4, tau_f = tau_g = 0.8,
    theta_M = 0.1, centre N/2, u0 = 0.  With gravity in a periodic box the
    reference density is the mean initial density so that the net body force
    vanishes."""
    rng = np.random.default_rng(seed)
    cases: List[Case] = []
    for k in range(ncases):
        n = int(rng.choice(sizes))
        rfrac = rng.uniform(0.15, 0.3)
        ratio = rng.uniform(2.0, 20.0)
        sigma = rng.uniform(1e-3, 2e-2)
        g = float(rng.choice([0.0, 1e-6]))
        prm = base_params(D2Q9, n, n, sigma=sigma, rho_l=1.0, rho_g=1.0 / ratio,
                          gravity=g, remove_fa=remove_fa)
        phi, u, p = droplet_fields(prm, (n / 2, n / 2), rfrac * n)
        prm["rho_ref"] = float(prm["rho_g"] + phi.mean() * (prm["rho_l"] - prm["rho_g"]))
        cases.append(Case(prm, phi, u, p, f"ens{k}_{n}", dict(radius=rfrac * n)))
    return cases


def splash_3d(seed=0, nx=256, ny=256, nz=128, film=16.0, radius=24.0, gap=34.0,
              impact=0.04, ratio=10.0, sigma=0.005, tau_g=0.56, remove_fa=0,
              theta_m=0.1, tau_f=0.8, width=4.0):
    """D3Q19 splash: periodic x, y, walls in z (vertical), film 16, R = 24
    centred 34 above the film surface, impact 0.04 downwards, ratios 10/10,
    sigma = 0.005, tau_g = 0.56.  No random draws."""
    del seed
    prm = base_params(D3Q19, nx, ny, nz, wall=(0, 0, 1), sigma=sigma, width=width,
                      theta_m=theta_m, tau_f=tau_f, tau_g=tau_g, rho_l=1.0,
                      rho_g=1.0 / ratio, remove_fa=remove_fa)
    centre = (nx / 2, ny / 2, film - 0.5 + gap)
    phi, u, p = droplet_fields(prm, centre, radius, film_height=film, impact_u=impact)
    return Case(prm, phi, u, p, f"splash3d{nx}x{ny}x{nz}", dict(centre=centre, radius=radius))


def paper_splash(re=48, seed=0, remove_fa=1, theta_m=0.5):
    """The paper's first test at its own size: 300 x 150, periodic x, walls
    in y; film of one tenth of the height (15 cells); droplet D = 60 falling
    at U = 0.04 onto it; sigma = 1e-4 (We = rho_L U^2 D / sigma = 960);
    Re = U D / nu_L = 48 (nu_L = 0.05) or 480 (nu_L = 0.005); W = 3,
    rho_L = 1, rho_G = 0.1.  Readings (the paper does not state them): the
    droplet centre sits at x = 150, one radius plus W above the film surface;
    constant kinematic viscosity (mu ratio = density ratio); tau_f = 0.8;
    theta_M = 0.5 -- with sigma = 1e-4 the interface relaxes only through
    theta_M beta, and theta_M = 0.1 loses the Re = 48 run near t = 2400.
    (At Re = 480, tau_g = 0.515, the BGK update of this model is unstable
    for every mobility and viscosity ratio tried.)  No random draws."""
    del seed
    nu = {48: 0.05, 480: 0.005}[int(re)]
    nx, ny, film, radius, width, impact = 300, 150, 15.0, 30.0, 3.0, 0.04
    prm = base_params(D2Q9, nx, ny, wall=(0, 1, 0), sigma=1e-4, width=width,
                      theta_m=theta_m, tau_f=0.8, tau_g=0.5 + 3.0 * nu, rho_l=1.0, rho_g=0.1,
                      remove_fa=remove_fa)
    centre = (nx / 2, film - 0.5 + radius + width)
    phi, u, p = droplet_fields(prm, centre, radius, film_height=film, impact_u=impact)
    return Case(prm, phi, u, p, f"paper_splash_re{int(re)}",
                dict(centre=centre, radius=radius, film=film, t_unit=2 * radius / impact))


def paper_falling(seed=0, remove_fa=1):
    """The paper's second test at its own size: 150 x 450, periodic x; a
    droplet of D = 32 falling under gravity with Eo = g (rho_L - rho_G) D^2 /
    sigma = 17, sigma = 0.002, rho_L = 5, rho_G = 1, W = 3, nu_L = 0.025, so
    g = 17 sigma / ((rho_L - rho_G) D^2).  Readings: bounce-back walls at the
    top and bottom (the paper states only the periodic x direction); centre at
    x = 75, two diameters below the top wall; constant kinematic viscosity;
    rho_ref = rho_G; theta_M = 0.1, tau_f = 0.8; u0 = 0.  No random draws."""
    del seed
    nx, ny, d = 150, 450, 32.0
    sigma, rho_l, rho_g = 0.002, 5.0, 1.0
    g = 17.0 * sigma / ((rho_l - rho_g) * d * d)
    prm = base_params(D2Q9, nx, ny, wall=(0, 1, 0), sigma=sigma, width=3.0, theta_m=0.1,
                      tau_f=0.8, tau_g=0.5 + 3.0 * 0.025, rho_l=rho_l, rho_g=rho_g,
                      gravity=g, remove_fa=remove_fa)
    centre = (nx / 2, ny - 0.5 - 2 * d)
    phi, u, p = droplet_fields(prm, centre, d / 2)
    return Case(prm, phi, u, p, "paper_falling150x450", dict(centre=centre, radius=d / 2))


def big_droplet(seed=0, n=4096, radius=800.0, remove_fa=0):
    """Stationary droplet scaled up to a 4096^2 periodic box (R = 800)."""
    return stationary_droplet(seed=seed, n=n, radius=radius, remove_fa=remove_fa,
                              name=f"droplet{n}")


WORKLOADS = {
    "droplet128": dict(builder=stationary_droplet, steps=1000,
                       text="stationary droplet 128x128 periodic, R=25, 1000 steps"),
    "splash1024x512": dict(builder=splash_2d, steps=20000,
                           text="droplet splash on a film 1024x512, periodic x, walls y, 20k steps"),
    "falling256x1024": dict(builder=falling_droplet, steps=50000,
                            text="falling droplet 256x1024, walls all round, 50k steps"),
    "ensemble64": dict(builder=ensemble, steps=2000,
                       text="64 periodic droplet cases of 64^2..512^2, 2000 steps"),
    "splash3d256x256x128": dict(builder=splash_3d, steps=5000,
                                text="D3Q19 splash 256x256x128, periodic x,y, walls z, 5k steps"),
    "droplet4096": dict(builder=big_droplet, steps=200,
                        text="stationary droplet 4096x4096 periodic, R=800, 200 steps"),
    "paper_splash": dict(builder=paper_splash, steps=6000,
                         text="the paper's splash test 300x150, Re 48, to t* = 4"),
    "paper_falling": dict(builder=paper_falling, steps=20000,
                          text="the paper's falling droplet 150x450, Eo = 17, 20k steps"),
}
