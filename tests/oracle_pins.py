"""Pins of the FP64 oracle: checks against facts fixed by the paper and by the
mathematics, not against the oracle's own formulas.

Every check takes the oracle library handle so that the mutation tests can run
the same checks against deliberately broken copies of the oracle.  A check
raises AssertionError when the oracle disagrees with the fact it pins.
"""
import math
from fractions import Fraction

import numpy as np

import workloads as W
from oracle import oracle as O

CS2 = 1.0 / 3.0


def _case(nx, ny, wall=(0, 0, 0), nz=1, lattice=W.D2Q9, **kw):
    base = dict(sigma=0.01, width=4.0, theta_m=0.1, tau_f=0.8, tau_g=0.8,
                rho_l=1.0, rho_g=0.1)
    base.update(kw)
    return W.base_params(lattice, nx, ny, nz, wall, **base)


# ------------------------------------------------------------------ P1 lattice
def check_lattice(lib, lat=W.D2Q9):
    """Weights of the paper (4/9, 1/9, 1/36 for D2Q9) and the isotropy
    moments sum w = 1, sum w e = 0, sum w e e = cs^2 I,
    sum w e e e e = cs^4 (dd + dd + dd), as exact rationals."""
    e, w, opp = O.lattice(lat, lib)
    q, dim = len(w), (2 if lat == W.D2Q9 else 3)
    wf = [Fraction(x).limit_denominator(1000) for x in w]
    for x, f in zip(w, wf):
        assert abs(float(f) - x) < 1e-16
    if lat == W.D2Q9:
        assert q == 9
        assert wf[0] == Fraction(4, 9)
        assert all(f == Fraction(1, 9) for f in wf[1:5])
        assert all(f == Fraction(1, 36) for f in wf[5:9])
        assert all(abs(e[i]).sum() == 1 for i in range(1, 5))
        assert all(abs(e[i]).sum() == 2 for i in range(5, 9))
    else:
        assert q == 19
    assert sum(wf) == 1
    for a in range(dim):
        assert sum(wf[i] * int(e[i, a]) for i in range(q)) == 0
        for b in range(dim):
            m2 = sum(wf[i] * int(e[i, a]) * int(e[i, b]) for i in range(q))
            assert m2 == (Fraction(1, 3) if a == b else 0)
            for c in range(dim):
                assert sum(wf[i] * int(e[i, a] * e[i, b] * e[i, c]) for i in range(q)) == 0
                for d in range(dim):
                    m4 = sum(wf[i] * int(e[i, a] * e[i, b] * e[i, c] * e[i, d])
                             for i in range(q))
                    dl = lambda x, y: 1 if x == y else 0
                    want = Fraction(1, 9) * (dl(a, b) * dl(c, d) + dl(a, c) * dl(b, d)
                                             + dl(a, d) * dl(b, c))
                    assert m4 == want
    for i in range(q):
        assert (e[opp[i]] == -e[i]).all() and opp[opp[i]] == i


# --------------------------------------------------------- P2-P5 local algebra
def _rand_state(rng, dim):
    u = np.zeros(3)
    u[:dim] = rng.uniform(-0.1, 0.1, dim)
    return u


def check_feq_moments(lib, lat=W.D2Q9, trials=50):
    """Order-parameter equilibrium moments: phi, phi u, Gamma mu I + phi u u
    (the moments whose Chapman-Enskog limit is Eq. 2)."""
    rng = np.random.default_rng(1)
    e, _, _ = O.lattice(lat, lib)
    dim = 2 if lat == W.D2Q9 else 3
    E = e[:, :dim].astype(float)
    for _ in range(trials):
        phi, mu, gam = rng.uniform(-0.2, 1.2), rng.uniform(-0.01, 0.01), rng.uniform(0.1, 2)
        u = _rand_state(rng, dim)
        f = O.feq(phi, mu, u, gam, lat, lib)
        assert abs(f.sum() - phi) < 1e-14
        assert np.allclose(E.T @ f, phi * u[:dim], rtol=0, atol=1e-15)
        m2 = (E.T * f) @ E
        want = gam * mu * np.eye(dim) + phi * np.outer(u[:dim], u[:dim])
        assert np.allclose(m2, want, rtol=0, atol=1e-15)


def check_geq_moments(lib, lat=W.D2Q9, trials=50):
    """Pressure equilibrium moments: p, cs^2 rho u, cs^2 (p I + rho u u)."""
    rng = np.random.default_rng(2)
    e, _, _ = O.lattice(lat, lib)
    dim = 2 if lat == W.D2Q9 else 3
    E = e[:, :dim].astype(float)
    for _ in range(trials):
        p, rho = rng.uniform(-1e-3, 1e-3), rng.uniform(0.05, 5.0)
        u = _rand_state(rng, dim)
        g = O.geq(p, rho, u, lat, lib)
        assert abs(g.sum() - p) < 1e-15
        assert np.allclose(E.T @ g, CS2 * rho * u[:dim], rtol=0, atol=1e-15)
        want = CS2 * (p * np.eye(dim) + rho * np.outer(u[:dim], u[:dim]))
        assert np.allclose((E.T * g) @ E, want, rtol=0, atol=1e-15)


def check_source_moments(lib, lat=W.D2Q9, trials=50):
    """Forcing term of Eq. 8: sum (e-u).K = -u . grad psi and
    sum e (e-u).K = cs^2 F."""
    rng = np.random.default_rng(3)
    e, _, _ = O.lattice(lat, lib)
    dim = 2 if lat == W.D2Q9 else 3
    E = e[:, :dim].astype(float)
    for _ in range(trials):
        u = _rand_state(rng, dim)
        F = _rand_state(rng, dim) * 1e-2
        gp = _rand_state(rng, dim) * 1e-2
        s = O.source(u, F, gp, lat, lib)
        assert abs(s.sum() + u[:dim] @ gp[:dim]) < 1e-16
        assert np.allclose(E.T @ s, CS2 * F[:dim], rtol=0, atol=1e-17)


def check_recover(lib, lat=W.D2Q9, trials=50):
    """Build gbar = g^eq(p, rho, u) - S/2 for chosen u, F = Fs + G + c u and
    grad p = 0 (grad psi = -cs^2 grad rho); recovery must return u, F, p."""
    rng = np.random.default_rng(4)
    dim = 2 if lat == W.D2Q9 else 3
    for _ in range(trials):
        u = _rand_state(rng, dim)
        rho = rng.uniform(0.1, 1.0)
        p = rng.uniform(-1e-3, 1e-3)
        fsg = _rand_state(rng, dim) * 1e-3
        c = rng.uniform(-1e-3, 1e-3)
        grho = _rand_state(rng, dim)
        F = fsg + c * u
        gpsi = -CS2 * grho
        gbar = O.geq(p, rho, u, lat, lib) - 0.5 * O.source(u, F, gpsi, lat, lib)
        ur, Fr, pr = O.recover(gbar, rho, fsg, c, grho, lat, lib)
        assert np.allclose(ur[:dim], u[:dim], rtol=0, atol=1e-15)
        assert np.allclose(Fr[:dim], F[:dim], rtol=0, atol=1e-16)
        assert abs(pr - p) < 1e-15


# --------------------------------------------------------------- P6 stencils
def check_stencil_polynomials(lib):
    """Central isotropic stencils are exact on cubic polynomials away from the
    periodic seam: grad and lap of a x^2 + b xy + c y^2 + d x + e y + x^3."""
    n = 24
    case = _case(n, n)
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    a, b, c, d, e3 = 0.3, -0.7, 0.45, 1.1, -0.2
    fld = a * x**2 + b * x * y + c * y**2 + d * x + e3 * y + 0.01 * x**3
    g, lap = O.grad_lap(case, fld.ravel(), lib)
    gx, gy, lap = g[0].reshape(n, n), g[1].reshape(n, n), lap.reshape(n, n)
    inner = (slice(2, n - 2), slice(2, n - 2))
    ex = 2 * a * x + b * y + d + 0.03 * x**2 + 0.01  # d/dx x^3 on the stencil: 3x^2 + 1
    ey = b * x + 2 * c * y + e3
    el = 2 * a + 2 * c + 0.06 * x
    # the isotropic first derivative of x^3 is 3x^2 + 1 (weighted second
    # difference term 3 sum w e_x^3 = 1); the Laplacian of x^3 is exact.
    assert np.allclose(gx[inner], ex[inner], atol=1e-10)
    assert np.allclose(gy[inner], ey[inner], atol=1e-10)
    assert np.allclose(lap[inner], el[inner], atol=1e-10)


def check_stencil_convergence(lib):
    """Second-order convergence of grad and lap on sin(kx x) sin(ky y)."""
    errs = []
    for n in (16, 32, 64):
        case = _case(n, n)
        y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float),
                           indexing="ij")
        k = 2 * math.pi / n
        fld = np.sin(k * x) * np.sin(2 * k * y)
        g, lap = O.grad_lap(case, fld.ravel(), lib)
        ex = k * np.cos(k * x) * np.sin(2 * k * y)
        ey = 2 * k * np.sin(k * x) * np.cos(2 * k * y)
        el = -5 * k * k * fld
        # compare relative to the scale of each derivative (k and k^2)
        errs.append((np.abs(g[0] - ex.ravel()).max() / k,
                     np.abs(g[1] - ey.ravel()).max() / k,
                     np.abs(lap - el.ravel()).max() / k**2))
    errs = np.array(errs)
    slopes = np.log2(errs[:-1] / errs[1:])
    assert (slopes > 1.9).all() and (slopes < 2.1).all(), slopes


def check_stencil_isotropy(lib):
    """The leading error of the isotropic Laplacian is isotropic: on a
    Gaussian, the error at (5, 0) and at (3, 4) from its centre agree to a
    small fraction of the error itself (the 5-point Laplacian fails this)."""
    n = 64
    case = _case(n, n)
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    s2 = 16.0
    r2 = (x - 32) ** 2 + (y - 32) ** 2
    fld = np.exp(-r2 / s2)
    _, lap = O.grad_lap(case, fld.ravel(), lib)
    exact = (4 * r2 / s2**2 - 4 / s2) * fld
    err = (lap.reshape(n, n) - exact)
    e_axis, e_diag = err[32, 37], err[36, 35]
    assert abs(e_axis - e_diag) < 0.1 * abs(e_axis), (e_axis, e_diag)


def check_mirror_ghosts(lib):
    """Wall axes use mirror ghosts about the wall half a cell outside the
    last node.  A grid with walls in y must give the same stencils as the
    periodic grid of twice the height holding the field and its reflection."""
    rng = np.random.default_rng(5)
    nx, ny = 12, 10
    fld = rng.standard_normal((ny, nx))
    g_w, l_w = O.grad_lap(_case(nx, ny, wall=(0, 1, 0)), fld.ravel(), lib)
    big = np.concatenate([fld, fld[::-1]], axis=0)
    g_p, l_p = O.grad_lap(_case(nx, 2 * ny), big.ravel(), lib)
    # the doubled periodic grid's seam at y = 2 ny - 1 / y = 0 mirrors the bottom wall
    assert np.allclose(g_w.reshape(2, ny, nx), g_p.reshape(2, 2 * ny, nx)[:, :ny], atol=1e-14)
    assert np.allclose(l_w.reshape(ny, nx), l_p.reshape(2 * ny, nx)[:ny], atol=1e-14)
    # same along x
    g_w, l_w = O.grad_lap(_case(nx, ny, wall=(1, 0, 0)), fld.ravel(), lib)
    big = np.concatenate([fld, fld[:, ::-1]], axis=1)
    g_p, l_p = O.grad_lap(_case(2 * nx, ny), big.ravel(), lib)
    assert np.allclose(g_w.reshape(2, ny, nx), g_p.reshape(2, ny, 2 * nx)[:, :, :nx], atol=1e-14)
    assert np.allclose(l_w.reshape(ny, nx), l_p.reshape(ny, 2 * nx)[:, :nx], atol=1e-14)


def check_stencils_d3q19(lib):
    """The D3Q19 stencils (18 neighbours, weights 1/18 and 1/36):
    exact on a quadratic in x, y, z plus x^3 away from the seams (the
    isotropic first derivative of x^3 is 3x^2 + 1, as in 2-D, since
    3 sum w e_x^3 = 1 on this lattice too; the Laplacian of x^3 is exact),
    second-order convergence on sin kx sin 2ky sin kz, an isotropic leading
    error on a Gaussian (same error along an axis, a face diagonal in the xy
    plane and one in the yz plane), and wall ghosts equal to a doubled periodic
    grid holding the field and its reflection in z."""
    def grid(nx, ny, nz):
        z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                              np.arange(nx, dtype=float), indexing="ij")
        return x, y, z

    n = 12
    case = _case(n, n, nz=n, lattice=W.D3Q19)
    x, y, z = grid(n, n, n)
    a, b, c, d, e, f, gx_, gy_, gz_ = 0.3, -0.7, 0.45, 0.2, 0.55, -0.35, 1.1, -0.2, 0.6
    fld = (a * x**2 + b * x * y + c * y**2 + d * z**2 + e * x * z + f * y * z
           + gx_ * x + gy_ * y + gz_ * z + 0.01 * x**3)
    g, lap = O.grad_lap(case, fld.ravel(), lib)
    g = g.reshape(3, n, n, n)
    lap = lap.reshape(n, n, n)
    inner = (slice(2, n - 2),) * 3
    want = [2 * a * x + b * y + e * z + gx_ + 0.03 * x**2 + 0.01,
            b * x + 2 * c * y + f * z + gy_,
            2 * d * z + e * x + f * y + gz_]
    for k in range(3):
        assert np.allclose(g[k][inner], want[k][inner], atol=1e-10), k
    assert np.allclose(lap[inner], (2 * a + 2 * c + 2 * d + 0.06 * x)[inner], atol=1e-10)

    errs = []
    for n in (16, 32, 64):
        case = _case(n, n, nz=n, lattice=W.D3Q19)
        x, y, z = grid(n, n, n)
        k = 2 * math.pi / n
        fld = np.sin(k * x) * np.sin(2 * k * y) * np.sin(k * z)
        g, lap = O.grad_lap(case, fld.ravel(), lib)
        ex = k * np.cos(k * x) * np.sin(2 * k * y) * np.sin(k * z)
        ey = 2 * k * np.sin(k * x) * np.cos(2 * k * y) * np.sin(k * z)
        ez = k * np.sin(k * x) * np.sin(2 * k * y) * np.cos(k * z)
        el = -6 * k * k * fld
        errs.append((np.abs(g[0] - ex.ravel()).max() / k, np.abs(g[1] - ey.ravel()).max() / k,
                     np.abs(g[2] - ez.ravel()).max() / k, np.abs(lap - el.ravel()).max() / k**2))
    errs = np.array(errs)
    slopes = np.log2(errs[:-1] / errs[1:])
    assert (slopes > 1.9).all() and (slopes < 2.1).all(), slopes

    n = 32
    case = _case(n, n, nz=n, lattice=W.D3Q19)
    x, y, z = grid(n, n, n)
    s2 = 16.0
    r2 = (x - 16) ** 2 + (y - 16) ** 2 + (z - 16) ** 2
    fld = np.exp(-r2 / s2)
    _, lap = O.grad_lap(case, fld.ravel(), lib)
    err = lap.reshape(n, n, n) - (4 * r2 / s2**2 - 6 / s2) * fld
    e_axis, e_xy, e_yz = err[16, 16, 21], err[16, 20, 19], err[19, 20, 16]
    assert abs(e_axis - e_xy) < 0.1 * abs(e_axis), (e_axis, e_xy)
    assert abs(e_axis - e_yz) < 0.1 * abs(e_axis), (e_axis, e_yz)

    rng = np.random.default_rng(6)
    nx, ny, nz = 6, 5, 7
    fld = rng.standard_normal((nz, ny, nx))
    g_w, l_w = O.grad_lap(_case(nx, ny, (0, 0, 1), nz=nz, lattice=W.D3Q19), fld.ravel(), lib)
    big = np.concatenate([fld, fld[::-1]], axis=0)
    g_p, l_p = O.grad_lap(_case(nx, ny, nz=2 * nz, lattice=W.D3Q19), big.ravel(), lib)
    assert np.allclose(g_w.reshape(3, nz, ny, nx), g_p.reshape(3, 2 * nz, ny, nx)[:, :nz],
                       atol=1e-14)
    assert np.allclose(l_w.reshape(nz, ny, nx), l_p.reshape(2 * nz, ny, nx)[:nz], atol=1e-14)


# ------------------------------------------------------- P7/P8 thermodynamics
def _uniform_mu(lib, phi, beta_sigma=0.01, width=4.0):
    n = 4
    case = _case(n, n, sigma=beta_sigma, width=width)
    s = O.Sim(case, np.full(n * n, phi), np.zeros(2 * n * n), np.zeros(n * n), lib=lib)
    return s.fields()["mu"][0]


def check_chemical_potential(lib):
    """On a uniform field mu = theta'(phi) of theta = beta phi^2 (phi-1)^2
    (Eq. 1a): zero at 0, 1/2 and 1, and equal to a centred difference of
    theta."""
    sigma, width = 0.01, 4.0
    beta, _ = O.beta_kappa(sigma, width, lib)
    for phi in (0.0, 0.5, 1.0):
        assert abs(_uniform_mu(lib, phi, sigma, width)) < 1e-17
    th = lambda p: beta * p * p * (p - 1) ** 2
    h = 1e-5
    for phi in (-0.1, 0.2, 0.7, 1.05):
        fd = (th(phi + h) - th(phi - h)) / (2 * h)
        assert abs(_uniform_mu(lib, phi, sigma, width) - fd) < 1e-10


def check_beta_kappa(lib):
    """beta, kappa from sigma, W make 1/2 + 1/2 tanh(2z/W) solve
    kappa phi'' = theta'(phi) and give tension int kappa phi'^2 dz = sigma."""
    from scipy.integrate import quad
    for sigma, width in ((0.01, 4.0), (0.005, 3.0), (1e-4, 3.0)):
        beta, kappa = O.beta_kappa(sigma, width, lib)
        for z in np.linspace(-6, 6, 25):
            t = math.tanh(2 * z / width)
            phi = 0.5 + 0.5 * t
            d1 = (1 - t * t) / width
            d2 = -4.0 / width**2 * t * (1 - t * t)
            dth = 2 * beta * phi * (phi - 1) * (2 * phi - 1)
            assert abs(kappa * d2 - dth) < 1e-12 * max(1.0, beta)
        tension = quad(lambda z: kappa * ((1 - math.tanh(2 * z / width) ** 2) / width) ** 2,
                       -50, 50, epsabs=1e-14)[0]
        assert abs(tension - sigma) < 1e-9 * sigma + 1e-15


# ---------------------------------------------------------------- P9 stream
def check_stream_permutation(lib):
    """Streaming moves words without changing them: a permutation; with
    reversal of directions it is an involution (stream, reverse, stream,
    reverse = identity), on periodic and wall axes."""
    rng = np.random.default_rng(6)
    for lat, dims, wall in ((W.D2Q9, (7, 5, 1), (0, 0, 0)), (W.D2Q9, (6, 9, 1), (0, 1, 0)),
                            (W.D2Q9, (5, 4, 1), (1, 1, 0)),
                            (W.D3Q19, (5, 4, 6), (0, 0, 1)), (W.D3Q19, (4, 5, 4), (1, 1, 1))):
        case = _case(dims[0], dims[1], wall=wall, nz=dims[2], lattice=lat)
        e, _, opp = O.lattice(lat, lib)
        q, n = len(e), dims[0] * dims[1] * dims[2]
        words = rng.integers(0, 2**32, size=(q, n), dtype=np.uint64).astype(np.uint32)
        out = O.stream_words(case, words, lib)
        assert np.array_equal(np.sort(out.ravel()), np.sort(words.ravel()))
        back = O.stream_words(case, out[opp], lib)[opp]
        assert np.array_equal(back, words)
        # pull semantics on an interior link: out_i(x) = in_i(x - e_i)
        if lat == W.D2Q9 and wall == (0, 0, 0):
            nx, ny = dims[0], dims[1]
            for i in range(q):
                x, y = 3, 2
                sx, sy = (x - e[i, 0]) % nx, (y - e[i, 1]) % ny
                assert out[i, x + nx * y] == words[i, sx + nx * sy]


# ----------------------------------------------------- P10/P11 whole steps
def check_fixed_point(lib):
    """Uniform phi in {0, 1} at rest with p = 0 and no gravity is a fixed point
    of the step, to the last bit: mu = 0, K = 0, f = phi delta_i0, gbar = 0."""
    for lat, dims, wall in ((W.D2Q9, (8, 6, 1), (0, 1, 0)), (W.D3Q19, (4, 5, 6), (0, 0, 1))):
        for phi in (0.0, 1.0):
            for rf in (0, 1, 2):
                case = _case(dims[0], dims[1], wall=wall, nz=dims[2], lattice=lat,
                             remove_fa=rf)
                n = dims[0] * dims[1] * dims[2]
                dim = 2 if lat == W.D2Q9 else 3
                s = O.Sim(case, np.full(n, phi), np.zeros(dim * n), np.zeros(n), lib=lib)
                f0, g0 = s.get_state()
                assert np.array_equal(f0[0], np.full(n, phi)) and not f0[1:].any()
                assert not g0.any()
                s.step(5)
                f1, g1 = s.get_state()
                assert np.array_equal(f0, f1) and np.array_equal(g0, g1)


def check_uniform_flow(lib):
    """A uniform phase moving uniformly in a periodic box stays as it is."""
    n = 8
    for phi in (0.0, 1.0, 0.3):
        case = _case(n, n)
        u0 = np.zeros((2, n * n))
        u0[0], u0[1] = 0.02, -0.013
        s = O.Sim(case, np.full(n * n, phi), u0, np.full(n * n, 1e-4), lib=lib)
        s.step(20)
        fl = s.fields()
        assert np.allclose(fl["phi"], phi, atol=1e-13)
        assert np.allclose(fl["u"][0], 0.02, atol=1e-13)
        assert np.allclose(fl["u"][1], -0.013, atol=1e-13)
        assert np.allclose(fl["p"], 1e-4, atol=1e-13)


def check_conservation(lib):
    """Sum phi is conserved (no flux through periodic seams or bounce-back
    walls; the paper's remark after Eq. 5) for both models and lattices."""
    for wall in ((0, 0, 0), (0, 1, 0), (1, 1, 0)):
        for rf in (0, 1):
            c = W.stationary_droplet(seed=3, n=32, radius=8.0, noise_amp=1e-3,
                                     remove_fa=rf)
            prm = dict(c.params, wall=list(wall))
            s = O.Sim(prm, c.phi0, c.u0 + 0.01, c.p0, lib=lib)
            m0 = s.diag()["mass"]
            s.step(100)
            m1 = s.diag()["mass"]
            assert abs(m1 - m0) < 1e-13 * abs(m0), (wall, rf, m0, m1)
    c = W.splash_3d(nx=12, ny=10, nz=14, film=3.0, radius=3.0, gap=4.0)
    s = O.Sim(dict(c.params, remove_fa=1), c.phi0, c.u0, c.p0, lib=lib)
    m0 = s.diag()["mass"]
    s.step(30)
    assert abs(s.diag()["mass"] - m0) < 1e-13 * m0


def check_uniform_force(lib):
    """Under a uniform body force in a uniform phase, the recovered velocity
    grows by F/rho each step; the initial state carries no half-force
    correction, so u(n) = (n + 1/2) F / rho exactly."""
    n = 6
    for phi, dims, lat in ((1.0, (n, n, 1), W.D2Q9), (0.0, (n, n, 1), W.D2Q9),
                           (1.0, (4, 4, 5), W.D3Q19)):
        case = _case(dims[0], dims[1], nz=dims[2], lattice=lat, gravity=1e-5,
                     rho_ref=0.55, tau_g=0.7)
        nn = dims[0] * dims[1] * dims[2]
        dim = 2 if lat == W.D2Q9 else 3
        s = O.Sim(case, np.full(nn, phi), np.zeros(dim * nn), np.zeros(nn), lib=lib)
        rho = 0.1 + phi * 0.9
        F = -(rho - 0.55) * 1e-5
        for k in (0, 1, 7):
            s.step(k - s.time)
            u = s.fields()["u"]
            # (omega - w) cancels to ~1e-16 absolute, so u ~ 1e-6 carries ~1e-11
            # relative rounding
            assert np.allclose(u[dim - 1], (k + 0.5) * F / rho, rtol=1e-9, atol=0)
            assert np.allclose(u[:dim - 1], 0.0, atol=1e-20)


def check_shear_wave(lib):
    """Decay of a shear wave u_x = A sin(k y) in one phase: rate nu k^2 with
    nu = cs^2 (tau - 1/2) (Eq. 3 with constant viscosity).  In the gas with
    mu_L / mu_G != rho_L / rho_G the gas viscosity mu_G / rho_G applies."""
    nx, ny = 4, 64
    k = 2 * math.pi / ny
    y = np.repeat(np.arange(ny, dtype=float), nx)
    for phi, mu_ratio, nu_expect in ((1.0, 10.0, CS2 * 0.3), (0.0, 10.0, CS2 * 0.3),
                                     (0.0, 4.0, CS2 * 0.3 * 1.0 / 4.0 / 0.1)):
        case = _case(nx, ny, tau_g=0.8, mu_ratio=mu_ratio)
        u0 = np.zeros((2, nx * ny))
        u0[0] = 1e-4 * np.sin(k * y)
        s = O.Sim(case, np.full(nx * ny, phi), u0, np.zeros(nx * ny), lib=lib)
        s.step(10)
        a1 = np.dot(s.fields()["u"][0], np.sin(k * y))
        s.step(200)
        a2 = np.dot(s.fields()["u"][0], np.sin(k * y))
        rate = math.log(a1 / a2) / 200
        assert abs(rate / (nu_expect * k * k) - 1) < 0.01, (phi, mu_ratio, rate, nu_expect * k * k)


def check_ch_diffusion(lib):
    """Linearised Cahn-Hilliard (Eq. 2 at rest): a small mode of phi around
    phi0 decays at theta_M k^2 (theta''(phi0) + kappa k^2), with the mobility
    theta_M given directly as a parameter."""
    nx, ny = 64, 4
    k = 2 * math.pi / nx
    x = np.tile(np.arange(nx, dtype=float), ny)
    for theta_m, tau_f, phi0 in ((0.1, 0.8, 0.0), (0.05, 1.2, 1.0), (0.2, 0.7, 0.0)):
        sigma, width = 0.01, 4.0
        case = _case(nx, ny, theta_m=theta_m, tau_f=tau_f, sigma=sigma, width=width,
                     rho_l=1.0, rho_g=1.0)
        beta, kappa = O.beta_kappa(sigma, width, lib)
        phi = phi0 + 1e-5 * np.cos(k * x)
        s = O.Sim(case, phi, np.zeros(2 * nx * ny), np.zeros(nx * ny), lib=lib)
        s.step(20)
        a1 = np.dot(s.fields()["phi"] - phi0, np.cos(k * x))
        s.step(400)
        a2 = np.dot(s.fields()["phi"] - phi0, np.cos(k * x))
        rate = math.log(a1 / a2) / 400
        # theta''(phi) = 2 beta (6 phi^2 - 6 phi + 1) = 2 beta at 0 and 1
        expect = theta_m * k * k * (2 * beta + kappa * k * k)
        assert abs(rate / expect - 1) < 0.02, (theta_m, tau_f, rate, expect)


# -------------------------------------------------------- P12/P13 interfaces
def flat_interface_error(lib, width, steps=6000):
    """Max deviation of a relaxed liquid slab from 1/2 + 1/2 tanh(2 z / W).
    The slab starts from that profile; the discrete scheme relaxes it to its
    own equilibrium, whose distance from the continuous one is measured."""
    ny = int(32 * width)
    nx = 4
    y = np.repeat(np.arange(ny, dtype=float), nx)
    lo, hi = ny / 4, 3 * ny / 4
    phi = 0.5 + 0.5 * np.tanh(2 * np.minimum(y - lo, hi - y) / width)
    case = _case(nx, ny, width=width, sigma=0.01)
    s = O.Sim(case, phi, np.zeros(2 * nx * ny), np.zeros(nx * ny), lib=lib)
    s.step(steps)
    got = s.fields()["phi"].reshape(ny, nx)[:, 0]
    yy = np.arange(ny, dtype=float)
    exact = 0.5 + 0.5 * np.tanh(2 * np.minimum(yy - lo, hi - yy) / width)
    return np.abs(got - exact).max()


def check_flat_interface(lib):
    """A flat interface relaxes to the tanh profile of width W; the error
    falls roughly fourfold each time W doubles (second-order stencils)."""
    e4 = flat_interface_error(lib, 4.0)
    e8 = flat_interface_error(lib, 8.0)
    assert e4 < 1e-2, e4
    assert 3.0 < e4 / e8 < 6.0, (e4, e8)


def laplace_dp(lib, radius, n=96, steps=3000, sigma=0.01, width=4.0, well=0, phi_star=0.5,
               theta_m=0.1):
    c = W.stationary_droplet(seed=0, n=n, radius=radius, noise_amp=0.0, centre_jitter=0.0,
                             sigma=sigma, width=width, well=well, phi_star=phi_star,
                             theta_m=theta_m)
    s = O.Sim(c.params, c.phi0, np.zeros_like(c.u0), np.zeros_like(c.p0), lib=lib)
    s.step(steps)
    p = s.fields()["p"].reshape(n, n)
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    r = np.hypot(x - n / 2, y - n / 2)
    return p[r < radius - 2 * width].mean() - p[r > radius + 2 * width].mean()


def check_laplace(lib):
    """Young-Laplace law for a resting 2-D droplet: dp = sigma / R.  The
    pressure starts at zero everywhere; the slope of dp against 1/R must
    give sigma to 5 %."""
    radii = np.array([12.0, 16.0, 20.0, 28.0])
    dps = np.array([laplace_dp(lib, r) for r in radii])
    slope = np.polyfit(1 / radii, dps, 1)[0]
    assert abs(slope / 0.01 - 1) < 0.05, (slope, dps)
    assert np.all(np.abs(dps * radii / 0.01 - 1) < 0.08), dps * radii


# ------------------------------------------------------------- P14 switch
def check_switch_noop(lib):
    """The correction -F_a = u drho theta_M lap mu vanishes with theta_M = 0 or
    rho_L = rho_G, so the switch has no effect there (to the last bit), and
    it does change a moving two-phase flow otherwise."""
    c = W.stationary_droplet(seed=1, n=32, radius=8.0, noise_amp=1e-2)
    u0 = c.u0 + 0.02

    def run(rf, **kw):
        s = O.Sim(dict(c.params, remove_fa=rf, **kw), c.phi0, u0, c.p0, lib=lib)
        s.step(40)
        return s.get_state()

    for kw in (dict(theta_m=0.0), dict(rho_g=1.0, mu_ratio=1.0)):
        a, b = run(0, **kw), run(1, **kw)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    a, b = run(0), run(1)
    assert not np.array_equal(a[1], b[1])


def check_fa_field(lib):
    """F_a = -u drho theta_M lap mu is interfacial: it vanishes in the bulk of
    both phases and is largest in the interface (remarks after Eq. 12)."""
    c = W.stationary_droplet(seed=2, n=64, radius=16.0, noise_amp=0.0, centre_jitter=0.0)
    u0 = np.zeros_like(c.u0)
    u0[1] = -0.02
    s = O.Sim(dict(c.params, remove_fa=0), c.phi0, u0, c.p0, lib=lib)
    s.step(10)
    fl = s.fields()
    fa = np.hypot(fl["fa"][0], fl["fa"][1])
    n, width = 64, c.params["width"]
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    # distance to the interface of the droplet, which moved 10 * 0.02 cells down
    dist = np.abs(np.hypot(x - 32, y - 32 + 0.2) - 16.0).ravel()
    interface = dist < 0.5 * width
    bulk = dist > 2.5 * width
    assert fa[interface].max() > 100 * max(fa[bulk].max(), 1e-30)


# ----------------------------------------------- momentum, Eq. 5, advection
def _total_force(lib, case, fl):
    """Sum over nodes of F_s + G (+ u drho theta_M lap mu in the corrected
    model) from the dumped fields, with grad phi from the pinned stencil."""
    dim = fl["u"].shape[0]
    grad, _ = O.grad_lap(case, fl["phi"], lib)
    rho = case["rho_g"] + fl["phi"] * (case["rho_l"] - case["rho_g"])
    F = fl["mu"] * grad
    F[dim - 1] += -(rho - case["rho_ref"]) * case["gravity"]
    if case["remove_fa"]:
        F -= fl["fa"]
    return F.sum(axis=1), (rho * fl["u"]).sum(axis=1)


def check_momentum_balance(lib):
    """Discrete momentum balance of the pressure LBE in a periodic box:
    streaming conserves sum e gbar and the collision turns rho u - F/2 into
    rho u + F/2, so sum rho u grows by (F^n + F^(n+1)) / 2 per step, with F
    the total force (Eq. 3 forces, plus -F_a in the corrected model)."""
    for rf in (0, 1):
        c = W.stationary_droplet(seed=4, n=32, radius=9.0, noise_amp=5e-3, remove_fa=rf)
        case = dict(c.params, gravity=2e-5, rho_ref=0.1)
        s = O.Sim(case, c.phi0, c.u0 + np.array([[0.01], [-0.02]]), c.p0, lib=lib)
        s.step(3)
        Fp, Pp = _total_force(lib, case, s.fields())
        for _ in range(4):
            s.step(1)
            Fn, Pn = _total_force(lib, case, s.fields())
            assert np.allclose(Pn - Pp, 0.5 * (Fn + Fp), rtol=1e-9, atol=1e-15), (
                rf, Pn - Pp, 0.5 * (Fn + Fp))
            Fp, Pp = Fn, Pn


def check_correction_velocity(lib):
    """On one and the same state, the corrected model's velocity differs from
    the original's only through the implicit -F_a in the half-force term:
    rho u_orig = (rho - drho theta_M lap mu / 2) u_corr, i.e.
    u_orig - u_corr = F_a,corr / (2 rho)."""
    c = W.stationary_droplet(seed=5, n=32, radius=9.0, noise_amp=5e-3)
    s = O.Sim(dict(c.params, remove_fa=0), c.phi0, c.u0 + 0.03, c.p0, lib=lib)
    s.step(5)
    f, g = s.get_state()
    s1 = O.Sim(dict(c.params, remove_fa=1), c.phi0, c.u0, c.p0, lib=lib)
    s1.set_state(f, g, 5)
    fo, fc = s.fields(), s1.fields()
    rho = c.params["rho_g"] + fo["phi"] * (c.params["rho_l"] - c.params["rho_g"])
    diff = fo["u"] - fc["u"]
    want = fc["fa"] / (2 * rho)
    assert np.abs(want).max() > 1e-9
    assert np.allclose(diff, want, rtol=1e-7, atol=1e-17)


def check_eq5_fa(lib):
    """Reading of Eq. 5 behind F_a: in this model d_t phi + div(phi u) =
    theta_M lap mu (Eq. 2 in conservative form), so d_t rho + div(rho u) is
    drho theta_M lap mu up to rho_G div u.  Measured from the data (centred
    differences in time and space) on a relaxing interface, it must track
    theta_M lap mu (correlation, slope near 1), and the dumped F_a must be
    -u drho theta_M lap mu."""
    n = 48
    c = W.stationary_droplet(seed=6, n=n, radius=10.0, noise_amp=0.0, centre_jitter=0.0,
                             width=5.0)
    # start off equilibrium (interface too thin) so that lap mu is large
    y, x = np.meshgrid(np.arange(float(n)), np.arange(float(n)), indexing="ij")
    phi = 0.5 + 0.5 * np.tanh(2 * (10.0 - np.hypot(x - 24, y - 24)) / 2.5).ravel()
    s = O.Sim(dict(c.params, remove_fa=0), phi, np.zeros_like(c.u0), c.p0, lib=lib)
    s.step(100)
    f_prev = s.fields()
    s.step(1)
    f_now = s.fields()
    s.step(1)
    f_next = s.fields()
    dt_phi = ((f_next["phi"] - f_prev["phi"]) / 2).reshape(n, n)
    ph = f_now["phi"].reshape(n, n)
    ux, uy = f_now["u"][0].reshape(n, n), f_now["u"][1].reshape(n, n)
    div = ((np.roll(ph * ux, -1, 1) - np.roll(ph * ux, 1, 1)) / 2
           + (np.roll(ph * uy, -1, 0) - np.roll(ph * uy, 1, 0)) / 2)
    lhs = (dt_phi + div).ravel()
    rhs = c.params["theta_m"] * f_now["lapmu"]
    corr = np.corrcoef(lhs, rhs)[0, 1]
    slope = np.dot(lhs, rhs) / np.dot(rhs, rhs)
    assert corr > 0.98 and 0.9 < slope < 1.3, (corr, slope)
    drho = c.params["rho_l"] - c.params["rho_g"]
    assert np.allclose(f_now["fa"], -f_now["u"] * drho * rhs, rtol=1e-12, atol=1e-24)


def check_advection(lib):
    """A droplet in a uniform stream is carried along with the flow (the
    phi u flux of Eq. 2): at equal densities it moves at the stream velocity;
    at density ratio 10 its centroid velocity follows the mean velocity
    sum rho u / sum rho (which the discrete surface force slowly changes)."""
    for rf in (0, 1):
        for ratio in (1.0, 10.0):
            c = W.stationary_droplet(seed=7, n=64, radius=12.0, noise_amp=0.0,
                                     remove_fa=rf, ratio=ratio)
            u0 = np.zeros_like(c.u0)
            u0[0], u0[1] = 0.02, -0.01
            s = O.Sim(c.params, c.phi0, u0, c.p0, lib=lib)
            x0 = s.diag()["centroid"][:2]
            s.step(400)
            d = s.diag()
            if ratio == 1.0:
                moved = d["centroid"][:2] - x0
                assert np.allclose(moved, [8.0, -4.0], rtol=0.01), moved
            rho = c.params["rho_g"] + s.fields()["phi"] * (c.params["rho_l"] - c.params["rho_g"])
            mean_u = d["momentum"][:2] / rho.sum()
            assert np.allclose(d["centroid_vel"][:2], mean_u, rtol=0.01), (
                d["centroid_vel"], mean_u)

def check_diagnostics(lib):
    """Diagnostics of a known field: the centroid weight clamp(2 phi - 1/2,
    0, 1) is 0 at phi = 1/4, 1/2 at phi = 1/2 and 1 at phi = 3/4; a resting
    symmetric droplet has its centroid at its centre, a disk's second
    moment per axis is R^2 / 4, and mass is sum phi."""
    n = 8
    case = _case(n, n)
    for phi, w in ((0.25, 0.0), (0.5, 0.5), (0.75, 1.0), (1.0, 1.0), (0.1, 0.0)):
        s = O.Sim(case, np.full(n * n, phi), np.zeros(2 * n * n), np.zeros(n * n), lib=lib)
        d = s.diag()
        assert abs(d["wsum"] - w * n * n) < 1e-12 and abs(d["mass"] - phi * n * n) < 1e-12
    c = W.stationary_droplet(seed=0, n=128, radius=40.0, noise_amp=0.0, centre_jitter=0.0)
    s = O.Sim(c.params, c.phi0, c.u0, c.p0, lib=lib)
    d = s.diag()
    assert np.allclose(d["centroid"][:2], [64.0, 64.0], atol=1e-9)
    assert np.allclose(d["second_moment"][:2], 40.0 ** 2 / 4, rtol=0.02), d["second_moment"]
    assert abs(d["mass"] - c.phi0.sum()) < 1e-9 and d["nonfinite"] == 0


def check_field_diag(lib):
    """Diagnostics from given node fields.  A 2 x 2 grid worked by hand: phi
    = 3/4, 1/2, 1/4, 1 at (0,0), (1,0), (0,1), (1,1) gives weights 1, 1/2,
    0, 1 (sum 5/2), centroid (0.6, 0.4), second moments 0.6 / 2.5 = 0.24 per
    axis; rho = 0.1 + 0.9 phi with u = (0.01, 0.02, 0.03, 0.04; 0, 0, 0,
    -0.03) gives momentum (0.0685, -0.03), centroid velocity (0.024, -0.012)
    and |u|max 0.05.  A non-finite u is counted.  The symmetric well's
    midpoint phi = 0 weighs 1/2.  A droplet that has moved for a few steps
    gives the diagnostics of the simulation that produced its fields."""
    phi = np.array([0.75, 0.5, 0.25, 1.0])
    u = np.array([[0.01, 0.02, 0.03, 0.04], [0.0, 0.0, 0.0, -0.03]])
    d = O.field_diag(phi, u, (2, 2), 0.0, 1.0, 0.1, 1.0, lib=lib)
    want = dict(mass=2.5, wsum=2.5, momentum=[0.0685, -0.03, 0.0], centroid=[0.6, 0.4, 0.0],
                centroid_vel=[0.024, -0.012, 0.0], second_moment=[0.24, 0.24, 0.0], umax=0.05)
    for k, v in want.items():
        assert np.allclose(d[k], v, rtol=0, atol=1e-15), (k, d[k], v)
    assert d["nonfinite"] == 0
    u[1, 2] = np.nan
    assert O.field_diag(phi, u, (2, 2), 0.0, 1.0, 0.1, 1.0, lib=lib)["nonfinite"] == 1
    ds = O.field_diag(np.zeros(8), np.zeros((3, 8)), (2, 2, 2), -0.5, 0.5, 0.1, 1.0, lib=lib)
    assert abs(ds["wsum"] - 4.0) < 1e-15 and np.allclose(ds["centroid"], 0.5)
    assert np.allclose(ds["second_moment"], 0.25) and abs(ds["momentum"]).max() == 0.0
    c = W.stationary_droplet(seed=3, n=48, radius=12.0, centre_jitter=3.0)
    sim = O.Sim(c.params, c.phi0, c.u0, c.p0, lib=lib)
    sim.step(5)
    f, ref = sim.fields(), sim.diag()
    d = O.field_diag(f["phi"], f["u"], (48, 48), 0.0, 1.0, c.params["rho_g"],
                     c.params["rho_l"], lib=lib)
    assert ref["umax"] > 0.0
    for k in ("mass", "wsum", "centroid", "centroid_vel", "second_moment", "umax", "momentum"):
        assert np.allclose(d[k], ref[k], rtol=1e-12, atol=1e-15), (k, d[k], ref[k])


def check_spread_radius(lib):
    """Diagnostic D6 (half-width of the widest row, as in the paper's Fig. 5)
    on fields whose answer is known: a two-level band of nodes 10..30 crosses
    1/2 half-way between nodes, 9.5 and 30.5 (half-width 10.5); a tanh disk
    whose centre lies on a grid row has half-width R there (the tanh profile
    is odd about its crossing, so linear interpolation lands on it); a centre
    between rows gives the chord sqrt(R^2 - d^2) of the nearest row; a field
    with no row crossing twice gives 0; the level is honoured."""
    nx, ny = 40, 5
    phi = np.zeros((ny, nx))
    phi[2, 10:31] = 1.0
    assert abs(O.spread_radius(phi.ravel(), (nx, ny), lib=lib) - 10.5) < 1e-14
    ramp = np.zeros((ny, nx))
    ramp[1, 10:31] = 0.8
    assert abs(O.spread_radius(ramp.ravel(), (nx, ny), 0.4, lib=lib) - 10.5) < 1e-14
    assert O.spread_radius(ramp.ravel(), (nx, ny), 0.9, lib=lib) == 0.0
    half = np.zeros((ny, nx))
    half[:, 20:] = 1.0                     # one crossing per row only
    assert O.spread_radius(half.ravel(), (nx, ny), lib=lib) == 0.0
    nx, ny = 150, 120
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    for R, xc, yc in ((20.0, 74.3, 60.0), (27.5, 70.0, 44.0)):
        ph = 0.5 + 0.5 * np.tanh(2.0 * (R - np.hypot(x - xc, y - yc)) / 3.0)
        assert abs(O.spread_radius(ph.ravel(), (nx, ny), lib=lib) - R) < 1e-9
    R, yc = 31.7, 55.3
    ph = 0.5 + 0.5 * np.tanh(2.0 * (R - np.hypot(x - 75.0, y - yc)) / 3.0)
    want = math.sqrt(R * R - 0.3 * 0.3)
    assert abs(O.spread_radius(ph.ravel(), (nx, ny), lib=lib) - want) < 2e-2


def check_fa_discrete(lib):
    """F_a from discrete data, -u [(rho^n - rho^(n-1)) + div(rho u)], against
    closed forms of the discrete operators on a periodic sine of phi:
    at rest it is 0; for a static field and uniform velocity the central
    difference of sin(kx) is sin(k) cos(kx), so F = -u (u . drho a sin(k) cos(kx));
    for a field shifted by one cell per step at unit speed the sum is
    minus half the second difference, -4 sin^2(k/2) of the sine, giving
    F_x = -(1/2) drho a 4 sin^2(k/2) sin(kx) (the first-order truncation of
    the backward difference); and a y-only field gives no x-divergence."""
    nx, ny = 64, 8
    case = _case(nx, ny, rho_l=1.0, rho_g=0.1)
    drho = 0.9
    x = np.tile(np.arange(nx, dtype=float), ny)
    k = 2 * math.pi * 3 / nx
    a = 0.2
    phi = 0.5 + a * np.sin(k * x)
    u0 = np.zeros((2, nx * ny))
    assert np.abs(O.fa_discrete(case, phi, phi, u0, lib=lib)).max() == 0.0
    U, V = 0.03, -0.02
    u = np.vstack([np.full(nx * ny, U), np.full(nx * ny, V)])
    f = O.fa_discrete(case, phi, phi, u, lib=lib)
    s_ = U * drho * a * math.sin(k) * np.cos(k * x)
    assert np.allclose(f[0], -U * s_, atol=1e-15) and np.allclose(f[1], -V * s_, atol=1e-15)
    prev = 0.5 + a * np.sin(k * (x + 1.0))    # phi^n(x) = phi^(n-1)(x - 1)
    u1 = np.vstack([np.ones(nx * ny), np.zeros(nx * ny)])
    f = O.fa_discrete(case, prev, phi, u1, lib=lib)
    want = -0.5 * drho * a * 4 * math.sin(k / 2) ** 2 * np.sin(k * x)
    assert np.allclose(f[0], want, atol=1e-14) and np.abs(f[1]).max() == 0.0
    y = np.repeat(np.arange(ny, dtype=float), nx)
    phiy = 0.5 + a * np.sin(2 * math.pi * y / ny)
    f = O.fa_discrete(case, phiy, phiy, np.vstack([np.full(nx * ny, U), np.zeros(nx * ny)]),
                      lib=lib)
    assert np.abs(f).max() < 1e-17


def check_fa_leelin(lib):
    """F_a in Lee and Lin's form, -u div[lambda (grad P - grad p)], against
    closed forms of x-only fields, for which the isotropic D2Q9 and D3Q19
    stencils reduce to the central difference (g(x+1) - g(x-1)) / 2 and the
    three-point second difference g(x+1) + g(x-1) - 2 g(x):
    (a) at rest it is 0;  (b) in a uniform bulk (P = 0 at both minima) with
    p = b sin(kx) it is -u lambda 4 b sin^2(k/2) sin(kx), lambda = tau_g - 1/2
    in the liquid and (tau_g - 1/2) (rho_L / rho_G) / ratio in the gas;
    (c) for phi = c + a sin(kx), p = b cos(kx) it is -u [lambda lap q +
    grad lambda . grad q] with the closed forms P = beta phi^2 (phi - 1)
    (3 phi - 1) (Eq. 1a) or beta (phi^2 - phi*^2)(3 phi^2 + phi*^2) (Eq. 1b)
    and lambda = 3 mu_dyn(phi) / rho(phi);  (d) a y-only field gives no
    x-force when u is along x only through the divergence's y part."""
    nx, ny = 48, 6
    k = 2 * math.pi * 2 / nx
    for lat, nz in ((W.D2Q9, 1), (W.D3Q19, 4)):
        n = nx * ny * nz
        x = np.tile(np.arange(nx, dtype=float), ny * nz)
        dim = 2 if lat == W.D2Q9 else 3
        U = np.zeros((dim, n))
        U[0], U[1] = 0.03, -0.02
        for well, ps, (c0, c1) in ((0, 0.5, (0.0, 1.0)), (1, 0.8, (-0.8, 0.8))):
            case = _case(nx, ny, nz=nz, lattice=lat, well=well, phi_star=ps, mu_ratio=4.0,
                         tau_g=0.7)
            beta, _ = (O.beta_kappa_sym(0.01, 4.0, ps, lib) if well
                       else O.beta_kappa(0.01, 4.0, lib))
            mu_l = 1.0 * (0.7 - 0.5) / 3.0
            mu_g = mu_l / 4.0

            def lam_of(ph):
                frac = (ph - c0) / (c1 - c0)
                return 3.0 * (mu_g + frac * (mu_l - mu_g)) / (0.1 + frac * 0.9)

            def p_of(ph):
                if well:
                    return beta * (ph * ph - ps * ps) * (3 * ph * ph + ps * ps)
                return beta * ph * ph * (ph - 1.0) * (3 * ph - 1.0)

            # (a)
            phi = c0 + (c1 - c0) * (0.5 + 0.2 * np.sin(k * x))
            assert np.abs(O.fa_leelin(case, phi, np.zeros((dim, n)), np.zeros(n), lib)).max() == 0
            # (b) both bulks
            b = 3e-4
            for bulk, lam in ((c1, 0.2), (c0, 0.2 * 10.0 / 4.0)):
                f = O.fa_leelin(case, np.full(n, bulk), U, b * np.sin(k * x), lib)
                want = -U * lam * 4 * b * math.sin(k / 2) ** 2 * np.sin(k * x)
                assert np.allclose(f, want, rtol=1e-12, atol=1e-18), (lat, well, bulk)
            # (c)
            phi = 0.5 * (c0 + c1) + 0.3 * (c1 - c0) * np.sin(k * x)
            pr = b * np.cos(k * x)
            f = O.fa_leelin(case, phi, U, pr, lib)
            q = p_of(phi) - pr
            lam = lam_of(phi)

            def sh(g, d):
                return np.roll(g.reshape(-1, nx), -d, axis=1).ravel()   # g(x + d)

            div = lam * (sh(q, 1) + sh(q, -1) - 2 * q) + \
                0.25 * (sh(lam, 1) - sh(lam, -1)) * (sh(q, 1) - sh(q, -1))
            assert np.allclose(f, -U * div, rtol=1e-10, atol=1e-20), (lat, well)
            assert np.abs(div).max() > 1e-5
    # (d) y-only field: the divergence is along y only, F_a is still -u times it
    case = _case(8, 32)
    y = np.repeat(np.arange(32, dtype=float), 8)
    phi = 0.5 + 0.3 * np.sin(2 * math.pi * y / 32)
    Ux = np.vstack([np.full(256, 0.01), np.zeros(256)])
    f = O.fa_leelin(case, phi, Ux, np.zeros(256), lib)
    assert np.abs(f[1]).max() == 0.0 and np.abs(f[0]).max() > 0.0
    fx = O.fa_leelin(_case(32, 8), np.tile(0.5 + 0.3 * np.sin(2 * math.pi *
                                                             np.arange(32.0) / 32), 8),
                     Ux, np.zeros(256), lib)
    assert np.allclose(np.sort(fx[0]), np.sort(f[0]), rtol=1e-12, atol=1e-20)


def check_correction_from_data(lib):
    """remove_fa = 2: the correction -F_a = D u with the rate D = (rho^n -
    rho^(n-1)) + div(rho u_o) taken from the data.  At the populations of any
    step, the velocity it recovers equals u_o rho / (rho - D / 2), where u_o is
    the original model's velocity at the same populations (a remove_fa = 0
    dump) and D is the rate of the pinned discrete estimator fa_discrete
    (F = -u_o D) with phi^(n-1) the phi of the previous step -- at the first
    step phi^(n-1) = phi^0, so only the divergence remains; phi and the
    populations' mass are those of the original model.  D2Q9 and D3Q19."""
    c = W.stationary_droplet(seed=2, n=40, radius=9.0, noise_amp=2e-3)
    u0 = c.u0.copy()
    u0[0] += 0.02
    u0[1] -= 0.01
    _check_data_rate(lib, dict(c.params, remove_fa=2, wall=[0, 1, 0]), c.phi0, u0, c.p0)
    prm = W.base_params(W.D3Q19, 14, 12, 10, (0, 0, 1), sigma=0.01, remove_fa=2)
    rng = np.random.default_rng(3)
    phi, u, p = W.droplet_fields(prm, (6.3, 5.8, 5.1), 3.5, impact_u=0.02,
                                 noise=rng.normal(0, 2e-3, (3, 14 * 12 * 10)))
    u[0] += 0.01
    _check_data_rate(lib, prm, phi, u, p)


def _check_data_rate(lib, prm2, phi0, u0, p0):
    prm0 = dict(prm2, remove_fa=0)
    n = phi0.size

    def check(sim, phi_prev):
        got = sim.fields()
        f, g = sim.get_state()
        o = O.Sim(prm0, phi0, u0, p0, lib=lib)
        o.set_state(f, g, sim.time)
        ref = o.fields()
        assert np.array_equal(got["phi"], ref["phi"])
        uo = ref["u"]
        fd = O.fa_discrete(prm0, phi_prev, ref["phi"], uo, lib=lib)
        d = -(fd * uo).sum(axis=0) / (uo * uo).sum(axis=0)
        rho = prm2["rho_g"] + (prm2["rho_l"] - prm2["rho_g"]) * ref["phi"]
        want = uo * rho / (rho - 0.5 * d)
        assert np.allclose(got["u"], want, rtol=1e-11, atol=1e-18)
        assert np.abs(got["u"] - uo).max() > 1e-9
        return got

    s = O.Sim(prm2, phi0, u0, p0, lib=lib)
    first = check(s, s.fields()["phi"])
    s.step(6)
    prev = s.fields()["phi"]
    s.step(1)
    check(s, prev)
    assert abs(s.diag()["mass"] - first["phi"].sum()) < 1e-12 * n


def check_symmetric_well(lib):
    """The symmetric well of Eq. 1b, theta = beta (phi^2 - phi*^2)^2, with the
    density law of Eq. 4b, rho = rho_G + (phi + phi*) / (2 phi*) (rho_L - rho_G):
    (a) beta, kappa from sigma, W make phi* tanh(2z/W) solve kappa phi'' =
    theta'(phi) with tension int kappa phi'^2 dz = sigma;  (b) on a uniform
    field mu = theta'(phi) = 4 beta phi (phi^2 - phi*^2);  (c) the density of
    a uniform field moving at u gives momentum rho(phi) u N with rho = rho_L at
    phi*, rho_G at -phi*, the mean at 0;  (d) the diagnostic weight maps
    phi* (2 phi01 - 1) with phi01 = 1/4, 1/2, 3/4 to 0, 1/2, 1;  (e) resting
    droplets with phi* = 0.8 obey Young-Laplace, dp R / sigma = 1 to 5 % for
    R = 12, 16, 20 (mobility theta_M scaled by (2 phi*)^2, which keeps the
    Cahn-Hilliard relaxation rate of the phi in [0, 1] runs)."""
    from scipy.integrate import quad
    for sigma, width, ps in ((0.01, 4.0, 0.5), (0.005, 3.0, 1.0), (0.01, 4.0, 0.8)):
        beta, kappa = O.beta_kappa_sym(sigma, width, ps, lib)
        for z in np.linspace(-6, 6, 25):
            t = math.tanh(2 * z / width)
            phi = ps * t
            d2 = -8.0 * ps / width**2 * t * (1 - t * t)
            dth = 4 * beta * phi * (phi * phi - ps * ps)
            assert abs(kappa * d2 - dth) < 1e-12 * max(1.0, beta)
        tension = quad(lambda z: kappa * (2 * ps / width * (1 - math.tanh(2 * z / width) ** 2))
                       ** 2, -50, 50, epsabs=1e-14)[0]
        assert abs(tension - sigma) < 1e-9 * sigma + 1e-15
    n, ps = 8, 0.8
    case = _case(n, n, well=1, phi_star=ps, rho_l=2.0, rho_g=0.5)
    beta, _ = O.beta_kappa_sym(0.01, 4.0, ps, lib)
    for phi in (0.3, -0.6, ps, -ps, 0.0):
        s = O.Sim(case, np.full(n * n, phi), np.zeros(2 * n * n), np.zeros(n * n), lib=lib)
        mu = s.fields()["mu"]
        assert np.allclose(mu, 4 * beta * phi * (phi * phi - ps * ps), rtol=1e-13, atol=1e-18)
    for phi, rho in ((ps, 2.0), (-ps, 0.5), (0.0, 1.25), (0.4, 1.625)):
        u = np.zeros((2, n * n))
        u[0] = 0.01
        s = O.Sim(case, np.full(n * n, phi), u, np.zeros(n * n), lib=lib)
        d = s.diag()
        assert abs(d["momentum"][0] - rho * 0.01 * n * n) < 1e-13
        assert abs(d["momentum"][1]) < 1e-15
    for frac, w in ((0.25, 0.0), (0.5, 0.5), (0.75, 1.0)):
        s = O.Sim(case, np.full(n * n, ps * (2 * frac - 1)), np.zeros(2 * n * n),
                  np.zeros(n * n), lib=lib)
        assert abs(s.diag()["wsum"] - w * n * n) < 1e-12
    # under phi -> c phi the Cahn-Hilliard equation keeps its rate only if the
    # mobility scales by c^2
    radii = np.array([12.0, 16.0, 20.0])
    dps = np.array([laplace_dp(lib, r, well=1, phi_star=ps, theta_m=0.1 * (2 * ps) ** 2)
                    for r in radii])
    assert np.all(np.abs(dps * radii / 0.01 - 1) < 0.05), dps * radii


ALL_CHECKS = [check_lattice, check_feq_moments, check_geq_moments, check_source_moments,
              check_recover, check_stencil_polynomials, check_stencil_convergence,
              check_stencil_isotropy, check_mirror_ghosts, check_stencils_d3q19,
              check_chemical_potential,
              check_beta_kappa, check_stream_permutation, check_fixed_point,
              check_uniform_flow, check_conservation, check_uniform_force,
              check_shear_wave, check_ch_diffusion, check_switch_noop, check_fa_field,
              check_momentum_balance, check_correction_velocity, check_eq5_fa,
              check_advection, check_diagnostics, check_field_diag, check_spread_radius, check_fa_discrete,
              check_symmetric_well, check_fa_leelin, check_correction_from_data]
