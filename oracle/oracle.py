"""ctypes wrapper of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It holds no
arithmetic of the method; every number comes from lbm_oracle.c.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

D2Q9, D3Q19 = 0, 1


class OrcParams(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("wall", C.c_int * 3),
        ("beta", C.c_double), ("kappa", C.c_double), ("theta_m", C.c_double),
        ("tau_f", C.c_double), ("tau_g", C.c_double),
        ("rho_l", C.c_double), ("rho_g", C.c_double), ("mu_ratio", C.c_double),
        ("gravity", C.c_double), ("rho_ref", C.c_double),
        ("remove_fa", C.c_int), ("well", C.c_int), ("phi_star", C.c_double),
    ]


_lib = None
_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_UP = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def load(path=None):
    """Load (building first if needed) the oracle library."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    lib = C.CDLL(path or os.environ.get("LBM_ORACLE_LIB") or _build.ensure_built())
    P = C.POINTER(OrcParams)
    dp = C.POINTER(C.c_double)
    lib.orc_lattice.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), dp,
                                C.POINTER(C.c_int)]
    lib.orc_beta_kappa.argtypes = [C.c_double, C.c_double, dp, dp]
    lib.orc_beta_kappa_sym.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
    lib.orc_create.argtypes = [P, _DP, _DP, _DP]
    lib.orc_create.restype = C.c_void_p
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_step.argtypes = [C.c_void_p, C.c_long]
    lib.orc_time.argtypes = [C.c_void_p]
    lib.orc_time.restype = C.c_long
    lib.orc_fields.argtypes = [C.c_void_p] + [dp] * 6
    lib.orc_diag.argtypes = [C.c_void_p, _DP]
    lib.orc_get_state.argtypes = [C.c_void_p, _DP, _DP]
    lib.orc_set_state.argtypes = [C.c_void_p, _DP, _DP, C.c_long]
    lib.orc_feq.argtypes = [C.c_int, C.c_double, C.c_double, _DP, C.c_double, _DP]
    lib.orc_geq.argtypes = [C.c_int, C.c_double, C.c_double, _DP, _DP]
    lib.orc_source.argtypes = [C.c_int, _DP, _DP, _DP, _DP]
    lib.orc_recover.argtypes = [C.c_int, _DP, C.c_double, _DP, C.c_double, _DP,
                                _DP, _DP, dp]
    lib.orc_grad_lap.argtypes = [P, _DP, dp, dp]
    lib.orc_stream_words.argtypes = [P, _UP, _UP]
    lib.orc_spread_radius.argtypes = [C.c_int, C.c_int, C.c_int, _DP, C.c_double]
    lib.orc_field_diag.argtypes = [C.c_int] * 4 + [_DP, _DP] + [C.c_double] * 4 + [_DP]
    lib.orc_fa_discrete.argtypes = [P, _DP, _DP, _DP, _DP]
    lib.orc_fa_leelin.argtypes = [P, _DP, _DP, _DP, _DP]
    lib.orc_spread_radius.restype = C.c_double
    if path is None:
        _lib = lib
    return lib


def lattice(lat=D2Q9, lib=None):
    """(e[Q,3] int, w[Q] float64, opp[Q] int) of the oracle's lattice."""
    lib = lib or load()
    q = C.c_int()
    e = (C.c_int * 57)()
    w = (C.c_double * 19)()
    opp = (C.c_int * 19)()
    lib.orc_lattice(lat, C.byref(q), e, w, opp)
    n = q.value
    return (np.array(e[:3 * n], dtype=np.int64).reshape(n, 3),
            np.array(w[:n]), np.array(opp[:n], dtype=np.int64))


def spread_radius(phi, dims, level=0.5, lib=None):
    """Diagnostic D6 of a phi field (nx*ny*nz values, node order): the largest
    half-distance between the outermost phi = level crossings of a grid row
    in x (see orc_spread_radius)."""
    lib = lib or load()
    nx, ny = int(dims[0]), int(dims[1])
    nz = int(dims[2]) if len(dims) > 2 else 1
    a = np.ascontiguousarray(phi, dtype=np.float64).ravel()
    assert a.size == nx * ny * nz
    return float(lib.orc_spread_radius(nx, ny, nz, a, float(level)))


def field_diag(phi, u, dims, phi_g, phi_l, rho_g, rho_l, lib=None):
    """Diagnostics of given node fields phi [N], u [dim, N] (see
    orc_field_diag): dict of mass, momentum, wsum, centroid, centroid_vel,
    second_moment, umax, nonfinite."""
    lib = lib or load()
    dim = len(dims)
    nz = int(dims[2]) if dim == 3 else 1
    ph = np.ascontiguousarray(phi, dtype=np.float64).ravel()
    uu = np.ascontiguousarray(u, dtype=np.float64).ravel()
    assert ph.size * dim == uu.size == int(np.prod(dims)) * dim
    d = np.zeros(16)
    lib.orc_field_diag(dim, int(dims[0]), int(dims[1]), nz, ph, uu, float(phi_g), float(phi_l),
                       float(rho_g), float(rho_l), d)
    return dict(mass=d[0], momentum=d[1:4].copy(), wsum=d[4], centroid=d[5:8].copy(),
                centroid_vel=d[8:11].copy(), second_moment=d[11:14].copy(), umax=d[14],
                nonfinite=int(d[15]), slots=d)


def fa_discrete(case, phi_prev, phi, u, lib=None):
    """F_a of Eq. 12 from discrete data: -u [(rho^n - rho^(n-1)) +
    div(rho u)^n] (see orc_fa_discrete).  Returns (dim, N)."""
    lib = lib or load()
    prm = make_params(case, lib)
    n = int(np.asarray(phi).size)
    dim = 2 if case["lattice"] == D2Q9 else 3
    out = np.zeros(dim * n)
    lib.orc_fa_discrete(C.byref(prm), np.ascontiguousarray(phi_prev, dtype=np.float64).ravel(),
                        np.ascontiguousarray(phi, dtype=np.float64).ravel(),
                        np.ascontiguousarray(u, dtype=np.float64).ravel(), out)
    return out.reshape(dim, n)


def fa_leelin(case, phi, u, p, lib=None):
    """F_a of Eq. 12 in Lee and Lin's form (Eq. 11): -u div[lambda (grad P -
    grad p)] (see orc_fa_leelin).  Returns (dim, N)."""
    lib = lib or load()
    prm = make_params(case, lib)
    n = int(np.asarray(phi).size)
    dim = 2 if case["lattice"] == D2Q9 else 3
    out = np.zeros(dim * n)
    lib.orc_fa_leelin(C.byref(prm), np.ascontiguousarray(phi, dtype=np.float64).ravel(),
                      np.ascontiguousarray(u, dtype=np.float64).ravel(),
                      np.ascontiguousarray(p, dtype=np.float64).ravel(), out)
    return out.reshape(dim, n)


def beta_kappa(sigma, width, lib=None):
    lib = lib or load()
    b, k = C.c_double(), C.c_double()
    lib.orc_beta_kappa(sigma, width, C.byref(b), C.byref(k))
    return b.value, k.value


def beta_kappa_sym(sigma, width, phi_star, lib=None):
    """beta, kappa of the symmetric well (Eq. 1b) for tension sigma and
    width W (orc_beta_kappa_sym)."""
    lib = lib or load()
    b, k = C.c_double(), C.c_double()
    lib.orc_beta_kappa_sym(sigma, width, phi_star, C.byref(b), C.byref(k))
    return b.value, k.value


def make_params(case, lib=None):
    """OrcParams from a case dict (keys as produced by workloads.Case.params).

    beta and kappa are derived here from sigma and W by the oracle's own
    formula unless the dict gives them directly."""
    p = OrcParams()
    well = int(case.get("well", 0))
    if "beta" not in case:
        if well:
            b, k = beta_kappa_sym(case["sigma"], case["width"], case["phi_star"], lib)
        else:
            b, k = beta_kappa(case["sigma"], case["width"], lib)
        case = dict(case, beta=b, kappa=k)
    p.lattice = case["lattice"]
    p.nx, p.ny, p.nz = case["nx"], case["ny"], case.get("nz", 1)
    for a in range(3):
        p.wall[a] = case["wall"][a]
    for k in ("beta", "kappa", "theta_m", "tau_f", "tau_g", "rho_l", "rho_g",
              "mu_ratio", "gravity", "rho_ref"):
        setattr(p, k, float(case[k]))
    p.remove_fa = int(case["remove_fa"])
    p.well = well
    p.phi_star = float(case.get("phi_star", 0.5))
    return p


def _vec(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.size == n, (a.size, n)
    return a


def _f3(v):
    return _vec(np.resize(np.asarray(v, float), 3), 3)


def feq(phi, mu, u, gamma, lat=D2Q9, lib=None):
    lib = lib or load()
    e, _, _ = lattice(lat, lib)
    out = np.zeros(len(e))
    lib.orc_feq(lat, phi, mu, _f3(u), gamma, out)
    return out


def geq(p, rho, u, lat=D2Q9, lib=None):
    lib = lib or load()
    e, _, _ = lattice(lat, lib)
    out = np.zeros(len(e))
    lib.orc_geq(lat, p, rho, _f3(u), out)
    return out


def source(u, force, gradpsi, lat=D2Q9, lib=None):
    lib = lib or load()
    e, _, _ = lattice(lat, lib)
    out = np.zeros(len(e))
    lib.orc_source(lat, _f3(u), _f3(force), _f3(gradpsi), out)
    return out


def recover(gbar, rho, fsg, c, gradrho, lat=D2Q9, lib=None):
    lib = lib or load()
    u = np.zeros(3)
    force = np.zeros(3)
    p = C.c_double()
    lib.orc_recover(lat, _vec(gbar, len(gbar)), rho, _f3(fsg), c, _f3(gradrho), u,
                    force, C.byref(p))
    return u, force, p.value


def grad_lap(case, field, lib=None):
    """Isotropic gradient (dim, N) and Laplacian (N) of a field on a case grid."""
    lib = lib or load()
    prm = make_params(case, lib)
    n = prm.nx * prm.ny * prm.nz
    dim = 2 if prm.lattice == D2Q9 else 3
    grad = np.zeros(dim * n)
    lap = np.zeros(n)
    lib.orc_grad_lap(C.byref(prm), _vec(field, n),
                     grad.ctypes.data_as(C.POINTER(C.c_double)),
                     lap.ctypes.data_as(C.POINTER(C.c_double)))
    return grad.reshape(dim, n), lap


def stream_words(case, words, lib=None):
    """One streaming pass over uint32 words laid out [Q, N]."""
    lib = lib or load()
    prm = make_params(case, lib)
    w = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.zeros_like(w)
    lib.orc_stream_words(C.byref(prm), w.ravel(), out.ravel())
    return out


class Sim:
    """One oracle simulation.  case: parameter dict; phi0[N], u0[dim, N], p0[N]."""

    def __init__(self, case, phi0, u0, p0, lib=None):
        self.lib = lib or load()
        self.prm = make_params(case, self.lib)
        self.n = self.prm.nx * self.prm.ny * self.prm.nz
        self.dim = 2 if self.prm.lattice == D2Q9 else 3
        self.q = 9 if self.prm.lattice == D2Q9 else 19
        h = self.lib.orc_create(C.byref(self.prm), _vec(phi0, self.n),
                                _vec(u0, self.dim * self.n), _vec(p0, self.n))
        if not h:
            raise ValueError("oracle rejected the case parameters")
        self.h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    @property
    def time(self):
        return self.lib.orc_time(self.h)

    def step(self, n):
        self.lib.orc_step(self.h, int(n))

    def fields(self):
        n, dim = self.n, self.dim
        out = dict(phi=np.zeros(n), u=np.zeros(dim * n), p=np.zeros(n), mu=np.zeros(n),
                   lapmu=np.zeros(n), fa=np.zeros(dim * n))
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        self.lib.orc_fields(self.h, dp(out["phi"]), dp(out["u"]), dp(out["p"]),
                            dp(out["mu"]), dp(out["lapmu"]), dp(out["fa"]))
        out["u"] = out["u"].reshape(dim, n)
        out["fa"] = out["fa"].reshape(dim, n)
        return out

    def diag(self):
        d = np.zeros(20)
        self.lib.orc_diag(self.h, d)
        return dict(mass=d[0], mass0=d[1], momentum=d[2:5].copy(), wsum=d[5],
                    centroid=d[6:9].copy(), centroid_vel=d[9:12].copy(),
                    second_moment=d[12:15].copy(), umax=d[15], nonfinite=int(d[16]))

    def get_state(self):
        f = np.zeros(self.q * self.n)
        g = np.zeros(self.q * self.n)
        self.lib.orc_get_state(self.h, f, g)
        return f.reshape(self.q, self.n), g.reshape(self.q, self.n)

    def set_state(self, f, g, time):
        self.lib.orc_set_state(self.h, _vec(f, self.q * self.n), _vec(g, self.q * self.n),
                               int(time))
