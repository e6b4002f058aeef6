"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the lattice Boltzmann path runs in the gfx950 library
_build/liblbm_hip.so.  PyTorch supplies the device arena and the HIP stream.
There is no fallback: without the built library or a GPU, the calls raise.
"""
import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_HIP_LIB selects another build of the same library (the host-sanitizer
# build of build.py, say)
LIB_PATH = os.environ.get("LBM_HIP_LIB") or os.path.join(HERE, "_build", "liblbm_hip.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

D2Q9, D3Q19 = 0, 1
PERIODIC, WALL = 0, 1
FP32, FP16, BF16 = 0, 1, 2
STORAGE = {"fp32": FP32, "fp16": FP16, "bf16": BF16}

OK, ERR_ARG, ERR_HIP, ERR_NONFINITE, ERR_STATE, ERR_OOM = 0, -1, -2, -3, -4, -5


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class CaseParams(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 3),
        ("beta", C.c_double), ("kappa", C.c_double), ("theta_m", C.c_double),
        ("tau_f", C.c_double), ("tau_g", C.c_double), ("rho_l", C.c_double),
        ("rho_g", C.c_double), ("mu_ratio", C.c_double), ("gravity", C.c_double),
        ("rho_ref", C.c_double), ("remove_fa", C.c_int32), ("storage", C.c_int32),
        ("p0", C.c_double), ("scale_f", C.c_double), ("scale_g", C.c_double),
        ("well", C.c_int32), ("phi_star", C.c_double),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("mass", C.c_double), ("mass0", C.c_double),
        ("mass_drift_rel", C.c_double), ("momentum", C.c_double * 3), ("wsum", C.c_double),
        ("centroid", C.c_double * 3), ("centroid_vel", C.c_double * 3),
        ("second_moment", C.c_double * 3), ("umax", C.c_double), ("nonfinite", C.c_int64),
    ]

    def to_dict(self):
        return dict(step=self.step, mass=self.mass, mass0=self.mass0,
                    mass_drift_rel=self.mass_drift_rel, momentum=np.array(self.momentum[:]),
                    wsum=self.wsum, centroid=np.array(self.centroid[:]),
                    centroid_vel=np.array(self.centroid_vel[:]),
                    second_moment=np.array(self.second_moment[:]), umax=self.umax,
                    nonfinite=self.nonfinite)


_lib = None
_vp = C.c_void_p


def lib():
    """The loaded gfx950 library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "python paper_1110_5004_amd/build.py (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    fp = C.POINTER(C.c_float)
    i32p = C.POINTER(C.c_int32)
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_beta_kappa.argtypes = [C.c_double, C.c_double, dp, dp]
    L.lbm_beta_kappa_sym.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
    L.lbm_required_bytes.argtypes = [C.POINTER(CaseParams), C.c_int32, C.POINTER(C.c_size_t)]
    L.lbm_init.argtypes = [C.POINTER(CaseParams), C.c_int32, C.POINTER(dp), C.POINTER(dp),
                           C.POINTER(dp), _vp, C.c_size_t, _vp, C.c_int32, C.POINTER(_vp)]
    L.lbm_step.argtypes = [_vp, C.c_int64]
    L.lbm_prepare.argtypes = [_vp]
    L.lbm_moments.argtypes = [_vp, C.c_int32, fp, fp, fp, fp, fp]
    L.lbm_moments_device.argtypes = [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp]
    L.lbm_diagnostics.argtypes = [_vp, C.c_int32, C.POINTER(Diag)]
    L.lbm_spread_radius.argtypes = [_vp, C.c_int32, C.c_double, C.POINTER(C.c_double)]
    L.lbm_fa_discrete.argtypes = [_vp, C.c_int32, _vp, _vp]
    L.lbm_fa_leelin.argtypes = [_vp, C.c_int32, _vp]
    L.lbm_info.argtypes = [_vp, i32p, C.POINTER(C.c_int64), i32p]
    L.lbm_state_bytes.argtypes = [_vp, C.c_int32, C.POINTER(C.c_size_t)]
    L.lbm_get_state.argtypes = [_vp, C.c_int32, _vp, C.c_size_t]
    L.lbm_set_state.argtypes = [_vp, C.c_int32, _vp, C.c_size_t]
    L.lbm_set_step.argtypes = [_vp, C.c_int64]
    L.lbm_set_launch.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32]
    L.lbm_get_launch.argtypes = [_vp, i32p, i32p, i32p]
    L.lbm_variant_count.argtypes = [C.c_int32, i32p]
    L.lbm_variant_info.argtypes = [C.c_int32, C.c_int32, i32p, i32p, i32p, i32p]
    L.lbm_variant_form.argtypes = [C.c_int32, C.c_int32, i32p]
    L.lbm_free.argtypes = [_vp]
    L.lbm_free.restype = None
    L.lbm_stream_words.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, i32p, _vp, _vp,
                                   _vp]
    L.lbm_encode16.argtypes = [C.c_int32, _vp, _vp, C.c_int64, _vp]
    L.lbm_encode16_stochastic.argtypes = [C.c_int32, _vp, _vp, C.c_int64, C.c_uint32, C.c_int32,
                                          _vp]
    L.lbm_copy_bw.argtypes = [_vp, _vp, C.c_int64, _vp]
    L.lbm_pull_copy_bw.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp,
                                   _vp, _vp]
    L.lbm_field_diagnostics.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp, _vp,
                                        C.c_double, C.c_double, C.c_double, C.c_double, _vp,
                                        _vp, C.c_size_t, _vp]
    L.lbm_field_diagnostics_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                                _vp, _vp, C.c_double, C.c_double, C.c_double,
                                                C.c_double, _vp, _vp]
    _lib = L
    return L


def declared_functions():
    """Names of the functions include/lbm.h declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def _check(rc):
    if rc != OK:
        raise LbmError(rc, lib().lbm_last_error().decode())
    return rc


def beta_kappa(sigma, width):
    b, k = C.c_double(), C.c_double()
    _check(lib().lbm_beta_kappa(sigma, width, C.byref(b), C.byref(k)))
    return b.value, k.value


def beta_kappa_sym(sigma, width, phi_star):
    b, k = C.c_double(), C.c_double()
    _check(lib().lbm_beta_kappa_sym(sigma, width, phi_star, C.byref(b), C.byref(k)))
    return b.value, k.value


def make_case(params, storage=FP32, p0=0.0, scale_f=0.0, scale_g=0.0):
    """CaseParams from a parameter dict (sigma and width, or beta and kappa;
    well 0 = asymmetric, 1 = symmetric with phi_star)."""
    c = CaseParams()
    c.lattice = params["lattice"]
    c.nx, c.ny, c.nz = params["nx"], params["ny"], params.get("nz", 1)
    for a in range(3):
        c.bc[a] = params["wall"][a]
    c.well = int(params.get("well", 0))
    c.phi_star = float(params.get("phi_star", 0.5))
    if "beta" in params:
        c.beta, c.kappa = params["beta"], params["kappa"]
    elif c.well:
        c.beta, c.kappa = beta_kappa_sym(params["sigma"], params["width"], c.phi_star)
    else:
        c.beta, c.kappa = beta_kappa(params["sigma"], params["width"])
    for k in ("theta_m", "tau_f", "tau_g", "rho_l", "rho_g", "mu_ratio", "gravity", "rho_ref"):
        setattr(c, k, float(params[k]))
    c.remove_fa = int(params["remove_fa"])
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.p0, c.scale_f, c.scale_g = p0, scale_f, scale_g
    return c


def _stream_handle(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Simulation:
    """Cases advancing together on one GPU (one fused launch per time step).

    cases: list of (params dict, phi0[N], u0[dim, N], p0[N]) or objects with
    .params/.phi0/.u0/.p0.  The device arena is a torch uint8 tensor."""

    def __init__(self, cases, storage="fp32", check_every=0, device="cuda:0", p0=0.0,
                 scale_f=0.0, scale_g=0.0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Simulation needs a GPU (no CPU fallback)")
        self.torch = torch
        self.device = torch.device(device)
        self.storage_name = storage if isinstance(storage, str) else \
            {v: k for k, v in STORAGE.items()}[int(storage)]
        L = lib()
        cases = [(c.params, c.phi0, c.u0, c.p0) if hasattr(c, "params") else c for c in cases]
        self.n_cases = len(cases)
        self.params = [c[0] for c in cases]
        self.dims = [(p["nx"], p["ny"], p.get("nz", 1)) for p in self.params]
        self.dim = 2 if self.params[0]["lattice"] == D2Q9 else 3
        arr = (CaseParams * self.n_cases)(*[make_case(p, storage, p0, scale_f, scale_g)
                                            for p in self.params])
        self._cparams = arr
        nbytes = C.c_size_t()
        _check(L.lbm_required_bytes(arr, self.n_cases, C.byref(nbytes)))
        with torch.cuda.device(self.device):
            self.arena = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._host = []
        dp = C.POINTER(C.c_double)

        def ptrs(idx, shape_fn):
            out = (dp * self.n_cases)()
            for k, c in enumerate(cases):
                a = np.ascontiguousarray(c[idx], dtype=np.float64).ravel()
                n = int(np.prod(self.dims[k]))
                assert a.size == shape_fn(n), (a.size, n)
                self._host.append(a)
                out[k] = a.ctypes.data_as(dp)
            return out

        phi = ptrs(1, lambda n: n)
        u = ptrs(2, lambda n: self.dim * n)
        pr = ptrs(3, lambda n: n)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.lbm_init(arr, self.n_cases, phi, u, pr, C.c_void_p(aligned),
                              nbytes.value, _stream_handle(torch, self.device), check_every,
                              C.byref(h)))
        self._host = []
        self.h = h

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            lib().lbm_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n_nodes(self, icase=0):
        return int(np.prod(self.dims[icase]))

    def step(self, n):
        _check(lib().lbm_step(self.h, int(n)))

    def prepare(self):
        """Capture the step graph of the current launch shape now (lbm_prepare),
        so that timed steps replay it without a capture."""
        _check(lib().lbm_prepare(self.h))

    @property
    def time(self):
        s = C.c_int64()
        _check(lib().lbm_info(self.h, None, C.byref(s), None))
        return s.value

    def moments(self, icase=0):
        """Host fields: phi[N], u[dim, N], p[N], mu[N], fa[dim, N] (float32)."""
        n, d = self.n_nodes(icase), self.dim
        out = dict(phi=np.empty(n, np.float32), u=np.empty(d * n, np.float32),
                   p=np.empty(n, np.float32), mu=np.empty(n, np.float32),
                   fa=np.empty(d * n, np.float32))
        fp = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))
        _check(lib().lbm_moments(self.h, icase, fp(out["phi"]), fp(out["u"]), fp(out["p"]),
                                 fp(out["mu"]), fp(out["fa"])))
        out["u"] = out["u"].reshape(d, n)
        out["fa"] = out["fa"].reshape(d, n)
        return out

    def moments_device(self, icase=0):
        """Device fields as torch float32 tensors (no host copy)."""
        t = self.torch
        n, d = self.n_nodes(icase), self.dim
        out = {k: t.empty(s, dtype=t.float32, device=self.device)
               for k, s in (("phi", n), ("u", d * n), ("p", n), ("mu", n), ("fa", d * n))}
        v = lambda k: C.c_void_p(out[k].data_ptr())
        _check(lib().lbm_moments_device(self.h, icase, v("phi"), v("u"), v("p"), v("mu"),
                                        v("fa")))
        out["u"] = out["u"].view(d, n)
        out["fa"] = out["fa"].view(d, n)
        return out

    def diagnostics(self, icase=0):
        d = Diag()
        _check(lib().lbm_diagnostics(self.h, icase, C.byref(d)))
        return d.to_dict()

    def fa_discrete(self, phi_prev, icase=0):
        """F_a from discrete data (see lbm_fa_discrete): phi_prev is a device
        float32 tensor of phi one step earlier; returns a (dim, N) device
        tensor."""
        t = self.torch
        n = self.n_nodes(icase)
        out = t.empty(self.dim * n, dtype=t.float32, device=self.device)
        _check(lib().lbm_fa_discrete(self.h, icase, C.c_void_p(phi_prev.data_ptr()),
                                     C.c_void_p(out.data_ptr())))
        return out.view(self.dim, n)

    def fa_leelin(self, icase=0):
        """F_a in Lee and Lin's form (see lbm_fa_leelin) on the current
        fields; returns a (dim, N) device tensor."""
        t = self.torch
        n = self.n_nodes(icase)
        out = t.empty(self.dim * n, dtype=t.float32, device=self.device)
        _check(lib().lbm_fa_leelin(self.h, icase, C.c_void_p(out.data_ptr())))
        return out.view(self.dim, n)

    def spread_radius(self, icase=0, level=None):
        """Largest half-distance between the outermost phi = level crossings
        of a grid row in x (the droplet half-width of the paper's Fig. 5);
        level defaults to the interface midpoint of the case's well (1/2, or
        0 for the symmetric well)."""
        if level is None:
            level = 0.0 if self.params[icase].get("well", 0) else 0.5
        r = C.c_double()
        _check(lib().lbm_spread_radius(self.h, icase, float(level), C.byref(r)))
        return r.value

    def state_bytes(self, icase=0):
        b = C.c_size_t()
        _check(lib().lbm_state_bytes(self.h, icase, C.byref(b)))
        return b.value

    def get_state(self, icase=0):
        buf = np.empty(self.state_bytes(icase), np.uint8)
        _check(lib().lbm_get_state(self.h, icase, buf.ctypes.data_as(C.c_void_p), buf.size))
        return buf

    def set_state(self, buf, icase=0, step=None):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().lbm_set_state(self.h, icase, buf.ctypes.data_as(C.c_void_p), buf.size))
        if step is not None:
            _check(lib().lbm_set_step(self.h, int(step)))

    def set_launch(self, variant=0, grid_blocks=0, graph_steps=16):
        _check(lib().lbm_set_launch(self.h, variant, grid_blocks, graph_steps))

    def get_launch(self):
        v, g, s = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lbm_get_launch(self.h, C.byref(v), C.byref(g), C.byref(s)))
        return v.value, g.value, s.value


FORM_THREE, FORM_FUSED, FORM_TWO = 0, 1, 2


def variants(lattice=D2Q9):
    """[(tx, ty, tz, threads, form)] of the compiled tile shapes (form: the
    D3Q19 step form, FORM_THREE / FORM_FUSED / FORM_TWO; 0 for D2Q9)."""
    n = C.c_int32()
    _check(lib().lbm_variant_count(lattice, C.byref(n)))
    out = []
    for v in range(n.value):
        tx, ty, tz, nt, fm = (C.c_int32() for _ in range(5))
        _check(lib().lbm_variant_info(lattice, v, C.byref(tx), C.byref(ty), C.byref(tz),
                                      C.byref(nt)))
        _check(lib().lbm_variant_form(lattice, v, C.byref(fm)))
        out.append((tx.value, ty.value, tz.value, nt.value, fm.value))
    return out


def stream_words(lattice, dims, bc, words_in, words_out):
    """One device streaming pass over int32/uint32 torch tensors [Q, N]."""
    import torch
    bc_arr = (C.c_int32 * 3)(*bc)
    _check(lib().lbm_stream_words(lattice, dims[0], dims[1], dims[2], bc_arr,
                                  C.c_void_p(words_in.data_ptr()),
                                  C.c_void_p(words_out.data_ptr()),
                                  _stream_handle(torch, words_in.device)))


def encode16(storage, x):
    """16-bit encodings (as an int16 tensor of the same bits) of a float32 tensor."""
    import torch
    out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(lib().lbm_encode16(STORAGE[storage] if isinstance(storage, str) else storage,
                              C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), x.numel(),
                              _stream_handle(torch, x.device)))
    return out


def encode16_stochastic(storage, x, step, direction=0):
    """The step's stochastic 16-bit rounding of a float32 tensor (element k as
    node k), as an int16 tensor of the same bits."""
    import torch
    out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(lib().lbm_encode16_stochastic(STORAGE[storage] if isinstance(storage, str) else storage,
                                         C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                         x.numel(), step, direction,
                                         _stream_handle(torch, x.device)))
    return out


def pull_copy_bytes(lattice, storage, dims):
    """Bytes of one state copy with plane stride nx*ny*nz (see lbm_pull_copy_bw)."""
    q = 9 if lattice == D2Q9 else 19
    n = int(np.prod(dims))
    st = STORAGE[storage] if isinstance(storage, str) else storage
    return n * (8 * q + 2 if st == STORAGE["fp32"] else 4 * q + 2)


def pull_copy_bw(lattice, storage, dims, src, dst):
    """The step's pull traffic without arithmetic, src -> dst (uint8 device
    tensors of pull_copy_bytes bytes)."""
    import torch
    st = STORAGE[storage] if isinstance(storage, str) else storage
    nz = dims[2] if len(dims) > 2 else 1
    _check(lib().lbm_pull_copy_bw(lattice, st, dims[0], dims[1], nz, C.c_void_p(src.data_ptr()),
                                  C.c_void_p(dst.data_ptr()), _stream_handle(torch, src.device)))


def copy_bw(x, y):
    import torch
    _check(lib().lbm_copy_bw(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), x.numel(),
                             _stream_handle(torch, x.device)))


DIAG_SLOTS = 16
DIAG_WORKSPACE_BYTES = 65536


def _diag_fields(phi, u, dims):
    dim = len(dims)
    n = int(np.prod(dims))
    if phi.numel() != n or u.numel() != dim * n or phi.dtype != u.dtype:
        raise ValueError("phi must hold N floats and u dim*N floats (N = prod(dims))")
    nz = dims[2] if dim == 3 else 1
    return dim, nz


def field_diagnostics(phi, u, dims, phi_g, phi_l, rho_g, rho_l, out=None, workspace=None):
    """lbm_field_diagnostics on device float32 tensors phi [N] and u [dim, N]
    of a grid dims = (nx, ny[, nz]); returns the float64 device tensor of the
    LBM_DIAG_* slots (out, or a new one).  workspace: a device tensor of at
    least DIAG_WORKSPACE_BYTES (a new one when None)."""
    import torch
    dim, nz = _diag_fields(phi, u, dims)
    if out is None:
        out = torch.empty(DIAG_SLOTS, dtype=torch.float64, device=phi.device)
    if workspace is None:
        workspace = torch.empty(DIAG_WORKSPACE_BYTES, dtype=torch.uint8, device=phi.device)
    _check(lib().lbm_field_diagnostics(
        dim, dims[0], dims[1], nz, C.c_void_p(phi.data_ptr()), C.c_void_p(u.data_ptr()),
        phi_g, phi_l, rho_g, rho_l, C.c_void_p(out.data_ptr()),
        C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
        _stream_handle(torch, phi.device)))
    return out


def field_diagnostics_noalloc(phi, u, dims, phi_g, phi_l, rho_g, rho_l, out):
    """lbm_field_diagnostics_noalloc: as field_diagnostics, into the caller's
    float64 device tensor out [DIAG_SLOTS], with no workspace (the library's
    own per-GPU partial-sum array; overlapping calls on one GPU race)."""
    import torch
    dim, nz = _diag_fields(phi, u, dims)
    if out.dtype != torch.float64 or out.numel() < DIAG_SLOTS or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of DIAG_SLOTS values")
    _check(lib().lbm_field_diagnostics_noalloc(
        dim, dims[0], dims[1], nz, C.c_void_p(phi.data_ptr()), C.c_void_p(u.data_ptr()),
        phi_g, phi_l, rho_g, rho_l, C.c_void_p(out.data_ptr()),
        _stream_handle(torch, phi.device)))
    return out
