"""CPU checks of the boundary: the library loads without a GPU and exports
every function include/lbm.h declares; argument errors come back as status
codes before any device work."""
import ctypes as C

import pytest

from paper_1110_5004_amd import binding as B


@pytest.fixture(scope="module")
def L():
    return B.lib()


def test_every_declared_symbol_is_exported(L):
    names = B.declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_beta_kappa(L):
    b, k = B.beta_kappa(0.01, 4.0)
    assert abs(b - 0.03) < 1e-15 and abs(k - 0.06) < 1e-15
    with pytest.raises(B.LbmError):
        B.beta_kappa(0.01, 0.0)


def test_beta_kappa_sym(L):
    # phi* = 1: beta = 3 sigma / (4 W), kappa = 3 sigma W / 8
    b, k = B.beta_kappa_sym(0.01, 4.0, 1.0)
    assert abs(b - 0.001875) < 1e-16 and abs(k - 0.015) < 1e-16
    # phi* = 1/2 maps phi in [-1/2, 1/2] onto the asymmetric well's [0, 1]:
    # same beta and kappa
    assert B.beta_kappa_sym(0.01, 4.0, 0.5) == pytest.approx(B.beta_kappa(0.01, 4.0), rel=1e-15)
    for bad in ((0.01, 4.0, 0.0), (0.01, 0.0, 1.0), (-1.0, 4.0, 1.0)):
        with pytest.raises(B.LbmError):
            B.beta_kappa_sym(*bad)


def _params(**kw):
    p = dict(lattice=0, nx=16, ny=16, nz=1, wall=[0, 0, 0], sigma=0.01, width=4.0,
             theta_m=0.1, tau_f=0.8, tau_g=0.8, rho_l=1.0, rho_g=0.1, mu_ratio=10.0,
             gravity=0.0, rho_ref=0.1, remove_fa=0)
    p.update(kw)
    return p


@pytest.mark.parametrize("bad", [dict(tau_f=0.5), dict(tau_g=0.3), dict(rho_g=0.0),
                                 dict(nx=3), dict(nz=2),
                                 dict(wall=[0, 2, 0]), dict(mu_ratio=-1.0),
                                 dict(theta_m=float("nan")), dict(well=2), dict(remove_fa=3),
                                 dict(well=1, phi_star=0.0, beta=0.01, kappa=0.01),
                                 dict(well=1, phi_star=float("inf"), beta=0.01, kappa=0.01)])
def test_invalid_parameters_rejected(L, bad):
    c = B.make_case(_params(**bad))
    nbytes = C.c_size_t()
    rc = L.lbm_required_bytes(C.byref(c), 1, C.byref(nbytes))
    assert rc == B.ERR_ARG
    assert L.lbm_last_error()


def test_required_bytes_grows_with_storage(L):
    sizes = {}
    for st in ("fp32", "fp16"):
        c = B.make_case(_params(nx=256, ny=256), storage=st)
        nbytes = C.c_size_t()
        assert L.lbm_required_bytes(C.byref(c), 1, C.byref(nbytes)) == 0
        sizes[st] = nbytes.value
    # two copies of 18 x 4 + 2 (FP32, f_0 carries a BF16 low part) or
    # 4 + 17 x 2 (16-bit) bytes per node
    assert sizes["fp32"] - sizes["fp16"] == 2 * (74 - 38) * 256 * 256


def test_variants_listed(L):
    v = B.variants(B.D2Q9)
    assert len(v) >= 2 and all(t[2] == 1 and t[4] == 0 for t in v)


def test_variant_forms(L):
    """Every D3Q19 step form is compiled; the three-kernel variants name a
    fields tile below 16 planes, the marching forms a z chunk of 16 or more;
    bad arguments are rejected."""
    v = B.variants(B.D3Q19)
    forms = {t[4] for t in v}
    assert forms == {B.FORM_THREE, B.FORM_FUSED, B.FORM_TWO}
    assert v[1][4] == B.FORM_THREE
    assert all((t[2] < 16) == (t[4] == B.FORM_THREE) for t in v)
    assert all(t[0] * t[1] == t[3] for t in v if t[4] != B.FORM_THREE)
    f = C.c_int32()
    assert L.lbm_variant_form(B.D3Q19, len(v), C.byref(f)) == B.ERR_ARG
    assert L.lbm_variant_form(B.D3Q19, -1, C.byref(f)) == B.ERR_ARG
    assert L.lbm_variant_form(7, 0, C.byref(f)) == B.ERR_ARG
    assert L.lbm_variant_form(B.D3Q19, 0, None) == B.ERR_ARG


def test_correction_modes_not_mixed(L):
    """remove_fa = 2 keeps an extra phi plane in the state, so a handle holds
    either only remove_fa = 2 cases or none."""
    arr = (B.CaseParams * 2)(B.make_case(_params(remove_fa=2)), B.make_case(_params(remove_fa=1)))
    nbytes = C.c_size_t()
    assert L.lbm_required_bytes(arr, 2, C.byref(nbytes)) == B.ERR_ARG
    arr = (B.CaseParams * 2)(B.make_case(_params(remove_fa=2)), B.make_case(_params(remove_fa=2)))
    assert L.lbm_required_bytes(arr, 2, C.byref(nbytes)) == 0
    one = C.c_size_t()
    c1 = B.make_case(_params(remove_fa=1))
    assert L.lbm_required_bytes(C.byref(c1), 1, C.byref(one)) == 0
    two = C.c_size_t()
    c2 = B.make_case(_params(remove_fa=2))
    assert L.lbm_required_bytes(C.byref(c2), 1, C.byref(two)) == 0
    # two copies, each with one more float plane (16 x 16 nodes, padded to 256)
    assert two.value - one.value == 2 * 4 * 256


def test_copy_over_4gib_rejected(L):
    """Kernels address a state copy with 32-bit byte offsets: 8192 x 7000 D2Q9
    nodes at 74 B fit, 8192 x 7100 do not (nor 8192 x 7000 with the extra
    phi plane of the correction from data, 78 B)."""
    nbytes = C.c_size_t()
    ok = B.make_case(_params(nx=8192, ny=7000))
    assert L.lbm_required_bytes(C.byref(ok), 1, C.byref(nbytes)) == 0
    for kw in (dict(ny=7100), dict(ny=7000, remove_fa=2)):
        c = B.make_case(_params(nx=8192, **kw))
        assert L.lbm_required_bytes(C.byref(c), 1, C.byref(nbytes)) == B.ERR_ARG
        assert "4 GiB" in L.lbm_last_error().decode()


def test_empty_case_list_rejected(L):
    """No cases, or no case array, is an argument error, not an empty handle."""
    c = B.make_case(_params())
    nbytes = C.c_size_t()
    assert L.lbm_required_bytes(C.byref(c), 0, C.byref(nbytes)) == B.ERR_ARG
    assert L.lbm_required_bytes(None, 1, C.byref(nbytes)) == B.ERR_ARG
    assert L.lbm_last_error()


def test_field_diagnostics_rejects_bad_arguments(L):
    """Argument errors of lbm_field_diagnostics come back before any device
    work (the pointers below are never dereferenced)."""
    p = C.c_void_p(4096)
    ws = B.DIAG_WORKSPACE_BYTES
    good = (2, 8, 8, 1, p, p, 0.0, 1.0, 0.1, 1.0, p, p, ws, None)
    bad = [dict(i=0, v=4), dict(i=1, v=0), dict(i=4, v=None), dict(i=5, v=None),
           dict(i=10, v=None), dict(i=11, v=None), dict(i=12, v=ws - 8),
           dict(i=11, v=C.c_void_p(4097)), dict(i=7, v=0.0), dict(i=8, v=float("nan")),
           dict(i=2, v=1 << 16)]
    for b in bad:
        args = list(good)
        args[b["i"]] = b["v"]
        if b["i"] == 2:
            args[0], args[1], args[3] = 3, 1 << 16, 1 << 16  # 2^48 nodes
        assert L.lbm_field_diagnostics(*args) == B.ERR_ARG, b
