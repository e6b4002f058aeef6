"""The allocation-free diagnostics entry point (lbm_field_diagnostics_noalloc,
whose partial sums live in a device array the library holds per GPU) against
lbm_field_diagnostics with a caller workspace, through the C ABI: two calls in
a row, the second on a smaller grid, each bit-identical to the workspace form
(the same kernels in the same fixed reduction order) and within rounding of
the oracle's definition of the diagnostics."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hip():
    import torch
    assert torch.cuda.is_available()
    import paper_1110_5004_amd as P
    return P


def fields(dims, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    axes = np.meshgrid(*[np.arange(d, dtype=np.float64) for d in reversed(dims)], indexing="ij")
    pos = [a.ravel() for a in reversed(axes)]
    r = np.sqrt(sum((p - 0.41 * d) ** 2 for p, d in zip(pos, dims)))
    phi = 0.5 + 0.5 * np.tanh(2.0 * (0.25 * min(dims) - r) / 4.0) + 1e-3 * rng.standard_normal(n)
    u = 0.03 * rng.standard_normal((len(dims), n))
    return phi.astype(np.float32), u.astype(np.float32)


def test_noalloc_matches_workspace_form_twice(hip):
    import torch
    out = torch.empty(hip.binding.DIAG_SLOTS, dtype=torch.float64, device="cuda")
    ws = torch.empty(hip.binding.DIAG_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda")
    ref_out = torch.empty_like(out)
    for dims, seed in (((96, 80, 40), 1), ((33, 17), 2)):  # the second call smaller
        phi, u = fields(dims, seed)
        dphi, du = torch.from_numpy(phi).cuda(), torch.from_numpy(u).cuda()
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        hip.field_diagnostics_noalloc(dphi, du, dims, 0.0, 1.0, 0.1, 1.0, out)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        got = out.cpu().numpy().copy()
        hip.field_diagnostics(dphi, du, dims, 0.0, 1.0, 0.1, 1.0, out=ref_out, workspace=ws)
        assert np.array_equal(got, ref_out.cpu().numpy()), (dims, got, ref_out.cpu().numpy())
        ref = O.field_diag(phi.astype(np.float64), u.astype(np.float64), dims, 0.0, 1.0, 0.1, 1.0)
        assert np.allclose(got[:14], ref["slots"][:14], rtol=1e-12, atol=1e-12 * ref["mass"])
        assert got[14] == pytest.approx(ref["umax"], rel=1e-15) and got[15] == ref["nonfinite"]


def test_noalloc_rejects_bad_arguments(hip):
    import torch
    phi = torch.zeros(64, device="cuda")
    u = torch.zeros(2 * 64, device="cuda")
    out = torch.empty(hip.binding.DIAG_SLOTS, dtype=torch.float64, device="cuda")
    with pytest.raises(hip.LbmError):
        hip.field_diagnostics_noalloc(phi, u, (8, 8), 0.5, 0.5, 0.1, 1.0, out)
    rc = hip.binding.lib().lbm_field_diagnostics_noalloc(5, 8, 8, 1, phi.data_ptr(), u.data_ptr(),
                                                         0.0, 1.0, 0.1, 1.0, out.data_ptr(), None)
    assert rc == hip.binding.ERR_ARG
