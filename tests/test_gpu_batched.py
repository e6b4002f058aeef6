"""Batched ensemble: 64 independent periodic droplet cases of 64^2 .. 512^2
with seed-drawn radius, density ratio, surface tension and gravity advance in
one launch per time step (HIP-graph replayed).  Each case must match its own
single-case run bit for bit, small cases must match the FP64 oracle, and the
whole ensemble must stay finite and conservative for its 2000 steps."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hip():
    import torch
    assert torch.cuda.is_available()
    import paper_1110_5004_amd as P
    return P


@pytest.fixture(scope="module")
def cases():
    return W.ensemble(seed=0)


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_ensemble_batched_equals_single(hip, cases, storage):
    batch = hip.Simulation(cases, storage=storage)
    batch.step(50)
    picks = [0, 1, 2, 3, 17, 40, 63]
    for k in picks:
        single = hip.Simulation([cases[k]], storage=storage)
        single.step(50)
        assert np.array_equal(batch.get_state(k), single.get_state(0)), (storage, k)
        single.close()


# max |d phi|, relL2(u), max |d p| / max |p| after 200 steps.  The 16-bit
# bounds follow the storage spacing (FP16 2^-11 relative, BF16 eight times
# that) above the FP32 arithmetic floor.
ENSEMBLE_TOL = {"fp32": (1e-5, 1e-4, 1e-4), "fp16": (3e-5, 3e-2, 3e-3),
                "bf16": (2.4e-4, 0.24, 2.4e-2)}


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_ensemble_small_cases_match_oracle(hip, cases, storage):
    small = [k for k, c in enumerate(cases) if c.params["nx"] <= 128][:6]
    sub = [cases[k] for k in small]
    sim = hip.Simulation(sub, storage=storage)
    sim.step(200)
    tphi, tu, tp = ENSEMBLE_TOL[storage]
    for j, c in enumerate(sub):
        got = sim.moments(j)
        ref = O.Sim(c.params, c.phi0, c.u0, c.p0)
        ref.step(200)
        want = ref.fields()
        dphi = np.abs(got["phi"] - want["phi"]).max()
        du = np.linalg.norm(got["u"] - want["u"]) / np.linalg.norm(want["u"])
        dp = np.abs(got["p"] - want["p"]).max() / np.abs(want["p"]).max()
        print(f"{storage} case {small[j]} n={c.params['nx']}: max|dphi|={dphi:.2e} "
              f"relL2(u)={du:.2e} rel|dp|={dp:.2e}")
        assert dphi <= tphi and du <= tu and dp <= tp


def test_ensemble_full_run(hip, cases):
    sim = hip.Simulation(cases)
    sim.step(2000)
    for k in range(len(cases)):
        d = sim.diagnostics(k)
        assert d["nonfinite"] == 0, k
        assert d["mass_drift_rel"] <= 1e-6, (k, d["mass_drift_rel"])
