"""The paper's qualitative claims about the annealing, run through the C ABI
on a synthetic max-cut instance (G(200, 0.05), +-1 weights, 512 replicas,
3000 steps, fixed seeds, so each number below is deterministic):
  * a triangular Ks waveform (Sec. III-D) beats a constant or a ramped Ks;
  * moderate noise helps escape local minima, extreme noise degrades the
    solutions (Sec. IV's parameter discussion)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
DT = float(np.float32(0.01))


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22631_amd as oim
    g = synth.erdos_renyi(200, 0.05, seed=4, signed=True)
    prob = oim.Problem.from_csr(g.n, g.row_ptr, g.col, (-g.w).astype(np.float32))
    yield oim, g, prob
    prob.close()


def _mean_cut(setup, shape, sigma, R=512, steps=3000):
    import torch
    oim, g, prob = setup
    dev = torch.device("cuda:0")
    kmax = 2.0 * 0.5 / (DT * prob.info["max_abs_row_sum"])
    ksmax = 0.5 / (DT * 2)
    Ks = {"ramp": synth.ramp(0, ksmax, steps), "const": synth.const(ksmax, steps),
          "triangle": synth.triangle(ksmax, 5, steps)}[shape]
    th = torch.from_numpy(synth.theta0(R, g.n, seed=1)).to(dev)
    oim.oim_run(prob.handle, g.n, th, torch.from_numpy(synth.ramp(0, kmax, steps)).to(dev),
                torch.from_numpy(Ks).to(dev), torch.from_numpy(synth.const(sigma, steps)).to(dev),
                torch.from_numpy(synth.seeds(R, 0)).to(dev), q=2, dt=DT)
    col = oim.oim_round(2, th)
    cut = oim.oim_cut(prob.handle, col).cpu().numpy().astype(np.float64)
    print(f"G(200,0.05) Ks {shape:8s} sigma {sigma:4.2f}: mean cut {cut.mean():7.2f}, "
          f"best {cut.max():4.0f}", flush=True)
    return cut.mean()


def test_triangular_ks_beats_constant_and_ramp(setup):
    tri = _mean_cut(setup, "triangle", 0.2)
    assert tri > _mean_cut(setup, "const", 0.2) + 20
    assert tri > _mean_cut(setup, "ramp", 0.2) + 20


def test_moderate_noise_helps_and_extreme_noise_hurts(setup):
    none = _mean_cut(setup, "triangle", 0.0)
    moderate = _mean_cut(setup, "triangle", 0.2)
    extreme = _mean_cut(setup, "triangle", 3.2)
    assert moderate > none + 20
    assert moderate > extreme
