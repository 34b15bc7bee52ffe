"""A sequence of implicit steps against the oracle: ten half-hour steps of the
512^2 multi-step workload (vortices drifting, each step's previous velocity the
step before's solution) on the GPU, plain FP64 from the previous step and the
FP32 + BF16-coarse mode with the learned start, against the oracle's own ten-step
sequence (tests/golden/medium_512_steps10.npz, written by the oracle alone)."""
import importlib.util
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "medium_512_steps10.npz")


@pytest.fixture(scope="module")
def seq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_10822_amd import sequences
    return sequences


@pytest.mark.parametrize("path", ["fp64", "bf16+learned"])
def test_ten_steps_match_oracle_sequence(seq, path):
    from paper_2204_10822_amd import inputs, warmstart
    learned = path.endswith("learned")
    if learned and not os.path.exists(warmstart.WEIGHTS):
        pytest.skip("no trained weights committed")
    if not os.path.exists(GOLD):
        pytest.skip("oracle sequence golden not written yet (tests/golden/make_goldens.py)")
    g = np.load(GOLD, allow_pickle=False)
    steps = int(g["steps"])
    print(f"[sequence] medium_512 x {steps} steps, {path}", flush=True)
    r = seq.run(inputs.medium_steps(512), steps, path.split("+")[0], learned=learned)
    err = np.linalg.norm(r["v"] - g["v"]) / np.linalg.norm(g["v"])
    s = seq.summary(r["rows"])
    print(f"[sequence] {path}: newton per step {s['newton_per_step']} (oracle {list(g['iterations'])}), "
          f"krylov/newton {s['krylov_per_newton']:.1f}, starts {s['starts']}, err vs oracle {err:.2e}", flush=True)
    assert all(row["rel_resid"] <= 1e-8 for row in r["rows"])
    assert err < 1e-6
