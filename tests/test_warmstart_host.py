"""Host-side bookkeeping of the learned warm start (no GPU needed)."""
import os

import numpy as np
import pytest

from oracle import unet_ref as U

torch = pytest.importorskip("torch")


def test_layer_shapes_match_reference_layout():
    from paper_2204_10822_amd import warmstart as W
    shapes = W.layer_shapes()
    ref = U.param_shapes()
    assert len(shapes) == len(ref)
    for (kin, kout, nb), (ws, bs) in zip(shapes, ref):
        assert (kin, kout) == tuple(ws) and nb == bs[0]
    theta = W.init_params(0, U.param_count())
    assert theta.dtype == np.float32 and theta.size == U.param_count()


def test_committed_weights_load_without_pickle():
    from paper_2204_10822_amd import warmstart as W
    if not os.path.exists(W.WEIGHTS):
        pytest.skip("no trained weights committed")
    th = np.load(W.WEIGHTS, allow_pickle=False)
    assert th.dtype == np.float32 and th.size == U.param_count() and np.isfinite(th).all()
