"""Host logic of the learned warm start: parameter layout and count agree
between the library and the oracle reference, and weights survive a
save/load round trip (CPU tensors; no GPU call)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_param_layout_matches_reference(tmp_path):
    from oracle import unet as U
    from paper_2604_15434_amd import warmstart as W

    n_ref = sum(27 * ci * co + co for _, ci, co in U.LAYERS) + 17
    assert W.param_count() == n_ref
    assert [tuple(x) for x in W.CONV_SHAPES] == [(ci, co) for _, ci, co in U.LAYERS]
    flat = W.init_params(seed=4)
    assert flat.dtype == np.float32 and flat.size == n_ref
    # He scaling of the first layer's weights
    w1 = flat[:27 * 4 * 16]
    assert w1.std() == pytest.approx(np.sqrt(2.0 / (27 * 4)), rel=0.1)


def test_save_load_roundtrip(tmp_path):
    from paper_2604_15434_amd import warmstart as W

    ws = W.WarmStart(seed=7, device="cpu")
    ws.step = 12
    path = str(tmp_path / "w.f32")
    ws.save(path, meta={"note": "test"})
    back = W.WarmStart.load(path, device="cpu")
    assert back.step == 12
    assert torch.equal(back.params, ws.params)
