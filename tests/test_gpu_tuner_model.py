"""GPU: the model-guided tuner (sampled timings, neural time model, top-k confirmation)."""
import numpy as np
import pytest

from conftest import gpu_available
from helpers import assert_close, storage

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

from oracle import oracle  # noqa: E402
from paper_1605_06399_amd import binding as B, synth  # noqa: E402

if gpu_available():
    import torch
    from paper_1605_06399_amd import torch_api as T


@pytest.mark.parametrize("op,r", [(B.ICL_OP_CONV_SEP, 3), (B.ICL_OP_CONV2D, 3)])
def test_model_guided_search_times_fewer_and_picks_a_valid_variant(op, r):
    H, W = 768, 1024
    n_cand = B.icl_variant_count(op) - 1
    try:
        st, timed = B.icl_tune_model(op, B.ICL_F32, r, W, H, 4, 2, seed=3)
        assert st == B.ICL_OK
        assert 4 <= timed <= 6 < n_cand, (timed, n_cand)
        st, idx = B.icl_selected_variant(op, B.ICL_F32, r, W, H)
        assert st == B.ICL_OK and 1 <= idx <= n_cand
        xd, x64 = storage(synth.image_uniform(60, H, W), "f32")
        n = 2 * r + 1
        if op == B.ICL_OP_CONV_SEP:
            h = synth.normal_taps_normalised(60, n, stream=1)
            v = synth.normal_taps_normalised(60, n, stream=2)
            out = T.conv_sep(xd, torch.from_numpy(h).cuda(), torch.from_numpy(v).cuda())
            ref, sc = oracle.conv_sep(x64, h, v), oracle.normwise_scale_sep(x64, h, v)
        else:
            w = synth.normal_taps_normalised(60, n * n, stream=3).reshape(n, n)
            out = T.conv2d(xd, torch.from_numpy(w).cuda())
            ref, sc = oracle.conv2d(x64, w), oracle.normwise_scale_conv2d(x64, w)
        torch.cuda.synchronize()
        assert_close(out, ref, sc, "f32", f"model-tuned op {op}")
        # the same seed samples the same candidates
        st2, timed2 = B.icl_tune_model(op, B.ICL_F32, r, W, H, 4, 2, seed=3)
        assert st2 == B.ICL_OK and timed2 == timed
    finally:
        B.icl_tune_clear()


def test_model_guided_search_small_space_times_everything():
    H, W = 256, 256
    try:
        n_cand = B.icl_variant_count(B.ICL_OP_NMS) - 1
        st, timed = B.icl_tune_model(B.ICL_OP_NMS, B.ICL_F32, 1, W, H, 4, 2, seed=1)
        assert st == B.ICL_OK and timed <= n_cand
    finally:
        B.icl_tune_clear()
