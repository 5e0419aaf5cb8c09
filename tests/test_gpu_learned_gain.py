"""The learned filter trained on the GPU by this library's kernels, on (mix, blood-only)
pairs that its own RF synthesis and beamforming generate, against the method without
it: no clutter filter, the untrained network, and the SVD filter (reported)."""
import numpy as np
import pytest

from fqscene import get_config, lcf_init_weights

pytestmark = pytest.mark.gpu


def test_training_gain():
    import torch
    from paper_2509_05464_amd.learned import LearnedFilter
    from paper_2509_05464_amd.train_lcf import evaluate, make_pairs, train
    cfg = get_config('c4_small')
    print('make pairs', flush=True)
    mix, blood = make_pairs(cfg, [2000, 2001, 2002, 2003])
    mt, bt = make_pairs(cfg, [2100])
    filt = LearnedFilter(lcf_init_weights(0), lr=2e-3)
    before = evaluate(filt, mt[0], bt[0])
    print('untrained', before, flush=True)
    hist = train(filt, mix, blood, steps=600, batch=2048, log_every=100)
    after = evaluate(filt, mt[0], bt[0])
    print('trained', after, 'loss', hist[0][1], '->', hist[-1][1], flush=True)
    assert hist[-1][1] < 0.5 * hist[0][1]
    assert after['learned_db'] < before['learned_db'] - 3.0
    assert after['learned_db'] < after['raw_db'] - 10.0
