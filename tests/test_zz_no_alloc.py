"""The allocation-free closure prediction (sph_closure_predict_static) through
the C ABI, against sph_closure_predict: bit-identical outputs on two calls in
a row, the second with fewer rows, and the size limit."""
import numpy as np
import pytest
import torch

import paper_2311_15088_amd as sph
from paper_2311_15088_amd import scenes

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _features(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 256)).astype(np.float32)
    bits = (x.view(np.uint32) >> 16).astype(np.uint16)  # bfloat16 by truncation: any bit pattern is valid input
    return torch.from_numpy(bits.view(np.int16)).to(DEV)


def test_static_predict_matches_predict_twice_then_smaller():
    rng = np.random.default_rng(3)
    p = scenes.mlp_init(21)
    for k in ("b1", "b2", "b3"):
        p[k] = (0.1 * rng.standard_normal(p[k].shape)).astype(np.float32)
    cl = sph.Closure(scenes.mlp_flat(p), force_scale=1.5)
    for n, seed in ((65536, 1), (1001, 2)):  # the maximum, then a smaller ragged call
        print(f"[no-alloc] rows {n}", flush=True)
        x = _features(n, seed)
        want = torch.zeros((n, 3), dtype=torch.float32, device=DEV)
        got = torch.full((n, 3), float("nan"), dtype=torch.float32, device=DEV)
        cl.predict(x, want)
        cl.predict_static(x, got)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy().view(np.uint32), want.cpu().numpy().view(np.uint32))
    # beyond the scratch: a clear error, nothing launched
    x = _features(65537, 4)
    out = torch.zeros((65537, 3), dtype=torch.float32, device=DEV)
    with pytest.raises(sph.SphError) as ei:
        cl.predict_static(x, out)
    assert ei.value.status == sph.ECAPACITY
    assert float(out.abs().max()) == 0.0
    cl.close()
