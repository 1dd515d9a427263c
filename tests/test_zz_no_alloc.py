"""rwgt_xsec_noalloc (the no-allocation variant of rwgt_xsec, partial sums in
a static device array) against rwgt_xsec through the C ABI: two calls in a
row, the second with fewer events and cards, each equal to rwgt_xsec's result
bit for bit (the same kernels in the same order); more cards than the static
array holds are refused."""
import numpy as np
import pytest

import synth

from gpu_util import dev, torch_cuda

pytestmark = pytest.mark.gpu


def test_xsec_noalloc_matches_xsec():
    print("[case] xsec no-alloc", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    rng = np.random.default_rng(14)
    with rw.Reweighter("g g > t t~ g g", synth.ORIG_QCD.slha()) as r:
        for nevt, nsets in ((300_000, 64), (70_001, 5)):
            w = rng.uniform(0.2, 2.0, nevt)
            wp = rng.uniform(0.1, 3.0, (nsets, nevt))
            wp[0, :10] = 0.0
            wd, wpd = dev(w), dev(wp)
            a = rw.rwgt_xsec(r.ctx, wd, wpd, 12.5, 0.3, 12.5 / nevt)
            b = rw.rwgt_xsec(r.ctx, wd, wpd, 12.5, 0.3, 12.5 / nevt, entry="rwgt_xsec_noalloc")
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)
            print(f"nevt {nevt}, nsets {nsets}: identical", flush=True)
        too_many = dev(np.ones((65, 10)))
        with pytest.raises(rw.RwgtError, match="64 cards"):
            rw.rwgt_xsec(r.ctx, dev(np.ones(10)), too_many, 1.0, 0.1, 0.1, entry="rwgt_xsec_noalloc")
