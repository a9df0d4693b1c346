"""The no-allocation entry point mlb_dilate_noalloc_dev against the entry
point it mirrors, mlb_dilate_dev (eq. postProcessingDilation): both run the
same kernels, so the dilated densities must agree bit for bit.  Two calls in
a row share the GPU's fixed scratch array, the second on a smaller grid with
fewer selected rows (the scratch keeps the first call's partial maxima, which
the second must overwrite rather than read)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call(nel, nsel, seed, rel_thr=0.5, r_th=2.0):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1909_13585_amd as mlb
    print(f"case noalloc dilation nel={nel} nsel={nsel} seed={seed}", flush=True)
    c = mlb.Context(nel, mg_levels=1, eig_level=1)
    m = c.m
    rng = np.random.default_rng(seed)
    # non-negative rows with a few large entries, so that thresholds select
    # scattered elements
    gradn = torch.from_numpy(np.ascontiguousarray(rng.random((nsel, m)) ** 8)).cuda()
    x = torch.from_numpy(rng.random(m)).cuda()
    ref = torch.empty_like(x)
    out = torch.full_like(x, float("nan"))
    c.dilate_dev(gradn, rel_thr, r_th, x, ref)
    c.dilate_noalloc_dev(gradn, rel_thr, r_th, x, out)
    torch.cuda.synchronize()
    assert torch.equal(ref, out)
    assert bool((out >= x).all())
    assert bool((out > x).any())
    c.close()


def test_noalloc_dilation_matches_dilate_dev_on_two_calls():
    _call((40, 16, 16), 3, 11)   # 10,240 elements, 3 rows
    _call((64, 32), 1, 12)       # 2,048 elements, 1 row: smaller input second
