"""GPU: mini-batch k-means quantisation (cmif_kmeans) against the FP64
oracle on the same draws.  Both sides round every product and sum on its
own in the same order, so the centres must be bitwise equal and the labels
identical."""

import numpy as np
import pytest

import synth
from gpu_common import say

pytestmark = pytest.mark.gpu


def _run(cm, torch, img, k, init, batches, mask=None):
    t = torch.from_numpy(np.ascontiguousarray(img, np.float32)).cuda()
    mt = None if mask is None else torch.from_numpy(mask).cuda()
    iters, batch = (0, 1) if batches is None else np.asarray(batches).shape
    return cm.kmeans_quantize(t, k, iters=iters, batch=batch, mask=mt,
                              init_idx=init, batches=batches)


def test_hand_worked_example(gpu, oracle):
    cm, torch = gpu
    img = np.array([[0, 2, 10, 12, 11]], np.float32)
    r = _run(cm, torch, img, 2, [0, 2], np.array([[1, 0, 3, 4]]))
    assert r["centers"].cpu().numpy().ravel().tolist() == [1.0, 11.5]
    assert r["labels"].cpu().numpy().ravel().tolist() == [0, 0, 1, 1, 1]
    r = _run(cm, torch, img, 2, [0, 2], np.array([[1, -1, 0, 3, 99, 4]]))
    assert r["centers"].cpu().numpy().ravel().tolist() == [1.0, 11.5]
    assert r["bad"] == 2


@pytest.mark.parametrize("shape,k,iters,batch,masked", [
    ((256, 256), 16, 25, 1000, False),
    ((256, 256, 3), 16, 25, 1000, True),
    ((300, 300), 64, 40, 500, True),
    ((97, 131, 2), 4, 10, 8192, False),
])
def test_matches_oracle(gpu, oracle, shape, k, iters, batch, masked):
    cm, torch = gpu
    rng = np.random.default_rng(77 + k)
    h, w = shape[:2]
    # smooth fields (what the paper quantises: image intensities)
    chans = [synth.field(rng, 3.0, (h, w)) * 40.0 + 120.0
             for _ in range(shape[2] if len(shape) == 3 else 1)]
    img = (np.stack(chans, axis=-1) if len(shape) == 3 else chans[0]).astype(np.float32)
    mask = (rng.random((h, w)) < 0.9).astype(np.uint8) if masked else None
    pool = np.arange(h * w) if mask is None else np.flatnonzero(mask)
    init = rng.choice(pool, size=k, replace=False)
    batches = pool[rng.integers(0, pool.size, size=(iters, batch))]
    say(f"[gpu] kmeans {shape} k={k} iters={iters} batch={batch} masked={masked}")
    r = _run(cm, torch, img, k, init, batches, mask)
    c_o = oracle.kmeans_minibatch(img, k, init_idx=init, batches=batches)
    l_o = oracle.kmeans_labels(img, c_o, mask)
    c_g = r["centers"].cpu().numpy()
    assert np.array_equal(c_g.view(np.uint64), c_o.view(np.uint64))
    assert np.array_equal(r["labels"].cpu().numpy(), l_o)
    assert r["bad"] == 0
    used = np.unique(l_o[mask == 1] if mask is not None else l_o)
    say(f"labels used {used.size} of {k}")


def test_quantised_images_align(gpu, oracle):
    """End to end as in Alg. 1: two intensity images quantised on the GPU,
    then aligned; the planted shift is found."""
    cm, torch = gpu
    rng = np.random.default_rng(21)
    n, m = 96, 12
    f = synth.field(rng, 3.0, (n + 2 * m, n + 2 * m))
    a = (f[m:m + n, m:m + n] * 50 + 100).astype(np.float32)
    s = (5, -7)
    b = (np.cos(2.5 * f[m - s[0]:m - s[0] + n, m - s[1]:m - s[1] + n]) * 30 + 60
         + rng.normal(scale=2.0, size=(n, n))).astype(np.float32)
    q = 8
    ra = cm.kmeans_quantize(torch.from_numpy(a).cuda(), q, rng=rng)
    rb = cm.kmeans_quantize(torch.from_numpy(b).cuda(), q, rng=rng)
    plan = cm.Plan([(n, n, n, n)], q, q)
    best = plan.align(ra["labels"], None, rb["labels"], None)["best"][0]
    assert (best["dy"], best["dx"]) == s, best
