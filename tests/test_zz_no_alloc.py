"""The allocation-free proxy inference (kvop_proxy_infer_noalloc) against kvop_proxy_infer at
the proxy's full shape (2048 -> 256): two calls in a row on the same scratch, the second with
fewer rows and other features, must equal the allocating call exactly (same kernels); a row
count beyond the scratch's limit is refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth

pytestmark = pytest.mark.gpu

D_IN, H = 2048, 256
SCRATCH_BYTES = 32 << 20
MAX_ROWS = (SCRATCH_BYTES - 256) // (2 * D_IN + 4 * H)      # 6553


def test_noalloc_proxy_inference_matches_allocating_call(device):
    rng = np.random.default_rng(5)
    p0 = synth.proxy_init(D_IN, H, 2, 5)
    p0["b1"] = (rng.standard_normal(H) * 0.05).astype(np.float32)
    p0["w2"] = (rng.standard_normal((2, H)) * 0.5).astype(np.float32)
    params = np.concatenate([p0["w1"].ravel(), p0["b1"], p0["w2"].ravel(), p0["b2"]]).astype(np.float32)
    px = K.kvop_proxy_create(D_IN, H, torch.from_numpy(params).to(device))
    feats = torch.from_numpy((rng.standard_normal((MAX_ROWS + 1, D_IN)) * 0.6 +
                              rng.standard_normal(D_IN) * 0.2).astype(np.float32)).to(device)
    K.kvop_proxy_fit_standardizer(px, feats[:4096])
    tau = 0.6
    for n, first in ((MAX_ROWS, 0), (777, 1234)):
        f = feats[first:first + n]
        outs = []
        for fn in (K.kvop_proxy_infer, K.kvop_proxy_infer_noalloc):
            cls = torch.full((n,), 7, dtype=torch.int8, device=device)
            conf = torch.full((n,), np.nan, dtype=torch.float32, device=device)
            ans = torch.full((n,), 7, dtype=torch.int8, device=device)
            print("proxy inference", fn.__name__, "rows", n, flush=True)
            fn(px, f, tau, cls, conf, ans)
            torch.cuda.synchronize()
            outs.append([x.cpu().numpy() for x in (cls, conf, ans)])
        ref, got = outs
        assert np.all(np.isfinite(ref[1])) and set(np.unique(ref[0])) <= {0, 1}
        assert 0 < ref[2].sum() < n, ref[2].sum()                 # some rows answered, some passed on
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
    cls = torch.zeros(MAX_ROWS + 1, dtype=torch.int8, device=device)
    conf = torch.zeros(MAX_ROWS + 1, dtype=torch.float32, device=device)
    ans = torch.zeros(MAX_ROWS + 1, dtype=torch.int8, device=device)
    with pytest.raises(K.KvopError) as e:
        K.kvop_proxy_infer_noalloc(px, feats, tau, cls, conf, ans)
    assert e.value.status == K.KVOP_EINVAL and str(MAX_ROWS) in str(e.value)
    torch.cuda.synchronize()
    K.kvop_proxy_destroy(px)
