"""The compress entry point that allocates nothing (hcz_compress_static, its workspace a
static device array) against hcz_compress with a caller workspace (GPU): two calls in a
row, the second smaller, each compared byte for byte; a batch beyond the array's capacity
is refused before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_2212_10733_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2212_10733_amd import hcz
    return hcz


def say(*a):
    print("[case]", *a, flush=True)


def static_compress(hcz, plan, model, p, x, centroids, out):
    """hcz_compress_static through the C ABI; returns the status."""
    Hn, hs, rs = hcz._strides(x)
    cb = hcz.Codebook(8, centroids.data_ptr())
    cs = out.cstruct()
    st = hcz.LIB.hcz_compress_static(plan.h, None if model is None else model.h, C.byref(cb), C.byref(p),
                                     C.c_void_p(x.data_ptr()), hcz._dtype_code(x), Hn, hs, rs, C.byref(cs),
                                     hcz._stream())
    return st


def same(a, b):
    torch.cuda.synchronize()
    n = int(a.offsets[-1].item())
    assert torch.equal(a.flags, b.flags)
    assert torch.equal(a.offsets, b.offsets)
    assert torch.equal(a.stream[:n], b.stream[:n])
    assert torch.equal(a.codes, b.codes)
    assert torch.equal(a.lam.view(torch.int64), b.lam.view(torch.int64))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_static_scratch_compress_matches_workspace_compress(H, dtype):
    ctx = H.Context(0)
    plan = H.Plan(ctx)
    F = synth.histograms(3000, seed=90, dtype=dtype)
    F[11, 3, 3] = np.nan                                  # one verbatim record
    W = synth.dense_ae_weights()
    mu, sd = oracle.ae.norm_stats(F[12:])
    model = H.Model(plan, W, mu, sd)
    p = H.params(tau=1e-3, fit_codebook=True, sample_every=4)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    x = torch.from_numpy(F).cuda()
    for n in (3000, 777):                                 # two calls in a row, the second smaller
        say("static compress", dtype.__name__, n)
        ref_cz = H.Compressor(plan, model, n, p, in_dtype=tdt)
        ref = ref_cz.compress(x[:n])
        out = H.alloc_compressed(n, plan.N, "cuda", in_bytes=F.itemsize)
        cent = torch.zeros((16, 256), dtype=torch.float32, device="cuda")
        assert static_compress(H, plan, model, p, x[:n], cent, out) == 0, H.LIB.hcz_last_error()
        same(out, ref)
        assert torch.equal(cent, ref_cz.centroids)
        s_ref, s = ref.stats(), out.stats()
        assert s == s_ref and s["n_raw"] == (1 if n > 11 else 0)
    # coder only, then a batch too large for the static array
    say("static compress, coder only")
    out = H.alloc_compressed(500, plan.N, "cuda", in_bytes=F.itemsize)
    cent = torch.zeros((16, 256), dtype=torch.float32, device="cuda")
    p0 = H.params(tau=1e-3)
    assert static_compress(H, plan, None, p0, x[:500], cent, out) == 0
    same(out, H.Compressor(plan, None, 500, p0, in_dtype=tdt).compress(x[:500]))
    big = torch.zeros((12000, 39, 39), dtype=tdt, device="cuda")
    outb = H.alloc_compressed(1, plan.N, "cuda")
    assert static_compress(H, plan, model, p, big, cent, outb) == -6          # HCZ_EWORKSPACE
    assert b"at most" in H.LIB.hcz_last_error()
