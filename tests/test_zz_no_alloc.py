"""GPU test of pldl_syrdk_noalloc (the allocation-free SYRDK / SYRD2K): its
output equals pldl_syrdk's, bit for bit, on two calls in a row (the second with
a smaller input, so stale scratch contents from the first would show), it
allocates no device memory, and it rejects sizes beyond its fixed scratch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1802_10453_amd import inputs  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).astype(np.float64)).cuda()


def host(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32)


def _case(g, p, n, k):
    A = g.integers(0, p, size=(n, k)).astype(np.uint32)
    B = g.integers(0, p, size=(n, k)).astype(np.uint32)
    C = np.tril(g.integers(0, p, size=(n, n)).astype(np.uint32))
    dd = g.integers(0, p, size=k).astype(np.uint32)
    de = np.zeros(k, dtype=np.uint32)
    for q in range(0, k - 1, 3):    # some 2x2 blocks
        de[q] = 1 + q % (p - 1)
        dd[q] = 0
        if p != 2:
            dd[q + 1] = 0
    return A, B, C, dd, de


@pytest.mark.parametrize("p", [2, 65521, 8388593])
def test_syrdk_noalloc_matches_syrdk(p):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10453_amd import pldl
    g = inputs.rng(7000 + p)
    ref_ctx = pldl.Context(0)
    cases = [_case(g, p, 700, 650), _case(g, p, 130, 77)]   # second call smaller
    refs = []
    for (A, B, C, dd, de) in cases:
        for withB in (False, True):
            Cd = dev(C)
            ref_ctx.syrdk(p, Cd, dev(A), dev(dd), dev(de), B=dev(B) if withB else None)
            refs.append(host(Cd))
    torch.cuda.synchronize()
    ctx = pldl.Context(0)          # a fresh context: no workspace exists on it
    try:
        ins = []
        for (A, B, C, dd, de) in cases:
            for withB in (False, True):
                ins.append((dev(C), dev(A), dev(dd), dev(de), dev(B) if withB else None))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        outs = []
        for (Cd, Ad, ddd, ded, Bd) in ins:
            print(f"[noalloc] p={p} n={Ad.shape[0]} k={Ad.shape[1]} B={Bd is not None}", flush=True)
            outs.append(ctx.syrdk_noalloc(p, Cd, Ad, ddd, ded, B=Bd))
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free0 - free1 < (1 << 20), f"device memory dropped by {free0 - free1} bytes"
        for got, ref in zip(outs, refs):
            assert (np.tril(host(got)) == np.tril(ref)).all()
        # beyond the scratch: a clear error, nothing queued
        n = 2048
        k = pldl.NOALLOC_SCRATCH_DOUBLES // n + 1
        Ad = torch.zeros((n, k), dtype=torch.float64, device="cuda")
        dd = torch.ones(k, dtype=torch.float64, device="cuda")
        de = torch.zeros(k, dtype=torch.float64, device="cuda")
        Cd = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        with pytest.raises(pldl.PldlError) as ei:
            ctx.syrdk_noalloc(p, Cd, Ad, dd, de)
        assert ei.value.code == pldl.ERRORS_BY_NAME["PLDL_ETOOBIG"]
    finally:
        ctx.close()
        ref_ctx.close()
