"""GPU parity of the batched factorization (one persistent launch over many
matrices of uneven order and rank) against the CPU oracle's canonical search:
the base-case elimination is the search's order, so P, L, D, e, r and R must
all match bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle.oracle as orc  # noqa: E402
from paper_1802_10453_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10453_amd import pldl
    c = pldl.Context(0)
    yield c
    c.close()


def make_batch(p, sizes, seed):
    mats = []
    for t, n in enumerate(sizes):
        if n <= 0:
            mats.append(np.zeros((0, 0), dtype=np.uint32))
            continue
        g = inputs.rng(seed + t)
        r = int(g.integers((n + 3) // 4, n + 1))
        c = r // 4
        A, _ = inputs.rank_profile_matrix_input(n, p, r - 2 * c, c, seed * 1000 + t, check=4)
        mats.append(A)
    return mats


def run_batch(ctx, p, mats, dtype=torch.int32):
    dev = [torch.from_numpy(np.ascontiguousarray(A).astype(np.int32 if dtype == torch.int32 else np.float64)).cuda()
           .reshape(A.shape) for A in mats]
    args = ctx.batched_args(dev)
    ctx.factor_batched(p, args)
    torch.cuda.synchronize()
    return args


def check_one(A, p, args, t):
    n = A.shape[0]
    assert int(args["status"][t]) == 0
    Ah = args["mats"][t].cpu().numpy()
    Ah = Ah.astype(np.int64).astype(np.uint32) if Ah.dtype == np.int32 else Ah.astype(np.uint32)
    ref = orc.search(A, p)
    assert int(args["rank"][t]) == ref["rank"]
    if n == 0:
        return
    perm = args["perm"][t].cpu().numpy()[:n]
    rpm = args["rpm"][t].cpu().numpy()[:n]
    e = args["e"][t].cpu().numpy()[:n]
    e = (e.astype(np.int64) if e.dtype == np.int32 else e).astype(np.uint32)
    assert (perm == ref["perm"]).all(), "canonical order differs"
    assert (rpm == ref["rpm"]).all(), "rank profile matrix differs"
    L = np.tril(Ah, -1)
    L[np.arange(n), np.arange(n)] = 1
    assert (L == ref["L"]).all(), f"L differs at {np.argwhere(L != ref['L'])[:5]}"
    assert (np.diag(Ah) == ref["dd"]).all()
    assert (e == ref["de"]).all()


@pytest.mark.parametrize("p", [2, 3, 32749, 65521, 8388593, 16777213])
def test_batched_parity(ctx, p):
    sizes = [1, 2, 3, 17, 64, 65, 100, 127, 128, 129, 200, 257, 383, 512, 31, 500]
    print(f"[batched] p={p} sizes={sizes}", flush=True)
    mats = make_batch(p, sizes, 500 + p % 1000)
    args = run_batch(ctx, p, mats)
    for t, A in enumerate(mats):
        check_one(A, p, args, t)


def test_batched_float64_and_uniform(ctx):
    p = 65521
    g = inputs.rng(4242)
    mats = [inputs.symmetric_uniform(n, p, 77 + n) for n in (5, 96, 300)]
    mats.append(np.zeros((40, 40), dtype=np.uint32))   # rank 0: every row set aside
    print("[batched] float64 storage, uniform and zero matrices", flush=True)
    args = run_batch(ctx, p, mats, dtype=torch.float64)
    for t, A in enumerate(mats):
        check_one(A, p, args, t)


def test_batched_char2_relaxed(ctx):
    mats = []
    for t, n in enumerate((64, 130, 256)):
        A, _, _ = inputs.char2_input(n, n // 4, n // 8, 900 + t, check=4)
        mats.append(A)
    print("[batched] characteristic 2", flush=True)
    args = run_batch(ctx, 2, mats)
    for t, A in enumerate(mats):
        check_one(A, 2, args, t)


def test_batched_status(ctx):
    """Out-of-range entries and orders are reported per matrix; the others still factor."""
    p = 32749
    good = make_batch(p, [50], 7)[0]
    bad = good.copy()
    bad[3, 2] = p + 5
    big = np.zeros((513, 513), dtype=np.uint32)
    print("[batched] status codes", flush=True)
    args = run_batch(ctx, p, [good, bad, big])
    st = args["status"].cpu().numpy()
    assert st[0] == 0 and st[1] == 1 and st[2] == -3
    check_one(good, p, args, 0)


def test_batched_graph_replay(ctx):
    """One captured launch replayed on new inputs: every replay equals the eager result."""
    p = 32749
    sizes = [40, 300, 7, 129, 512, 90]
    batches = [make_batch(p, sizes, 3000 + k) for k in range(3)]
    dev = [torch.zeros((n, n), dtype=torch.int32, device="cuda") for n in sizes]
    args = ctx.batched_args(dev)
    # first call outside the capture (allocates the workspace and the inverse table)
    for d, A in zip(dev, batches[0]):
        d.copy_(torch.from_numpy(A.astype(np.int32)))
    ctx.factor_batched(p, args)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            ctx.factor_batched(p, args)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for k in range(3):
        print(f"[batched] graph replay {k}", flush=True)
        for d, A in zip(dev, batches[k]):
            d.copy_(torch.from_numpy(A.astype(np.int32)))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for t, A in enumerate(batches[k]):
            check_one(A, p, args, t)
