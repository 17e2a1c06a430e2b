"""Full-size workloads on the GPU, in the configuration bench.py times, checked
by properties that hold at any size: rank and rank profile matrix against the
generator's closed form (RPM(L R L^T) = supp(R), Theorem 1), the block
structure of D, and A = P L D L^T P^T by Freivalds' test; sampled batch members
against the oracle's canonical search, exactly."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

import oracle.oracle as orc  # noqa: E402
from paper_1802_10453_amd import inputs  # noqa: E402

from gpu_helpers import freivalds, freivalds_f2, gpu_factor, structure  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10453_amd import pldl
    c = pldl.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c2_input():
    print("[fullsize] generating the n=16384 random-RPM input", flush=True)
    return inputs.config_input(inputs.C2, device="cuda", check=8)


@pytest.mark.parametrize("path", ["f64", "i8"])
def test_c2_full_size(ctx, c2_input, path):
    from paper_1802_10453_amd import pldl
    A, rpm = c2_input
    cfg = inputs.C2
    ctx.set_path(pldl.PLDL_PATH_I8 if path == "i8" else pldl.PLDL_PATH_F64)
    try:
        res = gpu_factor(ctx, A, cfg["p"])
    finally:
        ctx.set_path(pldl.PLDL_PATH_AUTO)
    assert res["rank"] == cfg["f"] + 2 * cfg["c"]
    assert (res["rpm"] == rpm).all()
    structure(res, cfg["p"])
    freivalds(A, cfg["p"], res, trials=3)


def test_c4_full_size(ctx):
    """The n = 8192 characteristic-2 workload: R against the closed form, (L, D, e)
    against the oracle's replay of the GPU's P (bit-exact), A = P L D L^T P^T by 64
    random vectors over F_2, and the Section 2.3 standard form against the
    oracle's transform of that replay, element by element."""
    cfg = inputs.C4
    print("[fullsize] generating the n=8192 characteristic-2 input", flush=True)
    A, rpm = inputs.config_input(cfg, device="cuda", check=8)
    res = gpu_factor(ctx, A, 2)
    r = cfg["f"] + 2 * cfg["c"]
    assert res["rank"] == r
    assert (res["rpm"] == rpm).all()
    structure(res, 2)
    freivalds_f2(A, res, nvec=64)
    print("[fullsize] oracle replay of the GPU pivot order (n=8192)", flush=True)
    rc, rp = orc.replay(A, 2, res["perm"], res["rpm"], r)
    assert rc == 0
    for key in ("L", "dd", "de"):
        assert (rp[key] == res[key]).all(), key
    std = gpu_factor(ctx, A, 2, standard_form=True)
    assert (std["perm"][:r] != res["perm"][:r]).any(), "the workload has relaxed blocks to transform"
    perm_s, L_s, dd_s, de_s = orc.char2_standard(rp["perm"], rp["L"], rp["dd"], rp["de"])
    assert (std["perm"] == perm_s).all() and (std["rpm"] == rpm).all()
    assert (std["L"] == L_s).all() and (std["dd"] == dd_s).all() and (std["de"] == de_s).all()
    freivalds_f2(A, std, nvec=64, seed=1)


def test_c3_full_batch(ctx):
    cfg = inputs.C3
    print("[fullsize] generating the 4096-matrix batch", flush=True)
    mats, params, rpms = inputs.batch_input(cfg, workers=min(16, os.cpu_count() or 1), with_rpm=True)
    dev = [torch.from_numpy(A.astype(np.int32)).cuda() for A in mats]
    args = ctx.batched_args(dev)
    ctx.factor_batched(cfg["p"], args)
    torch.cuda.synchronize()
    st = args["status"].cpu().numpy()
    rk = args["rank"].cpu().numpy()
    assert (st == 0).all()
    assert all(int(rk[t]) == params[t][1] for t in range(len(mats)))
    for t in range(len(mats)):
        assert (args["rpm"][t].cpu().numpy()[:params[t][0]] == rpms[t]).all(), t
    g = inputs.rng(31337)
    for t in sorted(set(int(x) for x in g.integers(0, len(mats), size=12))):
        A, n = mats[t], params[t][0]
        ref = orc.search(A, cfg["p"])
        Ah = args["mats"][t].cpu().numpy().astype(np.int64).astype(np.uint32)
        L = np.tril(Ah, -1)
        L[np.arange(n), np.arange(n)] = 1
        e = args["e"][t].cpu().numpy()[:n].astype(np.int64).astype(np.uint32)
        assert (args["perm"][t].cpu().numpy()[:n] == ref["perm"]).all()
        assert (L == ref["L"]).all() and (np.diag(Ah) == ref["dd"]).all() and (e == ref["de"]).all()
