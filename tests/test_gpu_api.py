"""GPU tests of the remaining entry points: the characteristic-2 standard-form
transform as its own call, and the threshold autotuner (its table, and that
factorizations with the tuned threshold still match the oracle)."""
import os
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle.oracle as orc  # noqa: E402
from paper_1802_10453_amd import inputs  # noqa: E402

from gpu_helpers import check_against_oracle, gpu_factor, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10453_amd import pldl
    c = pldl.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("dtype", [torch.int32, torch.float64])
def test_char2_to_standard_matches_factor_option(ctx, dtype):
    A, rpm, _ = inputs.char2_input(300, 90, 45, 515, check=0)
    print(f"[api] char2 standard form, dtype {dtype}", flush=True)
    ref = gpu_factor(ctx, A, 2, threshold=32, dtype=dtype, standard_form=True)
    Ad = to_dev(A, dtype)
    out = ctx.factor(Ad, 2, threshold=32)
    ctx.char2_to_standard(Ad, out["e"], out["perm"])
    torch.cuda.synchronize()
    Ah = Ad.cpu().numpy()
    Ah = Ah.astype(np.int64).astype(np.uint32) if dtype == torch.int32 else Ah.astype(np.uint32)
    L = np.tril(Ah, -1)
    L[np.arange(300), np.arange(300)] = 1
    assert (out["perm"].cpu().numpy() == ref["perm"]).all()
    assert (L == ref["L"]).all() and (np.diag(Ah) == ref["dd"]).all()
    e = out["e"].cpu().numpy()
    assert ((e.astype(np.int64) if dtype == torch.int32 else e).astype(np.uint32) == ref["de"]).all()
    # the standard form still reconstructs A
    rec = orc.reconstruct(2, ref["perm"], ref["L"], ref["dd"], ref["de"])
    assert (rec == A).all()


def test_autotune_table_and_use(ctx):
    p = 65521
    path = os.path.join(tempfile.mkdtemp(), "tune.txt")
    print("[api] autotune n = 256, 600", flush=True)
    ctx.autotune(p, [256, 600], table_path=path)
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    assert [int(r[1]) for r in rows] == [256, 600]
    assert all(int(r[0]) == p and int(r[2]) in (32, 48, 64, 96, 128) for r in rows)
    # a fresh context reads the table; threshold 0 then takes the tuned value
    from paper_1802_10453_amd import pldl
    c2 = pldl.Context(0)
    try:
        c2.autotune(p, [], table_path=path)
        A, _ = inputs.rank_profile_matrix_input(600, p, 200, 100, 6060, check=0)
        res = gpu_factor(c2, A, p, threshold=0)
        check_against_oracle(A, p, res)
    finally:
        c2.close()
