"""qx_cgemm_noalloc (no device allocation; split-BF16 operand copies in the library's
static per-device scratch) against qx_cgemm through the C-ABI: the same kernels on the
same inputs give bitwise the same products, on consecutive calls whose second input is
smaller than the first, and both are within the split / FP32 bounds of a complex128
product.  Sizes beyond the scratch are refused before anything runs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2110_09894_amd import qxtn  # noqa: E402

REL = {"c64": 2e-6, "split_bf16": 6e-5, "split_fp16": 4e-6}


def _case(M, N, K, batch, seed, akc, bkc):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((batch, M, K)) + 1j * rng.standard_normal((batch, M, K))).astype(np.complex64)
    Bm = (rng.standard_normal((batch, K, N)) + 1j * rng.standard_normal((batch, K, N))).astype(np.complex64)
    a_store = A if akc else np.ascontiguousarray(np.swapaxes(A, 1, 2))
    b_store = np.ascontiguousarray(np.swapaxes(Bm, 1, 2)) if bkc else Bm
    strides = ((K, 1) if akc else (1, M)) + ((1, K) if bkc else (N, 1))
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x).view(np.float32)).cuda()  # noqa: E731
    want = np.matmul(A.astype(np.complex128), Bm.astype(np.complex128))
    return dev(a_store), dev(b_store), strides, want


def _run(fn, a, b, strides, M, N, K, batch, precision, tile=None):
    c = torch.full((batch * M * N * 2,), float("nan"), dtype=torch.float32, device="cuda")
    fn(a, b, c, M, N, K, *strides, M * K, K * N, M * N, batch, precision, tile=tile)
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("precision", ["split_bf16", "c64", "split_fp16"])
def test_noalloc_matches_cgemm_on_consecutive_calls(precision):
    # first call larger than the second: the second reuses scratch the first filled
    for (M, N, K, batch, akc, bkc, tile) in [(384, 256, 200, 3, True, False, None), (37, 53, 19, 2, False, True, "64x64"),
                                             (512, 512, 512, 1, True, True, "256x128"), (64, 96, 24, 1, False, False, None)]:
        a, b, strides, want = _case(M, N, K, batch, M + 3 * N + 7 * K, akc, bkc)
        ref = _run(qxtn.cgemm, a, b, strides, M, N, K, batch, precision, tile)
        got = _run(qxtn.cgemm_noalloc, a, b, strides, M, N, K, batch, precision, tile)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (M, N, K)
        g = got.view(np.complex64).reshape(batch, M, N).astype(np.complex128)
        assert np.linalg.norm(g - want) / np.linalg.norm(want) < REL[precision], (M, N, K)


def test_noalloc_refuses_products_beyond_its_scratch():
    a = torch.zeros(16, dtype=torch.float32, device="cuda")
    # 8 * batch * (M + N) * roundup(K, 16) bytes just above the scratch size: refused on the host
    M = N = 1024
    K = qxtn.CGEMM_NOALLOC_SCRATCH_BYTES // (8 * (M + N)) + 16
    with pytest.raises(qxtn.QxError) as e:
        qxtn.cgemm_noalloc(a, a, a, M, N, K, K, 1, 1, K, batch=1, precision="split_bf16")
    assert e.value.status == qxtn.QX_ERR_INVALID_ARG
    assert "scratch" in str(e.value)
    # the largest split product that fits still runs
    K = qxtn.CGEMM_NOALLOC_SCRATCH_BYTES // (8 * (M + N))
    a, b, strides, want = _case(M, N, K, 1, 5, True, True)
    got = _run(qxtn.cgemm_noalloc, a, b, strides, M, N, K, 1, "split_bf16")
    g = got.view(np.complex64).reshape(1, M, N).astype(np.complex128)
    assert np.linalg.norm(g - want) / np.linalg.norm(want) < REL["split_bf16"]
