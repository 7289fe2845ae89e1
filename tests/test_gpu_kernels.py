"""Kernel-level GPU tests through the C-ABI: the LDS-tiled permute is bit-exact
against numpy.transpose, the matrix-core complex GEMM is within FP32
accumulation bounds of a complex128 product."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2110_09894_amd import qxtn  # noqa: E402


def _c64(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.float32)).cuda()


def _host_c64(t):
    return t.cpu().numpy().view(np.complex64)


@pytest.mark.parametrize("rank,items,seed", [(1, 1, 0), (3, 2, 1), (5, 1, 2), (8, 3, 3), (10, 1, 4),
                                             (13, 2, 5), (18, 1, 6), (21, 1, 7)])
def test_permute_bit_exact(rank, items, seed):
    rng = np.random.default_rng(seed)
    in_pos = rng.permutation(rank).astype(np.int32)
    x = _c64(rng, items, 2 ** rank)
    out = torch.empty_like(_dev(x))
    qxtn.permute_c64(_dev(x), out, in_pos, items)
    torch.cuda.synchronize()
    got = _host_c64(out).reshape(items, 2 ** rank)
    # axis a of the (2,)*rank view is bit rank-1-a; output bit i comes from input bit in_pos[i]
    xt = x.reshape((items,) + (2,) * rank)
    axes = [0] + [1 + rank - 1 - int(in_pos[rank - 1 - a]) for a in range(rank)]
    want = np.transpose(xt, axes).reshape(items, 2 ** rank)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_permute_identity_and_reversal():
    rng = np.random.default_rng(9)
    x = _c64(rng, 1, 2 ** 12)
    for in_pos in (np.arange(12), np.arange(12)[::-1]):
        out = torch.empty_like(_dev(x))
        qxtn.permute_c64(_dev(x), out, in_pos.astype(np.int32), 1)
        torch.cuda.synchronize()
        want = np.transpose(x.reshape((1,) + (2,) * 12), [0] + [1 + 11 - int(in_pos[11 - a]) for a in range(12)])
        assert np.array_equal(_host_c64(out).reshape(-1), want.reshape(-1))


def _gemm_case(M, N, K, akc, bkc, batch, seed, precision="c64", tile=None):
    rng = np.random.default_rng(seed)
    A = _c64(rng, batch, M, K)
    Bm = _c64(rng, batch, K, N)
    a_store = A if akc else np.ascontiguousarray(np.swapaxes(A, 1, 2))
    b_store = np.ascontiguousarray(np.swapaxes(Bm, 1, 2)) if bkc else Bm
    a_ms, a_ks = (K, 1) if akc else (1, M)
    b_ks, b_ns = (1, K) if bkc else (N, 1)
    dc = torch.zeros(batch * M * N * 2, dtype=torch.float32, device="cuda")
    qxtn.cgemm(_dev(a_store), _dev(b_store), dc, M, N, K, a_ms, a_ks, b_ks, b_ns, M * K, K * N, M * N, batch,
               precision, tile=tile)
    torch.cuda.synchronize()
    got = _host_c64(dc).reshape(batch, M, N).astype(np.complex128)
    want = np.matmul(A.astype(np.complex128), Bm.astype(np.complex128))
    bound = np.matmul(np.abs(A).astype(np.float64), np.abs(Bm).astype(np.float64))
    return got, want, bound


@pytest.mark.parametrize("M,N,K", [(128, 128, 128), (256, 512, 64), (64, 64, 16), (37, 53, 19), (1, 1, 1),
                                   (300, 129, 257), (32, 2048, 32), (512, 512, 512), (64, 96, 24), (80, 48, 8)])
@pytest.mark.parametrize("akc,bkc", [(True, True), (True, False), (False, True), (False, False)])
def test_cgemm_c64(M, N, K, akc, bkc):
    got, want, bound = _gemm_case(M, N, K, akc, bkc, 2, M * 7 + N * 3 + K)
    # FP32 accumulation: |err| <= K * 2^-23 * (|A||B|) componentwise, with margin
    assert np.all(np.abs(got - want) <= 2 * K * 2.0 ** -23 * bound + 1e-30)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < 2e-6


# Split precision: A ~ Ah + Al with 8 (BF16) or 11 (FP16) significant bits per part; the product drops
# Al Bl, so the normwise error is a few units of 2^-16 (BF16) or 2^-22 (FP16), plus FP32 accumulation.
SPLIT_REL = {"split_bf16": 6e-5, "split_fp16": 4e-6}


@pytest.mark.parametrize("precision", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("M,N,K", [(128, 128, 128), (256, 512, 64), (64, 64, 16), (37, 53, 19), (300, 129, 257),
                                   (512, 512, 512), (64, 96, 24), (80, 48, 8)])
@pytest.mark.parametrize("akc,bkc", [(True, True), (False, False), (True, False)])
def test_cgemm_split(precision, M, N, K, akc, bkc):
    got, want, bound = _gemm_case(M, N, K, akc, bkc, 2, M * 5 + N * 11 + K, precision)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < SPLIT_REL[precision], rel
    assert np.all(np.abs(got - want) <= 64 * SPLIT_REL[precision] * bound + 1e-30)


@pytest.mark.parametrize("tile", qxtn.TILES)
@pytest.mark.parametrize("precision", ["c64", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("M,N,K,akc,bkc", [(300, 129, 257, True, True), (512, 384, 64, False, False),
                                           (37, 53, 19, True, False), (64, 96, 24, False, True),
                                           (256, 256, 128, True, True), (1, 1, 1, True, True)])
def test_cgemm_every_tile(tile, precision, M, N, K, akc, bkc):
    """Every work-group tile the autotuner may pick, forced, in every precision: shapes spanning several
    tiles, ragged edges in m, n and k, tiles larger than the matrix."""
    got, want, bound = _gemm_case(M, N, K, akc, bkc, 2, M * 13 + N * 7 + K, precision, tile)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    if precision == "c64":
        assert np.all(np.abs(got - want) <= 2 * K * 2.0 ** -23 * bound + 1e-30)
        assert rel < 2e-6
    else:
        assert rel < SPLIT_REL[precision], rel
        assert np.all(np.abs(got - want) <= 64 * SPLIT_REL[precision] * bound + 1e-30)


def test_cgemm_tile_argument_validated():
    a = torch.zeros(64, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        qxtn.cgemm(a, a, a, 4, 4, 4, 4, 1, 1, 4, tile="16x16")
    # the C-ABI itself rejects tiles outside 0..9 before launching anything
    st = qxtn.lib().qx_cgemm(a.data_ptr(), a.data_ptr(), a.data_ptr(), 4, 4, 4, 4, 1, 1, 4, 0, 0, 0, 1, 0, 10, None)
    assert st == qxtn.QX_ERR_INVALID_ARG


@pytest.mark.parametrize("precision", ["c64", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("M,N,K,akc,bkc", [(16, 1000, 16, True, True), (16, 1000, 16, False, False),
                                           (512, 8, 8, True, False), (32, 333, 32, False, True),
                                           (5, 7, 3, True, True), (257, 31, 17, False, False),
                                           (2085, 16, 16, True, True), (20, 549, 24, True, False),
                                           (1, 130, 1, True, True), (4096, 32, 32, True, True),
                                           (3000, 20, 5, False, True), (777, 4, 4, True, True),
                                           (24, 300, 2, False, False), (1000, 32, 8, False, False)])
def test_cgemm_thin_kernel(precision, M, N, K, akc, bkc):
    """The memory-bound thin kernel (a side of at most 32, K at most 32) on the 16x16 matrix-core shapes:
    ragged rows across blocks and waves, a short side of 1..32 (one or two 16-column blocks), K of 1..32
    (one or two 16-k chunks; complex64 loads 1 or 2 k per lane for K up to 4 or 8), either operand the
    short one, k-contiguous or not."""
    got, want, bound = _gemm_case(M, N, K, akc, bkc, 3, M * 3 + N * 5 + K, precision, "thin")
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    if precision == "c64":
        assert np.all(np.abs(got - want) <= 2 * K * 2.0 ** -23 * bound + 1e-30)
        assert rel < 2e-6
    else:
        assert rel < SPLIT_REL[precision], rel
        assert np.all(np.abs(got - want) <= 64 * SPLIT_REL[precision] * bound + 1e-30)
