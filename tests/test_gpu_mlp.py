"""Warm-start network kernels (BF16 matrix-core GEMM, GELU, MSE, Adam)
against the FP64 oracle, through the C ABI.

Bars (derived from the arithmetic):
  - GEMM: products of BF16 values are exact in FP32, so the only error is
    FP32 accumulation: |C - C_ref| <= K 2^-23 (|A| |B|)_ij elementwise.
  - forward: both sides round X, W and hidden activations to BF16 at the
    same points; they differ by FP32 vs FP64 sums and the rare BF16
    rounding flip those cause (one flip moves one activation by 2^-8
    relative): max error <= 2e-3 max(1, max |Y|).
  - gradients: same, per parameter block, <= 1e-2 of the block's largest
    entry.
  - Adam: FP32 update vs FP64 update from the same gradient.
"""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2506_13624_amd import _lib as L  # noqa: E402

WIDTHS = [44, 256, 256, 256, 734]


def _params(widths, rng):
    parts = [rng.normal(0, math.sqrt(2.0 / widths[l]), widths[l] * widths[l + 1]) for l in range(len(widths) - 1)]
    parts += [rng.normal(0, 0.1, widths[l + 1]) for l in range(len(widths) - 1)]
    return np.concatenate(parts).astype(np.float32)


def _bf16_dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).cuda().contiguous()


def _bf16_host(a):
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).double().numpy()


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (64, 64, 16), (130, 70, 300), (512, 734, 256),
                                   (256, 256, 1024)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1)])
def test_gemm_bf16_matches_fp64(M, N, K, ta, tb):
    print(f"gemm M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(M * 7 + N * 3 + K + 11 * ta + 13 * tb)
    A = rng.normal(0, 1, (K, M) if ta else (M, K))
    B = rng.normal(0, 1, (N, K) if tb else (K, N))
    Ad, Bd = _bf16_dev(A), _bf16_dev(B)
    C = torch.zeros(M * N, dtype=torch.float32, device="cuda")
    L.bmpc_gemm_bf16(M, N, K, Ad, ta, Bd, tb, C)
    torch.cuda.synchronize()
    Aq, Bq = _bf16_host(A), _bf16_host(B)
    Aop = Aq.T if ta else Aq
    Bop = Bq.T if tb else Bq
    ref = Aop @ Bop
    bound = K * 2.0 ** -23 * (np.abs(Aop) @ np.abs(Bop)) + 1e-30
    err = np.abs(C.cpu().numpy().reshape(M, N).astype(np.float64) - ref)
    assert np.all(err <= bound), f"max err/bound {np.max(err / bound):.3f}"


def test_gemm_rejects_double_transpose():
    A = _bf16_dev(np.ones((4, 4)))
    C = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(L.BmpcError) as e:
        L.bmpc_gemm_bf16(4, 4, 4, A, 1, A, 1, C)
    assert e.value.status == 9


def _net(widths, max_batch, params):
    h = L.bmpc_mlp_create(widths, max_batch)
    assert L.bmpc_mlp_num_params(h) == oracle.mlp_num_params(widths)
    L.bmpc_mlp_set_params(h, params)
    return h


@pytest.mark.parametrize("B", [1, 37, 300])
def test_forward_matches_oracle(B):
    print(f"mlp forward B={B}", flush=True)
    rng = np.random.default_rng(100 + B)
    p = _params(WIDTHS, rng)
    X = rng.normal(0, 1, (B, WIDTHS[0])).astype(np.float32)
    h = _net(WIDTHS, 512, p)
    Y = torch.zeros(B * WIDTHS[-1], dtype=torch.float32, device="cuda")
    L.bmpc_mlp_forward(h, torch.from_numpy(X).cuda(), Y)
    torch.cuda.synchronize()
    L.bmpc_mlp_destroy(h)
    want = oracle.mlp_forward(WIDTHS, p.astype(np.float64), X.astype(np.float64), quant=True)
    got = Y.cpu().numpy().reshape(B, -1).astype(np.float64)
    err = np.abs(got - want).max()
    assert err <= 2e-3 * max(1.0, np.abs(want).max()), err


@pytest.mark.parametrize("B", [37, 1024])
def test_gradients_match_oracle(B):
    """Loss and every parameter-block gradient at the network's real widths,
    including the training batch of 1,024."""
    print(f"mlp gradients B={B}", flush=True)
    rng = np.random.default_rng(7)
    p = _params(WIDTHS, rng)
    X = rng.normal(0, 1, (B, WIDTHS[0])).astype(np.float32)
    T = rng.normal(0, 1, (B, WIDTHS[-1])).astype(np.float32)
    h = _net(WIDTHS, max(64, B), p)
    loss, g = L.bmpc_mlp_gradients(h, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    L.bmpc_mlp_destroy(h)
    oloss, og = oracle.mlp_loss_grad(WIDTHS, p.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                                     quant=True)
    assert loss == pytest.approx(oloss, rel=1e-3)
    off = 0
    blocks = [WIDTHS[l] * WIDTHS[l + 1] for l in range(4)] + WIDTHS[1:]
    for i, n in enumerate(blocks):
        gb, ob = g[off:off + n].astype(np.float64), og[off:off + n]
        err = np.abs(gb - ob).max() / np.abs(ob).max()
        print(f"block {i} size {n}: rel err {err:.2e}")
        assert err <= 1e-2, (i, err)
        off += n


def test_adam_step_matches_oracle():
    B = 64
    rng = np.random.default_rng(8)
    p = _params(WIDTHS, rng)
    X = torch.from_numpy(rng.normal(0, 1, (B, WIDTHS[0])).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.normal(0, 1, (B, WIDTHS[-1])).astype(np.float32)).cuda()
    h = _net(WIDTHS, B, p)
    lr = 1e-3
    pp = p.astype(np.float64)
    m, v = np.zeros_like(pp), np.zeros_like(pp)
    for t in (1, 2, 3):
        _, g = L.bmpc_mlp_gradients(h, X, T)
        L.bmpc_mlp_train_step(h, X, T, lr)
        oracle.adam(pp, g.astype(np.float64), m, v, t, lr)
        got = L.bmpc_mlp_get_params(h).astype(np.float64)
        err = np.abs(got - pp)
        assert np.all(err <= 1e-6 * lr * 10 + 2 ** -23 * np.abs(pp) * 2), (t, err.max())
    L.bmpc_mlp_destroy(h)


def test_training_reduces_loss_on_teacher_targets():
    B = 1024
    rng = np.random.default_rng(9)
    teacher = _params(WIDTHS, rng)
    X = torch.from_numpy(rng.normal(0, 1, (B, WIDTHS[0])).astype(np.float32)).cuda()
    ht = _net(WIDTHS, B, teacher)
    T = torch.zeros(B * WIDTHS[-1], dtype=torch.float32, device="cuda")
    L.bmpc_mlp_forward(ht, X, T)
    L.bmpc_mlp_destroy(ht)
    T = T.view(B, -1)
    hs = _net(WIDTHS, B, _params(WIDTHS, np.random.default_rng(10)))
    first = L.bmpc_mlp_train_step(hs, X, T, 1e-3)
    for _ in range(300):
        L.bmpc_mlp_train_step(hs, X, T, 1e-3, want_loss=False)
    last = L.bmpc_mlp_train_step(hs, X, T, 1e-3)
    L.bmpc_mlp_destroy(hs)
    print(f"teacher fit: loss {first:.4f} -> {last:.4f}")
    assert last < 0.3 * first


def test_batch_bounds_rejected():
    h = L.bmpc_mlp_create([4, 8, 2], 16)
    X = torch.zeros(17 * 4, dtype=torch.float32, device="cuda").view(17, 4)
    Y = torch.zeros(17 * 2, dtype=torch.float32, device="cuda")
    with pytest.raises(L.BmpcError) as e:
        L.bmpc_mlp_forward(h, X, Y)
    assert e.value.status == 1
    with pytest.raises(L.BmpcError) as e:
        L.bmpc_mlp_set_params(h, np.full(L.bmpc_mlp_num_params(h), np.nan, dtype=np.float32))
    assert e.value.status == 4
    L.bmpc_mlp_destroy(h)


def test_input_map_matches_oracle_on_mapped_inputs():
    """The FP32 input map (x - shift) * scale runs before the BF16 rounding;
    the same FP32 operations on the host followed by the oracle agree."""
    B = 29
    rng = np.random.default_rng(12)
    p = _params(WIDTHS, rng)
    X = (rng.normal(0, 1, (B, WIDTHS[0])) * 3 + 20).astype(np.float32)
    shift = rng.normal(20, 1, WIDTHS[0]).astype(np.float32)
    scale = rng.uniform(0.2, 2.0, WIDTHS[0]).astype(np.float32)
    h = _net(WIDTHS, 64, p)
    L.bmpc_mlp_set_input_map(h, shift, scale)
    Y = torch.zeros(B * WIDTHS[-1], dtype=torch.float32, device="cuda")
    L.bmpc_mlp_forward(h, torch.from_numpy(X).cuda(), Y)
    torch.cuda.synchronize()
    L.bmpc_mlp_destroy(h)
    Xm = ((X - shift[None, :]) * scale[None, :]).astype(np.float32)
    want = oracle.mlp_forward(WIDTHS, p.astype(np.float64), Xm.astype(np.float64), quant=True)
    got = Y.cpu().numpy().reshape(B, -1).astype(np.float64)
    assert np.abs(got - want).max() <= 2e-3 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("B", [256, 512, 1000])
def test_gradients_split_batch_match_oracle(B):
    """Large batches split the weight-gradient reduction over several
    workgroups and sum the parts in a fixed order."""
    widths = [44, 64, 64, 96]
    rng = np.random.default_rng(B)
    p = _params(widths, rng)
    X = rng.normal(0, 1, (B, widths[0])).astype(np.float32)
    T = rng.normal(0, 1, (B, widths[-1])).astype(np.float32)
    h = _net(widths, 1024, p)
    loss, g = L.bmpc_mlp_gradients(h, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    _, g2 = L.bmpc_mlp_gradients(h, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    L.bmpc_mlp_destroy(h)
    assert np.array_equal(g, g2)  # deterministic
    oloss, og = oracle.mlp_loss_grad(widths, p.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                                     quant=True)
    assert loss == pytest.approx(oloss, rel=1e-3)
    off = 0
    blocks = [widths[l] * widths[l + 1] for l in range(3)] + widths[1:]
    for i, n in enumerate(blocks):
        err = np.abs(g[off:off + n].astype(np.float64) - og[off:off + n]).max() / np.abs(og[off:off + n]).max()
        assert err <= 1e-2, (i, err)
        off += n
