"""FP8 e4m3 path: codes bit-exact, GEMM exact in float32, blocks vs the oracle.

The paper fixes no FP8 tolerance; blocks are checked against a sanity bound
of 1e-1 relative L2 and the measured errors are printed.
"""
import numpy as np
import pytest

import wm_synth as S
from oracle import wm_oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2503_22235_amd as wm
    assert torch.cuda.is_available()
    ctx = wm.wm_ctx_create(0)
    yield wm, torch, ctx
    ctx.close()


def test_quantize_codes_bit_exact(env):
    wm, torch, ctx = env
    r = np.random.default_rng(0)
    x = np.concatenate([r.standard_normal(200000) * 30, r.standard_normal(2000) * 1e-3,
                        np.array([448.0, -448.0, 1e4, -1e4, 0.0, -0.0, 2.0 ** -10, 3 * 2.0 ** -11])]
                       ).astype(np.float32)
    for mul in (1.0, 0.37, 7.5):
        prod = (x * np.float32(mul)).astype(np.float32)       # the kernel's float32 product
        ref = O.e4m3_encode(prod)
        out = torch.empty(x.size, dtype=torch.uint8, device="cuda")
        wm.wm_quantize_fp8(torch.from_numpy(x).cuda(), mul, out)
        got = out.cpu().numpy()
        # signed zero: both encodings of zero are zero
        ref0, got0 = ref & 0x7F == 0, got & 0x7F == 0
        assert np.array_equal(ref0, got0)
        assert np.array_equal(ref[~ref0], got[~got0]), (mul, np.argwhere(ref != got)[:5])


@pytest.mark.parametrize("epi", [0, 1, 2])
def test_linear_fp8(env, epi):
    wm, torch, ctx = env
    r = np.random.default_rng(1 + epi)
    # N = 512 takes the row walk (two row blocks of one feature tile per
    # workgroup): 6 row blocks with a 1-row tail, and an odd count (3) whose
    # last workgroup has a single, ragged tile
    for M, N, K in ((1000, 384, 128), (300, 128, 512), (129, 256, 256), (1281, 512, 512), (700, 512, 2048)):
        say("linear fp8", epi, M, N, K)
        a8 = O.e4m3_encode(r.standard_normal((M, K)) * 40)
        w8 = O.e4m3_encode(r.standard_normal((N, K)) * 40)
        ad, wd = 0.02, 0.005
        b = (0.1 * r.standard_normal(N)).astype(np.float32)
        ref = (O.e4m3_decode(a8) @ O.e4m3_decode(w8).T) * ad * wd + b
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        if epi == 2:
            x0 = r.standard_normal((M, N)).astype(np.float32)
            out = dev(x0)
            ref = x0 + ref
        else:
            out = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
            if epi == 1:
                ref = O.gelu(ref)
        wm.wm_linear_fp8(M, N, K, dev(a8), ad, dev(w8), wd, dev(b), epi, out)
        got = out.float().cpu().numpy()
        # fp8 products are exact in float32, but the fp8 MFMA's internal
        # dot-product accumulation is not exact float32 (about 1e-5 relative
        # measured on the residual output); bf16 outputs add their rounding.
        tol = 1e-4 if epi == 2 else 5e-3
        assert O.rel_l2(got, ref) < tol


def test_fp8_block_small_and_batch_invariance(env):
    wm, torch, ctx = env
    g = S.CFG1
    params = S.processor_params(g, 1, 1)
    x = S.latent_state(g, 3, 0)
    p = wm.wm_processor_create(ctx, g, 1, 4, wm.WM_FP8_E4M3, params)
    xb = torch.from_numpy(x).cuda()
    wm.wm_processor_block(ctx, p, 0, 3, xb)
    x1 = torch.from_numpy(x[1:2].copy()).cuda()
    wm.wm_processor_block(ctx, p, 0, 1, x1)
    assert torch.equal(xb[1:2], x1), "a state's FP8 result depends on its batch"
    ref = O.block(x[1], S.split_block_params(g, params, 0), g)
    got = x1.cpu().numpy()[0]
    err, inc = O.rel_l2(got, ref), O.rel_l2(got - x[1], ref - x[1])
    say(f"fp8 block cfg1 rel_l2={err:.3e} increment={inc:.3e}")
    assert err < 1e-1
    p.close()


def test_fp8_blocks_full_size_sampled(env):
    """Each block of the 8-block processor at 8x90x180 on a batch of 4
    states; outputs of state 2 checked at sampled tokens."""
    wm, torch, ctx = env
    g = S.CFG2
    nb = 8
    params = S.processor_params(g, nb, 1)
    x = S.latent_state(g, 4, 0)
    r = np.random.default_rng(5)
    tok = np.unique(np.concatenate([r.choice(g.T, 300, replace=False), np.arange(0, g.X, 6)]))
    p = wm.wm_processor_create(ctx, g, nb, 4, wm.WM_FP8_E4M3, params)
    xd = torch.from_numpy(x).cuda()
    for b in range(nb):
        y = xd.clone()
        wm.wm_processor_block(ctx, p, b, 4, y)
        got = y[2].reshape(g.T, g.C)[torch.from_numpy(tok).cuda()].cpu().numpy()
        ref = O.block_at(x[2], S.split_block_params(g, params, b), g, tok)
        xs = x[2].reshape(g.T, g.C)[tok]
        err, inc = O.rel_l2(got, ref), O.rel_l2(got - xs, ref - xs)
        say(f"fp8 block {b} rel_l2={err:.3e} increment={inc:.3e}")
        assert err < 1e-1
        assert inc < 1e-1
    p.close()


def test_fp8_block_smooth_field_sampled(env):
    """One full-size block on a smooth latent field (low-order lat/lon/level
    modes + 0.1 noise) instead of i.i.d. noise: FP8 error, with BF16 beside
    it, at sampled tokens.  Per-state FP8 scales see the field's dynamic
    range; the paper fixes no FP8 tolerance, so the FP8 error is printed
    and held to the same sanity bound as the i.i.d. case."""
    wm, torch, ctx = env
    g = S.CFG2
    params = S.processor_params(g, 1, 1)
    x = S.smooth_state(g, 1, 0)
    r = np.random.default_rng(7)
    tok = np.unique(np.concatenate([r.choice(g.T, 300, replace=False), np.arange(0, g.X, 6)]))
    ref = O.block_at(x[0], S.split_block_params(g, params, 0), g, tok)
    xs = x[0].reshape(g.T, g.C)[tok]
    errs = {}
    for prec, name in ((wm.WM_FP8_E4M3, "fp8"), (wm.WM_BF16, "bf16")):
        p = wm.wm_processor_create(ctx, g, 1, 4, prec, params)
        y = torch.from_numpy(x.copy()).cuda()
        wm.wm_processor_block(ctx, p, 0, 1, y)
        got = y[0].reshape(g.T, g.C)[torch.from_numpy(tok).cuda()].cpu().numpy()
        errs[name] = (O.rel_l2(got, ref), O.rel_l2(got - xs, ref - xs))
        say(f"smooth field {name} block rel_l2={errs[name][0]:.3e} increment={errs[name][1]:.3e}")
        p.close()
    assert errs["bf16"][0] < 1e-2
    assert errs["fp8"][0] < 1e-1


# ---------------------------------------------------------------------------
# FP8 attention (QK and PV on e4m3 codes).  The parity reference is the
# oracle's attention applied to q, k, v quantized with the oracle's e4m3
# codec at each (state, tensor) scale amax/448; the only further GPU
# rounding is that of the softmax weights (e4m3 has 3 mantissa bits: a
# relative rounding error of at most 2^-4, about 3.6% rms) and of the bf16
# output, averaged over the window: bound 0.04 relative L2.  Against the
# unquantized oracle the error depends on how sharp the softmax is (score
# errors scale with |q| |k|): about 5% for N(0,1) inputs, 9% for the state
# with q x 3 and k x 2; it is printed and held to a sanity bound of 0.15.

FP8_NAT_GRIDS = [
    S.Grid(Z=5, Y=45, X=90, C=128, heads=4, Kz=3, Ky=5, Kx=5, periodic_mask=4),
    S.Grid(Z=3, Y=10, X=21, C=128, heads=4, Kz=3, Ky=5, Kx=5, periodic_mask=4),
    S.Grid(Z=8, Y=16, X=24, C=64, heads=2, Kz=5, Ky=7, Kx=7, periodic_mask=4),
    S.Grid(Z=4, Y=9, X=12, C=64, heads=2, Kz=3, Ky=3, Kx=3, periodic_mask=4),
    # 5x7x7 with ragged query tiles in lat (18 = 4 x 4 + 2) and lon (20 = 2 x 8 + 4)
    S.Grid(Z=8, Y=18, X=20, C=64, heads=2, Kz=5, Ky=7, Kx=7, periodic_mask=4),
]


def _bf16(torch, a):
    return torch.from_numpy(a).to(torch.bfloat16).float().numpy().astype(np.float64)


def _q8(x, amax):
    s = amax / 448.0 if amax > 0 else 1.0
    return O.e4m3_decode(O.e4m3_encode(x / s)) * s


def _nat_fp8(env, g, q, k, v, rpb):
    wm, torch, ctx = env
    dev = [torch.from_numpy(a.astype(np.float32)).cuda().to(torch.bfloat16) for a in (q, k, v)]
    out = torch.empty(q.shape, dtype=torch.bfloat16, device="cuda")
    wm.wm_nat_forward(ctx, g, q.shape[0], wm.WM_FP8_E4M3, dev[0], dev[1], dev[2],
                      torch.from_numpy(rpb.astype(np.float32)).cuda(), out)
    return out.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("gi", range(len(FP8_NAT_GRIDS)))
def test_nat_fp8_against_quantized_operands(env, gi):
    wm, torch, ctx = env
    g = FP8_NAT_GRIDS[gi]
    B = 2
    r = np.random.default_rng(40 + gi)
    shape = (B, g.T, g.heads, 32)
    # state 1 gets larger q and k (a different per-state scale)
    q = _bf16(torch, r.standard_normal(shape) * np.array([1.0, 3.0])[:, None, None, None])
    k = _bf16(torch, r.standard_normal(shape) * np.array([1.0, 2.0])[:, None, None, None])
    v = _bf16(torch, r.standard_normal(shape))
    rpb = r.standard_normal(g.rpb_shape).astype(np.float32).astype(np.float64)
    got = _nat_fp8(env, g, q, k, v, rpb)
    for b in range(B):
        exact = O.neighborhood_attention(q[b], k[b], v[b], rpb, g)
        quant = O.neighborhood_attention(_q8(q[b], np.abs(q[b]).max()), _q8(k[b], np.abs(k[b]).max()),
                                         _q8(v[b], np.abs(v[b]).max()), rpb, g)
        e_q, e_x = O.rel_l2(got[b], quant), O.rel_l2(got[b], exact)
        say(f"fp8 nat {g.Z}x{g.Y}x{g.X} K={g.Kz}{g.Ky}{g.Kx} state {b}: vs quantized-operand reference "
            f"{e_q:.4f}, vs exact {e_x:.4f}")
        assert e_q < 0.04
        assert e_x < 0.15


def test_nat_fp8_exact_when_weights_are_equal(env):
    """q = 0 and a zero bias make every window weight 1 (exact in e4m3);
    values of v that are e4m3 codes at the state's scale then make the
    result the plain window mean up to float32 sums and bf16 output."""
    wm, torch, ctx = env
    g = FP8_NAT_GRIDS[2]
    r = np.random.default_rng(3)
    shape = (1, g.T, g.heads, 32)
    q = np.zeros(shape)
    k = _bf16(torch, r.standard_normal(shape))
    v = r.choice([-2.0, -1.0, -0.5, -0.25, 0.0, 0.25, 0.5, 1.0, 2.0], size=shape)
    v.flat[0] = 2.0                           # amax 2: v * 448 / 2 are e4m3 codes
    rpb = np.zeros(g.rpb_shape)
    got = _nat_fp8(env, g, q, k, v, rpb)
    ref = O.neighborhood_attention(q[0], k[0], v[0], rpb, g)
    err = np.abs(got[0] - ref).max()
    say(f"fp8 nat equal weights: max abs error {err:.2e}")
    assert err <= 2.0 ** -8 * 2.0 + 1e-6      # one bf16 rounding of a value of magnitude <= 2


def test_fp8_block_batch_17_row_chunks(env):
    """17 states at 8x90x180: the e4m3 GEMM operands exceed 2 GiB, so the
    GEMMs run in row chunks; the last state's result must equal its result
    alone (per-state scales, bit for bit)."""
    wm, torch, ctx = env
    g = S.CFG2
    params = S.processor_params(g, 1, 1)
    B = 17
    p = wm.wm_processor_create(ctx, g, 1, 4, wm.WM_FP8_E4M3, params)
    xb = torch.empty((B,) + (g.Z, g.Y, g.X, g.C), device="cuda")
    for b in range(B):
        xb[b] = torch.from_numpy(S.latent_state(g, 1, seed=0, index0=b)[0]).cuda()
    x1 = xb[B - 1:B].clone()
    say("fp8 block batch", B)
    wm.wm_processor_block(ctx, p, 0, B, xb)
    wm.wm_processor_block(ctx, p, 0, 1, x1)
    assert torch.equal(xb[B - 1:B], x1)
    p.close()


def test_nat_fp8_full_size_against_quantized_operands(env):
    """FP8 attention alone at 8 x 90 x 180, 16 heads, window 5x7x7 (ragged
    query tiles in lat and lon, poles, the lon seam), every output, two
    states with different per-state scales; reference: the oracle (C loops)
    on q, k, v quantized by the oracle's e4m3 codec."""
    wm, torch, ctx = env
    g = S.CFG2
    B = 2
    r = np.random.default_rng(60)
    shape = (B, g.T, g.heads, 32)
    q = _bf16(torch, r.standard_normal(shape) * np.array([1.0, 3.0])[:, None, None, None])
    k = _bf16(torch, r.standard_normal(shape) * np.array([1.0, 2.0])[:, None, None, None])
    v = _bf16(torch, r.standard_normal(shape))
    rpb = r.standard_normal(g.rpb_shape).astype(np.float32).astype(np.float64)
    say("fp8 nat full size")
    got = _nat_fp8(env, g, q, k, v, rpb)
    for b in range(B):
        quant = O.nat_c(_q8(q[b], np.abs(q[b]).max()), _q8(k[b], np.abs(k[b]).max()),
                        _q8(v[b], np.abs(v[b]).max()), rpb, g)
        e_q = O.rel_l2(got[b], quant)
        say(f"fp8 nat 8x90x180 state {b}: vs quantized-operand reference {e_q:.4f}")
        assert e_q < 0.04
