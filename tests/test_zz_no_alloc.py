"""wm_nat_forward_noalloc (the attention entry point that allocates nothing)
against wm_nat_forward, through the C ABI.

The no-allocation variant keeps its scratch (bias tables, FP8 amax slots)
in a fixed device array that every call on the GPU shares.  Each precision
makes two calls in a row, the second on a smaller input, so the second call
runs on the scratch the first one left behind.  FP32 and BF16 run the same
arithmetic as wm_nat_forward (BF16 on token-major v instead of the blocked
copy wm_nat_forward makes in its workspace, with the same key order) and
must be bit-identical to it.  FP8: wm_nat_forward quantizes k and v once
into its workspace for the level-ring kernel, while the no-allocation
variant (whose scratch holds no copies of k and v) runs the tiled kernel
that quantizes as it stages.  Both take the same e4m3 codes of q, k and v,
but the softmax weights are rounded to e4m3 relative to different
references (the tiled kernel's running maximum, the ring kernel's own
score of each query), so the two differ by a few e4m3 steps of the
weights; they are held to each other with the FP8 attention tolerance
(0.04, the bound against the oracle on quantized operands).  The first
call of each precision is also held to the oracle (FP8: both entry points).
"""
import numpy as np
import pytest

import wm_synth as S
from oracle import wm_oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _grid(Z, Y, X, C, heads, Kz, Ky, Kx, pm=0x4):
    return S.Grid(Z=Z, Y=Y, X=X, C=C, heads=heads, Kz=Kz, Ky=Ky, Kx=Kx, periodic_mask=pm)


# (precision, grid, batch): per precision a larger call, then a smaller one
CASES = {
    1: [(_grid(8, 16, 24, 128, 4, 5, 7, 7), 2), (_grid(3, 10, 21, 64, 2, 3, 5, 5), 1)],
    2: [(_grid(8, 18, 20, 128, 4, 5, 7, 7), 3), (_grid(3, 10, 21, 64, 2, 3, 5, 5), 1)],
    0: [(_grid(4, 9, 12, 128, 4, 3, 5, 5), 2), (_grid(2, 5, 6, 64, 2, 1, 5, 3, 0x5), 1)],
}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2503_22235_amd as wm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wm.lib()
    ctx = wm.wm_ctx_create(0)
    yield wm, torch, ctx
    torch.cuda.synchronize()
    ctx.close()


def _q8(x):
    """x quantized to e4m3 at the scale amax/448 by the oracle's codec."""
    amax = np.abs(x).max()
    s = amax / 448.0 if amax > 0 else 1.0
    return O.e4m3_decode(O.e4m3_encode(x / s)) * s


def _inputs(torch, g, B, prec, seed):
    r = np.random.default_rng(seed)
    shape = (B, g.T, g.heads, 32)
    q, k, v = (r.standard_normal(shape).astype(np.float32) * s for s in (2.0, 2.0, 1.0))
    rpb = r.standard_normal(g.rpb_shape).astype(np.float32)
    dt = torch.float32 if prec == 0 else torch.bfloat16
    dev = [torch.from_numpy(a).cuda().to(dt) for a in (q, k, v)]
    host = [d.float().cpu().numpy().astype(np.float64) for d in dev]   # what the kernels see
    return dev, host, torch.from_numpy(rpb).cuda(), rpb


@pytest.mark.parametrize("prec", [1, 2, 0])
def test_noalloc_matches_nat_forward(env, prec):
    wm, torch, ctx = env
    for i, (g, B) in enumerate(CASES[prec]):
        say(f"noalloc prec={prec} call={i} grid={g} B={B}")
        dev, host, rpb_d, rpb = _inputs(torch, g, B, prec, seed=10 * prec + i)
        out_na = torch.full_like(dev[0], float("nan"))
        out_ref = torch.full_like(dev[0], float("nan"))
        wm.wm_nat_forward_noalloc(g, B, prec, dev[0], dev[1], dev[2], rpb_d, out_na)
        wm.wm_nat_forward(ctx, g, B, prec, dev[0], dev[1], dev[2], rpb_d, out_ref)
        torch.cuda.synchronize()
        got = out_na.float().cpu().numpy()
        if prec == 2:
            d = O.rel_l2(got, out_ref.float().cpu().numpy())
            say(f"  rel_l2 vs wm_nat_forward {d:.3e} (tol 0.04)")
            assert d <= 0.04, (prec, i)
        else:
            assert torch.equal(out_na.view(torch.int16 if prec else torch.int32),
                               out_ref.view(torch.int16 if prec else torch.int32)), (prec, i)
        if i == 0:
            outs = [got]
            if prec == 2:
                # e4m3 operands: the oracle on q, k, v quantized by its own codec
                ref = np.stack([O.nat_c(*(_q8(h[b]) for h in host), rpb, g) for b in range(B)])
                tol = 0.04
                outs.append(out_ref.float().cpu().numpy())
            else:
                ref = np.stack([O.nat_c(host[0][b], host[1][b], host[2][b], rpb, g) for b in range(B)])
                tol = 1e-5 if prec == 0 else 1e-2
            for o in outs:
                err = O.rel_l2(o, ref)
                say(f"  rel_l2 vs oracle {err:.3e} (tol {tol})")
                assert err <= tol
