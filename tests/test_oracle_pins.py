"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every check below compares the oracle with something other than itself:
brute-force enumeration, textbook library routines (dense attention,
LayerNorm, GELU from torch / scipy), closed forms, invariants and the hand
enumerated schedule.  Each names the kind of mistake it would catch.
"""
import math
import os

import numpy as np
import pytest

import wm_synth as S
from oracle import wm_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(Z=3, Y=6, X=7, C=16, heads=2, Kz=3, Ky=3, Kx=3, periodic_mask=0x4):
    return S.Grid(Z=Z, Y=Y, X=X, C=C, heads=heads, Kz=Kz, Ky=Ky, Kx=Kx,
                  periodic_mask=periodic_mask)


def rand_qkv(g, seed=0, scale=1.0):
    r = np.random.default_rng(seed)
    shape = (g.T, g.heads, g.d)
    return (r.standard_normal(shape) * scale, r.standard_normal(shape) * scale,
            r.standard_normal(shape), r.standard_normal(g.rpb_shape))


# --------------------------------------------------------------------------
# Windows (Sec. 2.1 NATTEN, App. A.2 circular padding / bump attention).
# --------------------------------------------------------------------------
def test_clamped_window_is_nearest_full_window():
    """Brute force: the clamped window is the full-size in-range window whose
    centre is closest to the query (unique for odd K).  Catches off-by-one
    clamp bounds and a window that shrinks instead of shifting."""
    for N in range(1, 41):
        for K in range(1, N + 1, 2):
            r = (K - 1) // 2
            keys, off = O.window_axis(N, K, periodic=False)
            for i in range(N):
                cands = list(range(0, N - K + 1))
                best = min(cands, key=lambda s: abs(s + r - i))
                assert sum(abs(s + r - i) == abs(best + r - i) for s in cands) == 1
                assert list(keys[i]) == list(range(best, best + K))
                assert list(off[i]) == [j - i for j in range(best, best + K)]
                assert i in keys[i]


def test_periodic_window_is_wrapped_centered_set():
    """Periodic axis: the key set is {(i + delta) mod N : |delta| <= r} in
    increasing delta; offsets are the deltas.  Catches a one-sided window or
    a sign error in the wrap."""
    for N in range(1, 30):
        for K in range(1, N + 1, 2):
            r = (K - 1) // 2
            keys, off = O.window_axis(N, K, periodic=True)
            for i in range(N):
                exp_keys = [(i + dl) % N for dl in range(-r, r + 1)]
                assert list(keys[i]) == exp_keys
                assert list(off[i]) == list(range(-r, r + 1))


def test_invalid_windows_rejected():
    for N, K in ((5, 2), (5, 7), (4, 0)):
        with pytest.raises(ValueError):
            O.window_axis(N, K, False)


# --------------------------------------------------------------------------
# Neighborhood attention.
# --------------------------------------------------------------------------
def _dense_offset(i, j, N, periodic):
    dl = j - i
    if periodic:
        r = (N - 1) // 2
        if dl > r:
            dl -= N
        if dl < -r:
            dl += N
    return dl


def test_full_window_equals_dense_attention():
    """When the window covers the whole grid, neighborhood attention is plain
    softmax attention with the bias looked up from coordinate differences.
    The dense side uses torch's scaled_dot_product_attention in float64.
    Catches a wrong scale, a swapped q/k role, a bias sign or axis-order
    error."""
    import torch
    g = tiny(Z=3, Y=5, X=5, Kz=3, Ky=5, Kx=5)
    q, k, v, rpb = rand_qkv(g, 1)
    o = O.neighborhood_attention(q, k, v, rpb, g)
    oc = O.nat_c(q, k, v, rpb, g)
    coords = [(z, y, x) for z in range(g.Z) for y in range(g.Y) for x in range(g.X)]
    bias = np.zeros((g.heads, g.T, g.T))
    for n, (z, y, x) in enumerate(coords):
        for m, (zz, yy, xx) in enumerate(coords):
            dz = _dense_offset(z, zz, g.Z, False)
            dy = _dense_offset(y, yy, g.Y, False)
            dx = _dense_offset(x, xx, g.X, True)
            bias[:, n, m] = rpb[:, dz + g.Kz - 1, dy + g.Ky - 1, dx + g.Kx - 1]
    tq = torch.from_numpy(q).permute(1, 0, 2)
    tk = torch.from_numpy(k).permute(1, 0, 2)
    tv = torch.from_numpy(v).permute(1, 0, 2)
    ref = torch.nn.functional.scaled_dot_product_attention(
        tq, tk, tv, attn_mask=torch.from_numpy(bias)).permute(1, 0, 2).numpy()
    assert np.abs(o - ref).max() < 1e-13
    assert np.abs(oc - ref).max() < 1e-13


def test_unit_window_returns_v_exactly():
    g = tiny(Kz=1, Ky=1, Kx=1)
    q, k, v, rpb = rand_qkv(g, 2)
    assert np.array_equal(O.neighborhood_attention(q, k, v, rpb, g), v)
    assert np.array_equal(O.nat_c(q, k, v, rpb, g), v)


def test_softmax_rows_sum_to_one():
    g = tiny(Z=4, Y=7, X=9, Kz=3, Ky=5, Kx=5)
    q, k, v, rpb = rand_qkv(g, 3, scale=3.0)
    _, p = O.neighborhood_attention(q, k, v, rpb, g, return_probs=True)
    _, pc = O.nat_c(q, k, v, rpb, g, return_probs=True)
    assert np.abs(p.sum(-1) - 1).max() < 1e-15 * 8
    assert np.abs(pc.sum(-1) - 1).max() < 1e-15 * 8
    assert (p >= 0).all()


def test_pad_and_crop_equivalence():
    """Circular padding in longitude (App. A.2): padding lon by p >= r with
    wrapped copies, running attention with a clamped lon axis and cropping
    gives exactly the periodic result.  Catches a wrong periodic offset."""
    g = tiny(Z=3, Y=5, X=8, Kz=3, Ky=3, Kx=5)
    q, k, v, rpb = rand_qkv(g, 4)
    o = O.neighborhood_attention(q, k, v, rpb, g)
    for p in (2, 3):
        gp = S.Grid(Z=g.Z, Y=g.Y, X=g.X + 2 * p, C=g.C, heads=g.heads,
                    Kz=g.Kz, Ky=g.Ky, Kx=g.Kx, periodic_mask=0)

        def pad(a):
            a = a.reshape(g.Z, g.Y, g.X, g.heads, g.d)
            return np.pad(a, ((0, 0), (0, 0), (p, p), (0, 0), (0, 0)),
                          mode="wrap").reshape(gp.T, g.heads, g.d)
        op = O.neighborhood_attention(pad(q), pad(k), pad(v), rpb, gp)
        op = op.reshape(g.Z, g.Y, gp.X, g.heads, g.d)[:, :, p:p + g.X]
        assert np.array_equal(op.reshape(o.shape), o)


def test_roll_equivariance_lon_bit_exact():
    g = tiny(Z=3, Y=5, X=9, Kz=3, Ky=3, Kx=5)
    q, k, v, rpb = rand_qkv(g, 5)

    def roll(a, s):
        return np.roll(a.reshape(g.Z, g.Y, g.X, -1), s, axis=2).reshape(a.shape)
    o = O.neighborhood_attention(q, k, v, rpb, g)
    oc = O.nat_c(q, k, v, rpb, g)
    for s in (1, 4, -2):
        assert np.array_equal(O.neighborhood_attention(roll(q, s), roll(k, s), roll(v, s), rpb, g), roll(o, s))
        assert np.array_equal(O.nat_c(roll(q, s), roll(k, s), roll(v, s), rpb, g), roll(oc, s))


def test_translation_equivariance_interior_lat_level():
    """Away from the borders a shift in lat or level shifts the output."""
    g = tiny(Z=6, Y=9, X=5, Kz=3, Ky=3, Kx=3)
    q, k, v, rpb = rand_qkv(g, 6)
    o = O.nat_c(q, k, v, rpb, g).reshape(g.Z, g.Y, g.X, g.heads, g.d)
    sh = lambda a, ax: np.roll(a.reshape(g.Z, g.Y, g.X, g.heads, g.d), 1, axis=ax).reshape(a.shape)
    oz = O.nat_c(sh(q, 0), sh(k, 0), sh(v, 0), rpb, g).reshape(o.shape)
    oy = O.nat_c(sh(q, 1), sh(k, 1), sh(v, 1), rpb, g).reshape(o.shape)
    # query z+1 has an unclamped window that never touches the wrapped slab
    assert np.array_equal(oz[3:g.Z - 1], o[2:g.Z - 2])
    assert np.array_equal(oy[:, 3:g.Y - 1], o[:, 2:g.Y - 2])


def test_bias_offset_probe():
    """q = 0 and a bias of +60 at one offset delta*: every query takes the
    value of the key at query + delta* when its (possibly shifted) window
    holds that offset, and the plain window mean otherwise.  Catches bias
    index sign errors, axis swaps and wrong border offsets."""
    g = tiny(Z=4, Y=6, X=7, heads=1, C=8, Kz=3, Ky=3, Kx=5)
    r = np.random.default_rng(7)
    q = np.zeros((g.T, 1, g.d))
    k = r.standard_normal((g.T, 1, g.d))
    v = r.standard_normal((g.T, 1, g.d))
    dstar = (1, -2, 2)
    rpb = np.zeros(g.rpb_shape)
    rpb[0, dstar[0] + g.Kz - 1, dstar[1] + g.Ky - 1, dstar[2] + g.Kx - 1] = 60.0
    o = O.nat_c(q, k, v, rpb, g)
    on = O.neighborhood_attention(q, k, v, rpb, g)
    vv = v.reshape(g.Z, g.Y, g.X, g.d)
    hits = 0
    for z in range(g.Z):
        for y in range(g.Y):
            for x in range(g.X):
                n = (z * g.Y + y) * g.X + x
                # which z/y windows hold the offset: brute force over starts
                sz = min(max(z - 1, 0), g.Z - 3)
                sy = min(max(y - 1, 0), g.Y - 3)
                zt, yt = z + dstar[0], y + dstar[1]
                if sz <= zt < sz + 3 and sy <= yt < sy + 3:
                    expect = vv[zt, yt, (x + dstar[2]) % g.X]
                    hits += 1
                    assert np.abs(o[n, 0] - expect).max() < 1e-20
                else:
                    win = vv[sz:sz + 3, sy:sy + 3][:, :, [(x + t) % g.X for t in range(-2, 3)]]
                    assert np.abs(o[n, 0] - win.reshape(-1, g.d).mean(0)).max() < 1e-14
    assert hits > 0
    assert np.abs(o - on).max() < 1e-15


def test_bias_shift_invariance_linearity_heads():
    g = tiny(Z=3, Y=5, X=6, Kz=3, Ky=3, Kx=3, heads=2, C=16)
    q, k, v, rpb = rand_qkv(g, 8)
    o = O.nat_c(q, k, v, rpb, g)
    assert np.abs(O.nat_c(q, k, v, rpb + 3.25, g) - o).max() < 1e-14
    v2 = np.random.default_rng(9).standard_normal(v.shape)
    lin = O.nat_c(q, k, 2.0 * v - 0.5 * v2, rpb, g)
    assert np.abs(lin - (2.0 * o - 0.5 * O.nat_c(q, k, v2, rpb, g))).max() < 1e-13
    # heads are independent: changing head 1 leaves head 0 untouched
    q2 = q.copy()
    q2[:, 1] += 1.0
    o2 = O.nat_c(q2, k, v, rpb, g)
    assert np.array_equal(o2[:, 0], o[:, 0]) and not np.array_equal(o2[:, 1], o[:, 1])


def test_c_and_numpy_attention_agree_small_configs():
    for g in (tiny(), tiny(Z=5, Y=8, X=10, Kz=3, Ky=5, Kx=7, periodic_mask=0x5),
              tiny(Z=2, Y=3, X=4, Kz=1, Ky=3, Kx=3, periodic_mask=0x7)):
        q, k, v, rpb = rand_qkv(g, 10)
        assert np.abs(O.nat_c(q, k, v, rpb, g)
                      - O.neighborhood_attention(q, k, v, rpb, g)).max() < 1e-14


# --------------------------------------------------------------------------
# Block pieces against textbook routines and closed forms.
# --------------------------------------------------------------------------
def test_layernorm_closed_forms():
    a = 0.37
    y = O.layer_norm(np.array([a, -a]), np.ones(2), np.zeros(2))
    expect = a / math.sqrt(a * a + O.LN_EPS)
    assert abs(y[0] - expect) < 1e-15 and abs(y[1] + expect) < 1e-15
    assert np.allclose(O.layer_norm(np.full(8, 3.5), np.ones(8), np.arange(8.0)),
                       np.arange(8.0), atol=0)
    r = np.random.default_rng(11)
    x = r.standard_normal((50, 32)) * 4 + 1
    y = O.layer_norm(x, np.ones(32), np.zeros(32))
    var = x.var(axis=-1)
    assert np.abs(y.mean(-1)).max() < 1e-14
    assert np.abs(y.var(-1) - var / (var + O.LN_EPS)).max() < 1e-13


def test_layernorm_gelu_vs_torch():
    import torch
    r = np.random.default_rng(12)
    x = r.standard_normal((20, 24))
    gm, bt = r.standard_normal(24), r.standard_normal(24)
    ref = torch.nn.functional.layer_norm(torch.from_numpy(x), (24,), torch.from_numpy(gm),
                                         torch.from_numpy(bt), eps=1e-5).numpy()
    assert np.abs(O.layer_norm(x, gm, bt) - ref).max() < 1e-13
    z = np.linspace(-8, 8, 1001)
    refg = torch.nn.functional.gelu(torch.from_numpy(z)).numpy()
    assert np.abs(O.gelu(z) - refg).max() < 1e-15
    # GELU(z) = z * Phi(z); Phi(1) = 0.8413447460685429
    assert abs(O.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(O.gelu(np.array(-1.0)) + 0.15865525393145707) < 1e-15


def _params(g, seed=1, std=0.2):
    return S.split_block_params(g, S.processor_params(g, 1, seed, std=std), 0)


def test_block_with_zero_output_maps_is_identity():
    g = tiny()
    p = dict(_params(g))
    for name in ("w_o", "b_o", "w_2", "b_2"):
        p[name] = np.zeros_like(p[name])
    x = S.latent_state(g, 2, 0)
    assert np.array_equal(O.block(x, p, g), x.astype(np.float64))


def test_full_window_block_equals_dense_transformer_block():
    """With the window spanning the grid the block is a standard pre-norm
    transformer block with additive attention bias, built here from torch's
    float64 linear / layer_norm / scaled_dot_product_attention / gelu.
    Catches misplaced norms, missing residuals or biases, transposed maps."""
    import torch
    F = torch.nn.functional
    g = tiny(Z=3, Y=3, X=5, Kz=3, Ky=3, Kx=5, C=16, heads=2)
    p = _params(g, 3)
    x = S.latent_state(g, 1, 0)[0]
    y = O.block(x, p, g)
    t = {k: torch.from_numpy(np.asarray(v, np.float64)) for k, v in p.items()}
    xt = torch.from_numpy(x.astype(np.float64)).reshape(g.T, g.C)
    u = F.layer_norm(xt, (g.C,), t["ln1_g"], t["ln1_b"], eps=1e-5)
    qkv = F.linear(u, t["w_qkv"].T, t["b_qkv"])
    q, k, v = qkv.split(g.C, dim=-1)
    hs = lambda a: a.reshape(g.T, g.heads, g.d).permute(1, 0, 2)
    coords = [(z, yy, xx) for z in range(g.Z) for yy in range(g.Y) for xx in range(g.X)]
    bias = torch.zeros(g.heads, g.T, g.T, dtype=torch.float64)
    for n, (z, yy, xx) in enumerate(coords):
        for m, (z2, y2, x2) in enumerate(coords):
            dz = _dense_offset(z, z2, g.Z, False)
            dy = _dense_offset(yy, y2, g.Y, False)
            dx = _dense_offset(xx, x2, g.X, True)
            bias[:, n, m] = t["rpb"][:, dz + g.Kz - 1, dy + g.Ky - 1, dx + g.Kx - 1]
    o = F.scaled_dot_product_attention(hs(q), hs(k), hs(v), attn_mask=bias)
    o = o.permute(1, 0, 2).reshape(g.T, g.C)
    x1 = xt + F.linear(o, t["w_o"].T, t["b_o"])
    w = F.layer_norm(x1, (g.C,), t["ln2_g"], t["ln2_b"], eps=1e-5)
    x2 = x1 + F.linear(F.gelu(F.linear(w, t["w_1"].T, t["b_1"])), t["w_2"].T, t["b_2"])
    assert np.abs(y.reshape(g.T, g.C) - x2.numpy()).max() < 1e-12


def test_block_roll_equivariance_and_sampled_outputs():
    g = tiny(Z=3, Y=5, X=8, Kz=3, Ky=3, Kx=5)
    p = _params(g, 4)
    x = S.latent_state(g, 1, 0)[0]
    y = O.block(x, p, g)
    for s in (1, 3):
        yr = O.block(np.roll(x, s, axis=2), p, g)
        assert np.abs(yr - np.roll(y, s, axis=2)).max() <= 1e-15 * np.abs(y).max()
    tok = np.array([0, 5, g.T - 1, 17, 40])
    assert np.abs(O.block_at(x, p, g, tok) - y.reshape(g.T, g.C)[tok]).max() < 1e-14


# --------------------------------------------------------------------------
# Greedy schedule and rollout (Sec. 2.1, latent rollout).
# --------------------------------------------------------------------------
def _golden_schedule():
    out = {}
    with open(os.path.join(GOLDEN, "schedule_table.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            lead, steps = line.split(":")
            out[int(lead)] = [int(s) for s in steps.split()]
    return out


def test_schedule_hand_table():
    table = _golden_schedule()
    assert len(table) >= 10
    for lead, steps in table.items():
        assert O.schedule(lead) == steps
    assert O.schedule(336) == [6] * 56
    assert O.schedule(341) == [6] * 56 + [1] * 5


def test_schedule_properties():
    for L in range(0, 400):
        s = O.schedule(L)
        assert sum(s) == L
        assert s.count(6) == L // 6 and s.count(1) == L % 6
        assert s == sorted(s, reverse=True)
    with pytest.raises(ValueError):
        O.schedule(-1)


def test_rollout_identity_and_composition():
    g = tiny(C=8, heads=1)
    p6 = [S.split_block_params(g, S.processor_params(g, 2, 1, proc=0, std=0.1), b) for b in range(2)]
    p1 = [S.split_block_params(g, S.processor_params(g, 2, 2, proc=1, std=0.1), b) for b in range(2)]
    x = S.latent_state(g, 1, 0)
    assert np.array_equal(O.rollout(x, p6, p1, g, 0), x.astype(np.float64))
    y = O.rollout(x, p6, p1, g, 7)
    manual = O.processor_step(O.processor_step(x, p6, g), p1, g)
    assert np.array_equal(y, manual)
    # a 1 h step differs from a 6 h step (the two processors are not mixed up)
    assert not np.array_equal(O.rollout(x, p6, p1, g, 1), O.rollout(x, p6, p1, g, 6))


def test_rel_l2():
    a = np.array([3.0, 4.0])
    assert O.rel_l2(a, a) == 0.0
    assert abs(O.rel_l2(np.array([3.0, 5.0]), a) - 0.2) < 1e-16


# --------------------------------------------------------------------------
# e4m3 codec used to check FP8 codes (OCP FP8 format definition).
# --------------------------------------------------------------------------
def test_e4m3_table_and_rounding():
    v = O.e4m3_values()
    assert v[0x7E] == 448.0 and v[0x08] == 2.0 ** -6 and v[0x01] == 2.0 ** -9
    assert v[0x38] == 1.0 and np.isnan(v[0x7F])
    fin = v[:127]
    assert np.all(np.diff(fin) > 0)
    # every finite value encodes to itself, with either sign
    codes = np.arange(127, dtype=np.uint8)
    assert np.array_equal(O.e4m3_encode(fin), codes)
    assert np.array_equal(O.e4m3_encode(-fin[1:]), codes[1:] | 0x80)
    # midpoints go to the even code; saturation at 448
    mids = (fin[1:] + fin[:-1]) / 2
    enc = O.e4m3_encode(mids)
    assert np.all(enc % 2 == 0)
    assert O.e4m3_encode(np.array([1000.0, -500.0])).tolist() == [0x7E, 0xFE]
    assert O.e4m3_encode(np.array([2.0 ** -10])).tolist() == [0]
    r = np.random.default_rng(0).standard_normal(10000) * 50
    back = O.e4m3_decode(O.e4m3_encode(r))
    assert np.all(np.abs(back - np.clip(r, -448, 448)) <= np.maximum(np.abs(r) * 2.0 ** -4, 2.0 ** -10) + 1e-12)


# ---------------------------------------------------------------------------
# Rotary position embedding (the paper's encoding; its 3-D layout is a
# reading, see the oracle).  Pinned by what rotary embeddings must satisfy.

def _tok(g, z, y, x):
    return (np.asarray(z) * g.Y + np.asarray(y)) * g.X + np.asarray(x)


def test_rope_identity_at_origin_and_norms():
    g = S.Grid(Z=4, Y=9, X=12, C=64, heads=2, Kz=3, Ky=3, Kx=3)
    r = np.random.default_rng(0)
    t = r.standard_normal((g.T, 2, 32))
    ang = O.rope_angles(g)
    out = O.apply_rope(t, ang)
    assert np.array_equal(out[0], t[0])                      # token (0, 0, 0): no rotation
    pair_norm = lambda a: a[..., 0::2] ** 2 + a[..., 1::2] ** 2
    assert np.allclose(pair_norm(out), pair_norm(t), rtol=1e-13, atol=0)


def test_rope_scores_depend_on_offsets_only():
    """R(p) q . R(p') k is unchanged when both positions move by the same
    offset: any lon shift (with wrap: integer frequencies), lat and level
    shifts that stay on the grid."""
    g = S.Grid(Z=6, Y=15, X=20, C=32, heads=1, Kz=3, Ky=3, Kx=3)
    r = np.random.default_rng(1)
    q = r.standard_normal((1, 1, 32))
    k = r.standard_normal((1, 1, 32))

    def score(tq, tk):
        aq = O.rope_angles(g, [tq])
        ak = O.rope_angles(g, [tk])
        return float(np.sum(O.apply_rope(q, aq) * O.apply_rope(k, ak)))

    for _ in range(40):
        zq, zk = r.integers(0, 3, 2)
        yq, yk = r.integers(0, 8, 2)
        xq, xk = r.integers(0, g.X, 2)
        dz, dy, dx = r.integers(0, 3), r.integers(0, 7), r.integers(-40, 40)
        s0 = score(_tok(g, zq, yq, xq), _tok(g, zk, yk, xk))
        s1 = score(_tok(g, zq + dz, yq + dy, (xq + dx) % g.X), _tok(g, zk + dz, yk + dy, (xk + dx) % g.X))
        assert abs(s0 - s1) < 1e-11 * (1 + abs(s0))
    # and it does depend on the offset
    assert abs(score(_tok(g, 0, 0, 0), _tok(g, 0, 0, 1)) - score(_tok(g, 0, 0, 0), _tok(g, 0, 0, 2))) > 1e-6


def test_block_rope_wiring_and_lon_roll():
    g = S.Grid(Z=3, Y=7, X=10, C=64, heads=2, Kz=3, Ky=3, Kx=5)
    p = S.split_block_params(g, S.processor_params(g, 1, seed=5), 0)
    x = S.latent_state(g, 1, seed=6)[0].astype(np.float64)
    # q = k = 0 (zero W_q, W_k and their biases): rotating them changes nothing
    pz = {k_: np.array(v, np.float64) for k_, v in p.items()}
    pz["w_qkv"][:, :2 * g.C] = 0.0
    pz["b_qkv"][:2 * g.C] = 0.0
    assert np.array_equal(O.block(x, pz, g, rope=True), O.block(x, pz, g, rope=False))
    # with rotary q and k the block still commutes with a lon roll
    y = O.block(x, p, g, rope=True)
    yr = O.block(np.roll(x, 3, axis=2), p, g, rope=True)
    assert np.abs(yr - np.roll(y, 3, axis=2)).max() < 1e-10
    # and differs from the block without rotation
    assert np.abs(y - O.block(x, p, g, rope=False)).max() > 1e-6


def test_e4m3_codec_matches_torch_float8():
    """Inside the finite range (|x| <= 448) the oracle's e4m3 round trip is
    torch's float8_e4m3fn conversion (an independent implementation of the
    OCP format with round to nearest even); outside it the oracle saturates
    where torch gives NaN."""
    import torch
    r = np.random.default_rng(0)
    x = np.concatenate([np.linspace(-448.0, 448.0, 200001), r.standard_normal(100000) * 10.0,
                        [0.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10, 1.0625, 1.0625 + 1e-6]]).astype(np.float32)
    x = x[np.abs(x) <= 448.0]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = O.e4m3_decode(O.e4m3_encode(x))
    assert np.array_equal(got, ref)
    assert O.e4m3_decode(O.e4m3_encode(np.float32([500.0, -1e6])))[0] == 448.0
