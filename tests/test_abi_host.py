"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function include/wm.h declares, and its
host-only logic (the greedy schedule, argument validation) must match the
oracle bit for bit.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(wm_[a-z0-9_]+)\s*\(",
                             text, flags=re.M):
            names.append(m.group(1))
    return names


@pytest.fixture(scope="module")
def wm():
    import paper_2503_22235_amd as wm
    if not os.path.exists(wm.LIB_PATH):
        from paper_2503_22235_amd import build
        build.build()
    wm.lib()
    return wm


def test_header_symbols_exported(wm):
    names = _declared_functions()
    assert len(names) >= 15
    L = ctypes.CDLL(wm.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert "gfx950" in wm.wm_version()


def test_schedule_matches_oracle_bit_exact(wm):
    from oracle import wm_oracle as O
    for lead in list(range(0, 400)) + [341, 1000, 5000]:
        assert wm.wm_schedule(lead) == O.schedule(lead)


def test_schedule_errors(wm):
    L = wm.lib()
    assert L.wm_schedule(-1, None, 0) == -1
    assert b"negative" in L.wm_last_error()
    buf = (ctypes.c_int * 2)()
    assert L.wm_schedule(13, buf, 2) == -1          # needs 3 entries
    assert L.wm_schedule(12, buf, 2) == 2 and list(buf) == [6, 6]


def test_argument_validation_without_gpu(wm):
    """Invalid windows, shapes and precisions are rejected before any GPU work."""
    L = wm.lib()
    bad = [
        wm.wm_grid(8, 90, 180, 512, 16, 4, 7, 7, 4),     # even window
        wm.wm_grid(4, 90, 180, 512, 16, 5, 7, 7, 4),     # window larger than axis
        wm.wm_grid(8, 90, 180, 500, 16, 5, 7, 7, 4),     # head dim not 32
        wm.wm_grid(8, 90, 180, 512, 16, 5, 7, 7, 9),     # bad periodic mask
    ]
    for g in bad:
        assert L.wm_nat_indices(ctypes.byref(g), 1, None) == wm_status("WM_EINVAL")
    assert L.wm_layernorm(4, 100, 1, 1, 1, 1e-5, 1, 1, None) == wm_status("WM_EINVAL")
    assert L.wm_linear(4, 100, 64, 1, 1, 1, 1, 0, 1, None) == wm_status("WM_EINVAL")
    assert L.wm_linear(4, 128, 64, 1, 1, 1, 1, 5, 1, None) == wm_status("WM_EINVAL")
    assert L.wm_processor_block(None, None, 0, 1, None, None) == wm_status("WM_EINVAL")
    assert L.wm_rollout(None, None, None, 1, None, 6, None) == wm_status("WM_EINVAL")


def wm_status(name):
    text = open(os.path.join(ROOT, "include", "wm.h")).read()
    m = re.search(name + r"\s*=\s*(-?\d+)", text)
    return int(m.group(1))


def test_fp8_processor_needs_e4m3_attention_without_gpu(wm):
    """An FP8 processor runs QK and PV on e4m3 codes; on a grid or window the
    e4m3 attention does not cover it is refused (WM_EINVAL) before any
    device work -- it never falls back to bf16 attention.  The same grids in
    BF16 are accepted up to the context check."""
    import numpy as np
    L = wm.lib()
    einval = wm_status("WM_EINVAL")
    params = np.zeros(16, np.float32)       # never read: the call fails first
    out = ctypes.c_void_p()
    uncovered = [
        wm.wm_grid(8, 90, 180, 512, 16, 3, 5, 7, 4),   # window without an e4m3 kernel
        wm.wm_grid(8, 90, 180, 512, 16, 5, 7, 7, 0),   # lon not periodic
        wm.wm_grid(8, 90, 180, 512, 16, 5, 7, 7, 6),   # lat periodic too
        wm.wm_grid(8, 90, 13, 512, 16, 5, 7, 7, 4),    # lon shorter than the halo (8 + Kx - 1)
    ]
    for g in uncovered:
        assert L.wm_processor_create(None, ctypes.byref(g), 1, 4, 2, params.ctypes.data,
                                     ctypes.byref(out)) == einval
        assert b"e4m3" in L.wm_last_error(), L.wm_last_error()
        # BF16 gets past the grid checks and stops at the missing context
        assert L.wm_processor_create(None, ctypes.byref(g), 1, 4, 1, params.ctypes.data,
                                     ctypes.byref(out)) == einval
        assert b"ctx" in L.wm_last_error()
    ok = wm.wm_grid(8, 90, 180, 512, 16, 5, 7, 7, 4)
    assert L.wm_processor_create(None, ctypes.byref(ok), 1, 4, 2, params.ctypes.data,
                                 ctypes.byref(out)) == einval
    assert b"ctx" in L.wm_last_error()


def test_nat_forward_noalloc_limits_without_gpu(wm):
    """The no-allocation attention entry point checks its arguments like
    wm_nat_forward and refuses work whose scratch exceeds its fixed array,
    before touching a device."""
    L = wm.lib()
    einval = wm_status("WM_EINVAL")
    assert wm.WM_NAT_NOALLOC_SCRATCH_BYTES == int(eval(re.search(
        r"#define WM_NAT_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)",
        open(os.path.join(ROOT, "include", "wm.h")).read()).expand(r"\1 << \2")))
    g = wm.wm_grid(8, 90, 180, 1024, 32, 5, 7, 7, 4)
    # FP8: B * heads * 8 KiB + 128 KiB of scratch; 16 states x 32 heads need 4.1 MiB
    assert L.wm_nat_forward_noalloc(ctypes.byref(g), 16, 2, 1, 1, 1, 1, 1, None) == einval
    assert b"exceeds" in L.wm_last_error(), L.wm_last_error()
    # the same checks as wm_nat_forward come first
    bad = wm.wm_grid(8, 90, 180, 512, 16, 4, 7, 7, 4)
    assert L.wm_nat_forward_noalloc(ctypes.byref(bad), 1, 1, 1, 1, 1, 1, 1, None) == einval
    assert L.wm_nat_forward_noalloc(ctypes.byref(g), 1, 1, None, 1, 1, 1, 1, None) == einval
    assert b"NULL" in L.wm_last_error()
    # nothing to do: no device needed
    assert L.wm_nat_forward_noalloc(ctypes.byref(g), 0, 1, None, None, None, None, None, None) == 0


def test_serve_validation_without_gpu(wm):
    L = wm.lib()
    einval = wm_status("WM_EINVAL")
    out = ctypes.c_void_p()
    cfg = wm.wm_serve_cfg(4, 1, 0, 0)
    assert L.wm_serve_create(None, None, None, ctypes.byref(cfg), ctypes.byref(out)) == einval
    rid = ctypes.c_uint64()
    assert L.wm_serve_submit(None, None, 6, ctypes.byref(rid)) == einval
    assert L.wm_serve_poll(None, 1, None, None) == einval


def test_missing_library_raises_no_fallback(wm, monkeypatch, tmp_path):
    """With the shared library absent every call raises: there is no CPU path."""
    monkeypatch.setattr(wm, "_LIB", None)
    monkeypatch.setattr(wm, "LIB_PATH", str(tmp_path / "libwm.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        wm.lib()
    with pytest.raises(ImportError):
        wm.wm_schedule(6)


def test_traffic_hash_covers_kernel_sources(tmp_path):
    """The counter file goes stale on any kernel or launch source change, not on the server's."""
    import shutil
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src = os.path.join(ROOT, "paper_2503_22235_amd", "csrc")
    d = tmp_path / "csrc"
    shutil.copytree(src, d)
    h0 = bench.kernel_source_hash(str(d))
    assert h0 == bench.kernel_source_hash()
    with open(d / "serve.cpp", "a") as f:
        f.write("\n// host-only edit\n")
    assert bench.kernel_source_hash(str(d)) == h0
    with open(d / "k_nat_tile.hip", "a") as f:
        f.write("\n// kernel edit\n")
    assert bench.kernel_source_hash(str(d)) != h0


def test_counter_attribution_per_block_kernel():
    """rocprofv3 counter rows are attributed to the block's kernels by launch
    order; a bias-table preparation joins the attention launch after it, and
    tables prepared at processor creation (not followed by an attention
    launch) are left out."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    ns = "wm::(anonymous namespace)::"
    block = [(ns + "layernorm_kernel", 1.0), (ns + "gemm_lds_kernel", 2.0),
             (ns + "nat_bias_prep", 0.5), (ns + "nat_tile_kernel", 3.0), (ns + "gemm_lds_kernel", 4.0),
             (ns + "layernorm_kernel", 5.0), (ns + "gemm_lds_kernel", 6.0), (ns + "gemm_lds_kernel", 7.0)]
    cached = [b for b in block if "bias_prep" not in b[0]]
    rows = [(ns + "nat_bias_prep", 100.0)] * 3 + [("at::neg_kernel", 9.0)] + block + cached
    rows = [(i, n, v) for i, (n, v) in enumerate(rows)]
    import wm_synth as S
    got = bench._per_kind(rows, bench.kind_order(S.CFG1))
    assert got == {"ln1": 1.0, "qkv": 2.0, "nat": 3.25, "proj": 4.0, "ln2": 5.0, "mlp1": 6.0, "mlp2": 7.0}
    # C = 512: LN2 runs inside the out-projection, six launches per block
    fused = [b for b in block if b[1] != 5.0]
    rows = [(i, n, v) for i, (n, v) in enumerate(fused + [b for b in fused if "bias_prep" not in b[0]])]
    assert bench.kind_order(S.CFG2) == ("ln1", "qkv", "nat", "proj", "mlp1", "mlp2")
    got = bench._per_kind(rows, bench.kind_order(S.CFG2))
    assert got == {"ln1": 1.0, "qkv": 2.0, "nat": 3.25, "proj": 4.0, "mlp1": 6.0, "mlp2": 7.0}
    with pytest.raises(SystemExit):     # seven launches per block are not the fused order
        bench._per_kind([(i, n, v) for i, (n, v) in enumerate(block)], bench.kind_order(S.CFG2))


def test_block_kernel_work_with_fused_ln2():
    """At C = 512 LN2 runs in the out-projection's epilogue: the algorithmic
    work of "proj" adds LN2's FLOPs and its bf16 output (the rows it reads are
    the ones the projection just wrote), and there is no "ln2" launch.  Other
    widths keep the separate LayerNorm with the same figures as LN1."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    import wm_synth as S
    g = S.CFG2
    T, C = g.Z * g.Y * g.X, g.C
    w = bench.block_kernel_work(g)
    assert "ln2" not in w and set(w) == set(bench.kind_order(g))
    assert w["proj"] == (2.0 * T * C * C + 8.0 * T * C, T * C * 2 + C * C * 2 + 2 * T * C * 4 + T * C * 2)
    g1 = S.CFG1
    T1, C1 = g1.Z * g1.Y * g1.X, g1.C
    w1 = bench.block_kernel_work(g1)
    assert w1["ln2"] == w1["ln1"] == (8.0 * T1 * C1, T1 * C1 * 6)
    assert w1["proj"] == (2.0 * T1 * C1 * C1, T1 * C1 * 2 + C1 * C1 * 2 + 2 * T1 * C1 * 4)
