"""CPU check of the direct-to-LDS load mapping of the tile-aligned contraction kernel.

gemm_f64_dma_kernel fills a two-stage ring of 16-deep K-tiles with 16-byte global->LDS loads
(one per lane and instruction): wave w, instruction q covers row/chunk i = w * NQ + q of the tile
(NQA for A, NQB for B; the WIDE variant's B tile is 256 x 16).
A mapping that reads past the tile faults the GPU, so this test rebuilds the mapping from the
constants in the kernel's header, for every lane of every wave, and checks that:
  * every (row, 16-byte chunk) of the 128 x 16 operand tile is fetched exactly once and no fetch
    leaves the tile (so a global address never exceeds the tile's rows and columns);
  * every LDS slot of the stage is written exactly once and stays inside the stage;
  * the fragment reads of the MFMA loop find the element they expect (the XOR swizzle of
    K-contiguous rows written by the loads is the one the reads undo).
It also replays the host's stream-K schedule: no workgroup takes pieces of more than two tiles
and every partial slot index stays below the partial buffer's slot count.
"""
import os
import re

import pytest

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1602_07527_amd", "csrc")


def _src(name):
    with open(os.path.join(HDR, name)) as f:
        return f.read()


def _const(src, name):
    m = re.search(r"constexpr\s+(?:int|int64_t)\s+" + name + r"\s*=\s*([^;]+);", src)
    assert m, name
    return m.group(1).strip()


@pytest.fixture(scope="module", params=[False, True], ids=["tile128x128", "wide128x256"])
def k(request):
    """Constants of gemm_f64_dma_kernel; the WIDE variant has 128 x 256 output tiles (B tile
    256 x 16, A tile unchanged)."""
    s = _src("cg_gemm.hpp")
    BM, BN = int(_const(s, "GEMM_BM")), int(_const(s, "GEMM_BN"))
    BK, THREADS = int(_const(s, "DMA_BK")), int(_const(s, "DMA_THREADS"))
    assert "BN = WIDE ? 2 * GEMM_BN : GEMM_BN" in s, "tile width of the WIDE variant"
    if request.param:
        BN *= 2
    m = re.search(r"constexpr int WM = (\d+), WN = (\d+), NW = WM \* WN;", s)
    assert m, "wave arrangement of gemm_f64_dma_kernel"
    WM, WN = int(m.group(1)), int(m.group(2))
    NW = WM * WN
    assert NW * 64 == THREADS
    TILE_A, TILE_B = BM * BK, BN * BK
    NQA, NQB = TILE_A * 8 // 1024 // NW, TILE_B * 8 // 1024 // NW
    assert NQA * NW * 1024 == TILE_A * 8 and NQB * NW * 1024 == TILE_B * 8
    CH = BK // 2
    return dict(BM=BM, BN=BN, BK=BK, NW=NW, WM=WM, WN=WN, TILE_A=TILE_A, TILE_B=TILE_B, NQA=NQA, NQB=NQB,
                CH=CH, RPI=64 // CH, NH=BN // int(_const(s, "GEMM_BN")), wide=request.param)


def _kcontig_fetches(k, ld, nq):
    """(global row, global chunk, lds double index) of every lane for an operand stored
    contiguously along K (A not transposed, B transposed): offsets as in the kernel."""
    out = []
    for wave in range(k["NW"]):
        for q in range(nq):
            i = wave * nq + q
            for lane in range(64):
                r = i * k["RPI"] + lane // k["CH"]
                c = (lane % k["CH"]) ^ (r % k["CH"])
                off = r * ld * 8 + c * 16                 # bytes from the tile's base
                lds = i * k["RPI"] * k["BK"] + lane * 2   # doubles: the instruction's base + lane * 16 B
                assert off % (ld * 8) % 16 == 0
                out.append((off // (ld * 8), (off % (ld * 8)) // 16, lds))
    return out


def _mcontig_fetches(k, ld, width, nq, nh):
    """Same for an operand stored contiguously along M or N (A transposed, B not): instruction i
    takes K-row i // nh, 128-column piece i % nh."""
    out = []
    for wave in range(k["NW"]):
        for q in range(nq):
            i = wave * nq + q
            for lane in range(64):
                off = (i // nh) * ld * 8 + (i % nh) * 1024 + lane * 16
                lds = (i // nh) * width + (i % nh) * 128 + lane * 2
                out.append((off // (ld * 8), (off % (ld * 8)) // 16, lds))
    return out


@pytest.mark.parametrize("ld", [256, 258, 16384, 20002])
@pytest.mark.parametrize("operand", ["A", "B"])
def test_k_contiguous_tile_covered_once(k, ld, operand):
    rows_n = k["BM"] if operand == "A" else k["BN"]
    tile = k["TILE_A"] if operand == "A" else k["TILE_B"]
    f = _kcontig_fetches(k, ld, k["NQA"] if operand == "A" else k["NQB"])
    rows = {(r, c) for r, c, _ in f}
    assert len(f) == len(rows) == rows_n * k["CH"]
    assert all(0 <= r < rows_n and 0 <= c < k["CH"] for r, c, _ in f)
    slots = [s for _, _, s in f]
    assert len(set(slots)) == len(slots)
    assert all(0 <= s and s + 1 < tile for s in slots)
    # the fragment read of row m, chunk g is as[m * BK + ((g ^ (m % CH)) << 1)]
    where = {(r, c): s for r, c, s in f}
    for m in range(rows_n):
        for g in range(k["CH"]):
            assert where[(m, g)] == m * k["BK"] + ((g ^ (m % k["CH"])) << 1)


@pytest.mark.parametrize("ld", [256, 258, 16384])
@pytest.mark.parametrize("operand", ["A", "B"])
def test_m_contiguous_tile_covered_once(k, ld, operand):
    width = k["BM"] if operand == "A" else k["BN"]
    tile = k["TILE_A"] if operand == "A" else k["TILE_B"]
    nq, nh = (k["NQA"], 1) if operand == "A" else (k["NQB"], k["NH"])
    assert width * k["BK"] == tile
    f = _mcontig_fetches(k, ld, width, nq, nh)
    got = {(r, c) for r, c, _ in f}
    assert len(f) == len(got) == k["BK"] * width // 2
    assert all(0 <= r < k["BK"] and 0 <= c < width // 2 for r, c, _ in f)
    slots = [s for _, _, s in f]
    assert len(set(slots)) == len(slots) and max(slots) + 1 < tile
    # element (kk, m) lands at as[kk * width + m], where the fragment reads look for it
    for r, c, s in f:
        assert s == r * width + 2 * c


def test_fragment_reads_stay_in_the_stage(k):
    """MFMA fragment reads of both operands: index < the operand's tile for every lane, slot, t and u."""
    BM, BN, BK, CH, WM, WN = k["BM"], k["BN"], k["BK"], k["CH"], k["WM"], k["WN"]
    TMW, TNW = BM // WM // 16, BN // WN // 16
    for wave in range(k["NW"]):
        wm, wn = wave // WN, wave % WN
        for lane in range(64):
            fk, fi = lane >> 4, lane & 15
            for u in range(BK // 8):
                g = 4 * u + fk
                k0 = 2 * g
                for t in range(TMW):
                    m = wm * (BM // WM) + t * 16 + fi
                    assert m * BK + ((g ^ (m % CH)) << 1) + 1 < k["TILE_A"]
                    assert (k0 + 1) * BM + m < k["TILE_A"]
                for t in range(TNW):
                    n = wn * (BN // WN) + t * 16 + fi
                    assert n * BK + ((g ^ (n % CH)) << 1) + 1 < k["TILE_B"]
                    assert (k0 + 1) * BN + n < k["TILE_B"]


def test_streamk_schedule_bounds():
    """The host's stream-K choice (workgroup count, at most two tile pieces per workgroup, partial
    slot w + t below the slot count) over the panel shapes of the sweeps."""
    s = _src("cholgrad.hip")
    SK_WGS, SK_SHORT = int(_const(s, "SK_WGS")), int(_const(s, "SK_WGS_SHORT"))
    SHORT_KT = int(_const(s, "SK_SHORT_KTILES"))
    slots = 2 * int(_const(s, "TARGET_WGS"))
    assert _const(s, "PART_SLOTS") == "2 * TARGET_WGS"
    BK = 16
    target = int(_const(s, "TARGET_WGS"))
    for tiles in (2, 3, 7, 31, 64, 127):
        for Kt in (BK * x for x in (1, 2, 8, 64, 255, 1016, 2040)):
            for min_kchunk in (32, 64, 256):
                for alone in (False, True):      # single-stream sweeps take all TARGET_WGS slots
                    for wide in (False, True):   # 128 x 256 tiles: half the workgroups and slots
                        units = tiles * (Kt // BK)
                        skw = target if alone else (SK_SHORT if units < SHORT_KT * SK_WGS else SK_WGS)
                        if wide:
                            skw //= 2
                        wslots = slots // 2 if wide else slots
                        skw = min(skw, units * BK // max(min_kchunk, BK))
                        skw = min(skw, wslots - tiles + 1)
                        if skw <= tiles:
                            continue
                        T, kt = units, Kt // BK
                        assert T // skw <= kt
                        for w in range(skw):
                            su, su1 = w * T // skw, (w + 1) * T // skw
                            t_first, t_last = su // kt, (su1 - 1) // kt if su1 > su else su // kt
                            assert t_last - t_first <= 1
                            assert w + t_last < wslots
