"""Structure of the gfx950 code the compiler emits for our own kernels.

Compiles the library's HIP sources to AMDGPU assembly (this repository's code
only) and checks that the two forms differ where they should:
  * the divergent bitonic compare-exchange keeps a load pair, a compare and a
    store pair inside each side of the direction branch (Figure 1 as written),
  * the melded one has a single load pair / store pair and no side blocks,
  * the divergent region runs one gather loop per side, the melded region
    keeps each side's gathers in its own block and the fma chain outside, and
    the in-place melded region has no side blocks at all.
It also checks that the merge tails and gathered passes issue their tile's
global loads inside a raised wave-priority window that closes before any
LDS work.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2107_05681_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def _asm(src, tmp_path, defines=()):
    out = tmp_path / (os.path.basename(src) + ".s")
    subprocess.check_call(
        [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", "--offload-device-only", "-S",
         *[f"-D{d}" for d in defines], os.path.join(CSRC, src), "-o", str(out)],
        stderr=subprocess.DEVNULL)
    return out.read_text()


# The local tile sorts are checked at the two tile sizes the tests read
# (2^11 and 2^13); the same templates as the library's build, fewer of them.
LOCAL_SIZES = ("MELD_REGS_SIZES(X)=X(11) X(13)",)


def _kernel(asm, pattern):
    names = re.findall(r"^(_Z\S*):", asm, flags=re.M)
    match = [n for n in names if re.search(pattern, n)]
    assert match, f"no kernel matches {pattern}"
    start = asm.index(match[0] + ":")
    end = asm.index("s_endpgm", start)
    return asm[start:end]


def _blocks_after(body, marker):
    """Instruction text from each occurrence of an asm marker to the next marker."""
    parts = re.split(r";;#ASMSTART\s*\n\s*; side ", body)
    return [p for p in parts[1:] if p.startswith(marker)]


@pytest.fixture(scope="module")
def bitonic_asm(tmp_path_factory):
    return _asm("bitonic.hip", tmp_path_factory.mktemp("isa"))


@pytest.fixture(scope="module")
def local_lds_asm(tmp_path_factory):
    return _asm("bitonic_local_lds.hip", tmp_path_factory.mktemp("isa"), LOCAL_SIZES)


@pytest.fixture(scope="module")
def local_xch_asm(tmp_path_factory):
    return _asm("bitonic_local_xch.hip", tmp_path_factory.mktemp("isa"), LOCAL_SIZES)


@pytest.fixture(scope="module")
def region_asm(tmp_path_factory):
    return _asm("region.hip", tmp_path_factory.mktemp("isa"))


@pytest.mark.parametrize("pairs", [False, True])
def test_bitonic_divergent_sides_hold_lds_ops(bitonic_asm, pairs):
    p = "b1" if pairs else "b0"
    body = _kernel(bitonic_asm, rf"bitonic_tile_kernelIL{p}ELb0ELb0ELi512ELi1E")
    width = "b64" if pairs else "b32"
    for side in ("ascending\n", "descending\n"):
        blocks = _blocks_after(body, side)
        assert blocks, side
        text = blocks[0]
        assert text.count(f"ds_read_{width}") == 2, side
        assert text.count(f"ds_write_{width}") == 2, side
        assert re.search(r"v_cmp_[lg]t_u(32|64)", text), side
    assert "s_and_saveexec_b64" in body


@pytest.mark.parametrize("pairs", [False, True])
def test_bitonic_melded_has_one_load_store_pair(bitonic_asm, pairs):
    p = "b1" if pairs else "b0"
    body = _kernel(bitonic_asm, rf"bitonic_tile_kernelIL{p}ELb1ELb1ELi512ELi1E")
    width = "b64" if pairs else "b32"
    assert "; side" not in body
    # the comparator loop: one load pair and one (conditional) store pair
    loop = body[body.index(f"ds_read_{width}", body.index("s_barrier")):]
    assert loop.count(f"ds_write_{width}") >= 2
    # select(up, b < a, b > a) as lane-mask logic: an order compare whose mask
    # the direction flips (a scalar xor), and the tie test
    assert re.search(r"v_cmp_(lt|gt|le|ge)_u(32|64)", body)
    assert re.search(r"v_cmp_ne_u(32|64)", body)
    assert re.search(r"s_xn?or_b64", body)


def test_region_divergent_has_a_loop_per_side(region_asm):
    body = _kernel(region_asm, r"region_divergent_kernel")
    for side in ("true\n", "false\n"):
        blocks = _blocks_after(body, side)
        assert blocks and "global_load_dword" in blocks[0] and "v_fma" in blocks[0], side


def test_region_melded_gathers_per_side_fma_once(region_asm):
    body = _kernel(region_asm, r"region_melded_kernel")
    assert _blocks_after(body, "gathers true") and _blocks_after(body, "gathers false")
    assert "v_cndmask_b32" in body  # the selected multiplier


def test_region_melded_inplace_has_no_side_blocks(region_asm):
    body = _kernel(region_asm, r"region_melded_inplace_kernel")
    assert "; side" not in body
    assert "v_cndmask_b32" in body and "global_load_dword" in body


@pytest.mark.parametrize("pairs", [False, True])
def test_register_phases_divergent_vs_melded(local_lds_asm, pairs):
    # Phases k >= 128 of the tile sort run in registers: the divergent form
    # keeps Figure 1's two sides (one per direction), the melded one has none.
    p = "b1" if pairs else "b0"
    div = _kernel(local_lds_asm, rf"bitonic_sort_regs_kernelIL{p}ELi13ELb0ELb0ELb0E")
    mel = _kernel(local_lds_asm, rf"bitonic_sort_regs_kernelIL{p}ELi13ELb1ELb1ELb0E")
    width = "u64" if pairs else "u32"
    for side in ("ascending regs\n", "descending regs\n"):
        blocks = _blocks_after(div, side)
        assert blocks, side
        assert re.search(rf"v_cmp_[lg]t_{width}", blocks[0]), side
    assert "; side" not in mel
    # one order compare per comparator, its mask flipped by the direction
    # (a scalar xor), then the selects
    assert re.search(rf"v_cmp_(lt|gt|le|ge)_{width}", mel) and "v_cndmask_b32" in mel
    assert re.search(r"s_xn?or_b64", mel)


@pytest.fixture(scope="module")
def variants_asm(tmp_path_factory):
    return _asm("region_variants.hip", tmp_path_factory.mktemp("isa"))


def test_region3_divergent_runs_a_loop_per_way(variants_asm):
    body = _kernel(variants_asm, r"region3_divergent_kernel")
    for way in ("way 0\n", "way 1\n", "way 2\n"):
        blocks = _blocks_after(body, way)
        assert blocks and "global_load_dword" in blocks[0] and "v_fma" in blocks[0], way


def test_region3_melded_gathers_per_way_fma_once(variants_asm):
    body = _kernel(variants_asm, r"region3_melded_kernel")
    for way in ("gathers way 0", "gathers way 1", "gathers way 2"):
        assert _blocks_after(body, way), way
    assert "v_cndmask_b32" in body  # the selected multiplier


def test_region3_melded_inplace_has_no_way_blocks(variants_asm):
    body = _kernel(variants_asm, r"region3_melded_inplace_kernel")
    assert "; side" not in body


@pytest.fixture(scope="module")
def oddeven_asm(tmp_path_factory):
    return _asm("oddeven.hip", tmp_path_factory.mktemp("isa"))


def test_oddeven_divergent_sides_each_load(oddeven_asm):
    body = _kernel(oddeven_asm, r"oddeven_bucket_kernelILi8ELi1024ELb0E")
    for side in ("lower\n", "upper\n"):
        blocks = _blocks_after(body, side)
        # each side issues its own LDS loads (single or paired)
        assert blocks and all(re.search(r"ds_read\w*_b32", blk) for blk in blocks), side


def test_oddeven_melded_has_no_sides(oddeven_asm):
    body = _kernel(oddeven_asm, r"oddeven_bucket_kernelILi8ELi1024ELb1E")
    assert "; side" not in body and re.search(r"ds_read\w*_b32", body)
    assert "v_cndmask_b32" in body


@pytest.fixture(scope="module")
def mergesort_asm(tmp_path_factory):
    return _asm("mergesort.hip", tmp_path_factory.mktemp("isa"))


def test_merge_step_divergent_sides_each_load(mergesort_asm):
    body = _kernel(mergesort_asm, r"merge_pass_kernelILb0E")
    for side in ("take a\n", "take b\n"):
        blocks = _blocks_after(body, side)
        assert blocks and "ds_read_b32" in blocks[0], side


def test_merge_step_melded_has_no_sides(mergesort_asm):
    body = _kernel(mergesort_asm, r"merge_pass_kernelILb1E")
    assert "; side" not in body and "v_cndmask_b32" in body


def _kernel_all(asm, pattern):
    """A kernel's whole text, with the blocks the compiler placed after its
    first s_endpgm."""
    names = re.findall(r"^(_Z\S*):", asm, flags=re.M)
    match = [n for n in names if re.search(pattern, n)]
    assert match, f"no kernel matches {pattern}"
    start = asm.index(match[0] + ":")
    return asm[start:asm.index(".Lfunc_end", start)]


def _lane_sides(body):
    """(direction, text) of every side block of the divergent lane steps: from
    its mark to the end of its basic block."""
    return re.findall(r"; side ((?:a|de)scending) lanes\n(.*?)(?=^\.LBB|^; %bb\.)", body,
                      re.S | re.M)


# Tile sort of 2^11 with lane exchanges, each phase unrolled: three lane steps
# in phases k <= 64 (element bits 4, 5, 4), and in the later phases the steps
# of each phase's last layout W0 on element bits 6 .. 4 that remain: bits 6, 5,
# 4 for phases 2^7 and 2^11, bit 4 for 2^9, bits 5, 4 for 2^10. Steps on bits
# 4 and 5 (lane bits 0, 1) take one DPP move per 32-bit value, those on bit 6
# (lane t ^ 4) two.
LANE_STEPS_LOW_BITS = 3 + 2 + 1 + 2 + 2    # on lane bits 0 and 1
LANE_STEPS_BIT2 = 2                           # on lane bit 2


@pytest.mark.parametrize("pairs", [False, True])
def test_lane_exchanges_sit_outside_the_divergent_sides(local_xch_asm, pairs):
    # The divergent form moves each partner value with DPP moves of its own,
    # before the branch; its sides hold only compares and selects.
    p = "b1" if pairs else "b0"
    div = _kernel_all(local_xch_asm, rf"bitonic_sort_regs_kernelIL{p}ELi11ELb0ELb0ELb1E")
    sides = _lane_sides(div)
    steps = LANE_STEPS_LOW_BITS + LANE_STEPS_BIT2
    assert sum(1 for d, _ in sides if d == "ascending") >= steps
    assert sum(1 for d, _ in sides if d == "descending") >= steps
    for _, text in sides:
        assert "_dpp" not in text and "ds_" not in text and "permlane" not in text
        # each side its own compare (keys: min and max) and select
        assert (re.search(r"v_cmp_\w+_u64", text) if pairs else
                ("v_min_u32" in text and "v_max_u32" in text)), text[:400]
        assert "v_cndmask_b32" in text
    halves = 2 if pairs else 1
    assert div.count("v_mov_b32_dpp") == (LANE_STEPS_LOW_BITS + 2 * LANE_STEPS_BIT2) * 16 * halves
    assert "quad_perm:[1,0,3,2]" in div and "quad_perm:[2,3,0,1]" in div
    assert "row_half_mirror" in div and "quad_perm:[3,2,1,0]" in div


@pytest.mark.parametrize("pairs", [False, True])
def test_lane_exchanges_melded_compare_select_on_the_full_wave(local_xch_asm, pairs):
    p = "b1" if pairs else "b0"
    mel = _kernel_all(local_xch_asm, rf"bitonic_sort_regs_kernelIL{p}ELi11ELb1ELb1ELb1E")
    assert "; side" not in mel
    if pairs:
        # both halves moved, one 64-bit compare, a select per half
        assert mel.count("v_mov_b32_dpp") == (LANE_STEPS_LOW_BITS + 2 * LANE_STEPS_BIT2) * 16 * 2
        assert re.search(r"v_cmp_(lt|gt)_u64", mel)
    else:
        # on lane bits 0 and 1 the move folds into the min and max that use it
        assert mel.count("v_min_u32_dpp") == LANE_STEPS_LOW_BITS * 16
        assert mel.count("v_max_u32_dpp") == LANE_STEPS_LOW_BITS * 16
        assert mel.count("v_mov_b32_dpp") == 2 * LANE_STEPS_BIT2 * 16


@pytest.fixture(scope="module")
def segsort_asm(tmp_path_factory):
    return _asm("segsort.hip", tmp_path_factory.mktemp("isa"))


def test_segmented_lane_exchanges_outside_the_sides(segsort_asm):
    div = _kernel_all(segsort_asm, r"seg_sort_kernelILb0ELb0ELb1E")
    sides = _lane_sides(div)
    assert sides
    for _, text in sides:
        assert "_dpp" not in text and "ds_" not in text
    mel = _kernel_all(segsort_asm, r"seg_sort_kernelILb1ELb1ELb1E")
    assert not _lane_sides(mel)
    assert "v_min_u32_dpp" in mel and "v_max_u32_dpp" in mel


@pytest.mark.parametrize("kernel", [
    r"bitonic_pass_regs_kernelILb1ELi13ELi13ELi13E",  # merge tail, pairs
    r"bitonic_pass_regs_kernelILb0ELi14ELi14ELi14E",  # merge tail, keys
    r"bitonic_pass_regs_kernelILb1ELi13ELi6ELi7E",    # gathered pass of 6 pair steps
])
def test_pass_tile_loads_at_raised_priority(bitonic_asm, kernel):
    # The streaming passes issue every global load of their tile at wave
    # priority 2 and drop back to 0 before any LDS work.
    body = _kernel(bitonic_asm, kernel)
    up = body.index("s_setprio 2")
    down = body.index("s_setprio 0")
    loads = [m.start() for m in re.finditer(r"\bglobal_load", body)]
    lds = [m.start() for m in re.finditer(r"\bds_(read|write|load|store)", body)]
    assert loads and lds
    assert all(up < p < down for p in loads)
    assert min(lds) > down
