"""The offline meld planner (melding profitability, instruction alignment and
region discovery of the Detailed Design section) on the CPU."""
import itertools
import os
import random
import shutil

import pytest

from paper_2107_05681_amd import planner as P


def test_mp_b_identical_profiles_is_half():
    # The paper's example: two blocks with the same opcode histogram score 0.5.
    b = ["load.global", "fadd", "fmul", "fadd", "store.global", "icmp", "br"]
    assert P.mp_b(b, list(reversed(b))) == pytest.approx(0.5)


def test_mp_b_disjoint_and_hand_value():
    assert P.mp_b(["fadd", "fmul"], ["load.lds", "store.lds"]) == 0.0
    # fadd shared once (4), load.global shared once (500); latencies 508 + 1004
    b1 = ["fadd", "fadd", "load.global"]
    b2 = ["fadd", "load.global", "load.global"]
    assert P.mp_b(b1, b2) == pytest.approx(504 / 1512)
    # phi nodes and side marks neither count nor cost
    assert P.mp_b(b1 + ["phi", "call.mark"], b2) == pytest.approx(504 / 1512)


def _brute_local(a, b, score, gap):
    """Best local alignment score by enumerating every increasing matching."""
    best = 0.0
    cells = [(i, j) for i in range(len(a)) for j in range(len(b))
             if score(a[i], b[j]) is not None]
    for r in range(1, min(len(a), len(b)) + 1):
        for combo in itertools.combinations(cells, r):
            ok = all(combo[k][0] < combo[k + 1][0] and combo[k][1] < combo[k + 1][1]
                     for k in range(r - 1))
            if not ok:
                continue
            val = sum(score(a[i], b[j]) for i, j in combo)
            val -= gap * sum((combo[k + 1][0] - combo[k][0] - 1) +
                             (combo[k + 1][1] - combo[k][1] - 1) for k in range(r - 1))
            best = max(best, val)
    return best


@pytest.mark.parametrize("seed", range(40))
def test_smith_waterman_matches_brute_force(seed):
    rng = random.Random(seed)
    alphabet = ["fadd", "load.global", "icmp", "select"]
    a = [rng.choice(alphabet) for _ in range(rng.randint(1, 5))]
    b = [rng.choice(alphabet) for _ in range(rng.randint(1, 5))]
    gap = rng.choice([0.0, 1.0, 4.0, 300.0])
    best, pairs = P.smith_waterman(a, b, P._instr_score, gap)
    assert best == pytest.approx(_brute_local(a, b, P._instr_score, gap))
    # the traced alignment is increasing, compatible and reaches the score
    assert all(a[i] == b[j] for i, j in pairs)
    assert all(p[0] < q[0] and p[1] < q[1] for p, q in zip(pairs, pairs[1:]))
    if pairs:
        val = sum(P.latency(a[i]) for i, _ in pairs)
        val -= gap * sum((q[0] - p[0] - 1) + (q[1] - p[1] - 1) for p, q in zip(pairs, pairs[1:]))
        assert val == pytest.approx(best)
    else:
        assert best == 0.0


def _reachable(succ, entry, removed):
    seen, stack = set(), [entry]
    while stack:
        u = stack.pop()
        if u in seen or u == removed:
            continue
        seen.add(u)
        stack.extend(succ.get(u, ()))
    return seen


@pytest.mark.parametrize("seed", range(30))
def test_dominators_match_definition(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 9)
    nodes = [str(k) for k in range(n)]
    succ = {u: sorted({rng.choice(nodes) for _ in range(rng.randint(0, 3))}) for u in nodes}
    idom = P.dominators(succ, "0")
    live = _reachable(succ, "0", None)
    assert set(idom) == live
    for b in live - {"0"}:
        # strict dominators of b: removing d cuts b off the entry
        doms = {d for d in live if d != b and b not in _reachable(succ, "0", d)}
        # the dominator-tree chain above b is exactly that set
        assert idom[b] in doms
        assert set(P._ancestors(idom, b)) - {b} == doms


_IR = """
define amdgpu_kernel void @k(ptr addrspace(1) %0, i1 %1) {
  %3 = load float, ptr addrspace(1) %0, align 4
  br i1 %1, label %4, label %7

4:                                                ; preds = %2
  tail call void asm sideeffect "; side true", "~{memory}"()
  %5 = fmul float %3, 2.000000e+00
  %6 = fadd float %5, 1.000000e+00
  store float %6, ptr addrspace(1) %0, align 4
  br label %10

7:                                                ; preds = %2
  tail call void asm sideeffect "; side false", "~{memory}"()
  FALSE_BODY
  br label %10

10:                                               ; preds = %7, %4
  ret void
}
"""


def test_region_from_handwritten_ir():
    same = ("%8 = fmul float %3, 3.000000e+00\n  %9 = fadd float %8, 2.000000e+00\n"
            "  store float %9, ptr addrspace(1) %0, align 4")
    fns = P.parse_ir(_IR.replace("FALSE_BODY", same))
    fn = fns["k"]
    assert fn.order == ["2", "4", "7", "10"]
    (r,) = P.analyse_function(fn, (("true", "false"),))
    assert r.instances == 1 and r.blocks == (1, 1)
    assert r.mp_s == pytest.approx(0.5)
    # everything aligns: saved is half of both sides, no gaps
    assert r.saved_fraction == pytest.approx(0.5) and r.gaps == 0
    assert r.predicted_speedup == pytest.approx(2.0)

    # the false side shares fadd and br with the true side, but in an order
    # that leaves an unaligned instruction between them on both sides
    lds = ("%8 = fadd float %3, 2.000000e+00\n"
           "  %9 = load float, ptr addrspace(3) null, align 4")
    (r2,) = P.analyse_function(P.parse_ir(_IR.replace("FALSE_BODY", lds))["k"],
                               (("true", "false"),))
    lat_t = P.latency("fmul") + P.latency("fadd") + P.latency("store.global") + P.latency("br")
    lat_f = P.latency("load.lds") + P.latency("fadd") + P.latency("br")
    assert r2.lat == (lat_t, lat_f)
    # MP_S counts every shared opcode regardless of order (the paper's
    # over-approximation) ...
    shared = P.latency("fadd") + P.latency("br")
    assert r2.mp_s == pytest.approx(shared / (lat_t + lat_f))
    # ... the instruction alignment cannot align both across two gaps
    # (4 + 4 - 2 * GAP < 4), so one of the two is aligned
    assert P.GAP == 4 and r2.saved == 4
    assert r2.profitable == (r2.mp_s >= P.THRESHOLD)


def test_gap_runs_and_occupancy():
    assert P.gap_runs(6, {1, 2, 5}) == 2
    assert P.gap_runs(3, set()) == 1
    assert P.gap_runs(0, set()) == 0
    assert P.waves_per_simd(64) == 8
    assert P.waves_per_simd(79) == 6
    assert P.waves_per_simd(128) == 4
    assert P.waves_per_simd(256, 256) == 1


@pytest.mark.skipif(not os.path.exists(P.HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not installed")
def test_planner_on_region_kernel():
    # The two sides of the divergent region kernel are the same code with
    # different operands: fully aligned, MP_S 0.5, above the threshold.
    fns = P.parse_ir(P.emit_ir("region.hip"))
    fn = P._find(fns, r"region_divergent_kernel", "region.hip")
    (r,) = P.analyse_function(fn, (("true", "false"),))
    assert r.instances == 1
    assert r.mp_s == pytest.approx(0.5) and r.profitable
    assert r.lat[0] == r.lat[1] > 0
    res = P.resources("region.hip")
    d = P._find(res, r"region_divergent_kernel", "region.hip")
    m = P._find(res, r"region_melded_kernel", "region.hip")
    assert 0 < d["vgpr_count"] <= 512 and 0 < m["vgpr_count"] <= 512
    assert d["private_segment_fixed_size"] == 0 and m["private_segment_fixed_size"] == 0


@pytest.mark.skipif(not os.path.exists(P.HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not installed")
def test_planner_on_oddeven_kernel():
    # The odd-even network's divergent form has a lower / upper side pair per
    # step shape (the uniform-role steps and one per compile-time row class of
    # the edge steps). Both sides load a partner and keep one key, so MP_S is
    # high but below the 0.5 of identical sides: the edge rows add idle tests
    # on one side only. The melded form has no sides left and no spills.
    fns = P.parse_ir(P.emit_ir("oddeven.hip"))
    fn = P._find(fns, r"oddeven_bucket_kernelILi8ELi1024ELb0E", "oddeven.hip")
    (r,) = P.analyse_function(fn, (("lower", "upper"),))
    assert r.instances >= 2
    assert P.THRESHOLD <= r.mp_s < 0.5 and r.profitable
    assert min(r.lat) > 0
    melded = P._find(fns, r"oddeven_bucket_kernelILi8ELi1024ELb1E", "oddeven.hip")
    assert not any(b.marks for b in melded.blocks.values())
    res = P.resources("oddeven.hip")
    for pat in (r"oddeven_bucket_kernelILi8ELi1024ELb0E", r"oddeven_bucket_kernelILi8ELi1024ELb1E"):
        k = P._find(res, pat, "oddeven.hip")
        assert k["private_segment_fixed_size"] == 0 and 0 < k["vgpr_count"] <= 64
