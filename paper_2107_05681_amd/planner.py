"""Offline meld planner: the paper's melding profitability and instruction
alignment (Detailed Design section, "Melding Profitability" and "Instruction
Alignment"), run over this library's own divergent kernels as a checker.

For every divergent region of a kernel (located by the side marks the
divergent forms carry, ``; side <name>``), the planner

* takes the LLVM IR that hipcc emits for gfx950 and builds each function's
  control-flow graph,
* finds the region: the branch block is the nearest common dominator of the
  sides' entry blocks, the join is its immediate post-dominator, and a side's
  subgraph is every block reachable from its entry without passing the join,
* scores block pairs with the basic-block melding profitability
      MP_B(b1, b2) = sum_i min(freq(i, b1), freq(i, b2)) w_i / (lat(b1) + lat(b2))
  (freq: opcode histogram, w_i: static latency of opcode class i, lat: summed
  latency), aligns the two sides' linearised blocks with Smith-Waterman on
  that score, and reports the subgraph profitability
      MP_S = sum_O MP_B(b1, b2) (lat(b1) + lat(b2)) / sum_O (lat(b1) + lat(b2))
  over the aligned block pairs O,
* aligns the instructions of every aligned block pair with Smith-Waterman:
  only instructions of the same opcode class align, an aligned pair scores
  its latency, an unaligned instruction costs a gap (the branch that
  unpredication puts around it), and the aligned latency is the cycles a
  meld saves in a wave that runs both sides.

The latency table is a static model of gfx950 (cycles a wave64 instruction
occupies its unit, LDS and global memory at their load-to-use latency); the
paper takes w_i from LLVM's cost model, which has no table for this target.

Command line: ``python -m paper_2107_05681_amd.planner [bench.json]`` prints one
line per region, with the measured melded/divergent speedups of a bench.py
JSON line beside the kernels they belong to.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "csrc")
_INCLUDE = os.path.join(os.path.dirname(_HERE), "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Static latency per opcode class (cycles), gfx950 model.
LATENCY = {
    "load.lds": 64, "store.lds": 64, "load.global": 500, "store.global": 100,
    "load": 100, "store": 100, "atomicrmw": 500, "cmpxchg": 500,
    "fadd": 4, "fsub": 4, "fmul": 4, "fdiv": 16, "fneg": 4, "fcmp": 4,
    "add": 4, "sub": 4, "mul": 4, "shl": 4, "lshr": 4, "ashr": 4, "and": 4, "or": 4,
    "xor": 4, "udiv": 32, "urem": 32, "sdiv": 32, "srem": 32, "icmp": 4, "select": 4,
    "zext": 4, "sext": 4, "trunc": 4, "bitcast": 0, "getelementptr": 4, "extractelement": 4,
    "insertelement": 4, "shufflevector": 4, "uitofp": 4, "fptoui": 4, "sitofp": 4,
    "fptosi": 4, "fpext": 4, "fptrunc": 4, "freeze": 0, "phi": 0,
    "call.fma": 4, "call.umin": 4, "call.umax": 4, "call.smin": 4, "call.smax": 4,
    "call.barrier": 32, "call.other": 8, "call.mark": 0,
    "br": 4, "switch": 8, "ret": 4, "unreachable": 0, "fence": 16,
}
GAP = 4  # an unaligned instruction: the branch unpredication adds around it


def latency(op: str) -> int:
    return LATENCY.get(op, 4)


@dataclass
class Block:
    name: str
    ops: list = field(default_factory=list)
    succ: list = field(default_factory=list)
    marks: list = field(default_factory=list)


@dataclass
class Function:
    name: str
    blocks: dict  # name -> Block, in source order
    order: list


_CALL_CLASSES = (("llvm.fma", "call.fma"), ("llvm.fmuladd", "call.fma"),
                 ("llvm.umin", "call.umin"), ("llvm.umax", "call.umax"),
                 ("llvm.smin", "call.smin"), ("llvm.smax", "call.smax"),
                 ("llvm.amdgcn.s.barrier", "call.barrier"))


def _op_class(line: str) -> str:
    body = line.strip()
    if "=" in body.split("(")[0] and body.startswith("%"):
        body = body.split("=", 1)[1].strip()
    words = body.split()
    while words and words[0] in ("tail", "musttail", "notail"):
        words = words[1:]
    if not words:
        return "unknown"
    op = words[0]
    if op == "call":
        if "asm sideeffect" in body:
            return "call.mark"
        for key, cls in _CALL_CLASSES:
            if key in body:
                return cls
        return "call.other"
    if op in ("load", "store"):
        if "addrspace(3)" in body:
            return op + ".lds"
        if "addrspace(1)" in body:
            return op + ".global"
        return op
    return op


def parse_ir(text: str) -> dict:
    """Functions of an LLVM IR module: name -> Function (blocks with opcode
    classes, successors and side marks)."""
    funcs = {}
    lines = text.split("\n")
    i = 0
    while i < len(lines):
        m = re.match(r"define .*@([\w.$]+)\((.*)", lines[i])
        if not m:
            i += 1
            continue
        name = m.group(1)
        # the entry block is numbered after the unnamed arguments
        nargs = len(re.findall(r"%\d+(?=[,)])", lines[i]))
        blocks, order = {}, []
        cur = Block(str(nargs))
        blocks[cur.name] = cur
        order.append(cur.name)
        i += 1
        while i < len(lines) and not lines[i].startswith("}"):
            ln = lines[i]
            lm = re.match(r"^([\w.]+):", ln)
            if lm:
                cur = Block(lm.group(1))
                blocks[cur.name] = cur
                order.append(cur.name)
            elif ln.startswith("  ") and ln.strip():
                op = _op_class(ln)
                cur.ops.append(op)
                mk = re.search(r'asm sideeffect "; side ([^"]+)"', ln)
                if mk:
                    cur.marks.append(mk.group(1))
                if op in ("br", "switch"):
                    cur.succ += re.findall(r"label %([\w.]+)", ln)
            i += 1
        funcs[name] = Function(name, blocks, order)
        i += 1
    return funcs


def _rpo(succ: dict, entry: str) -> list:
    seen, out = set(), []

    def dfs(u):
        stack = [(u, iter(succ.get(u, ())))]
        seen.add(u)
        while stack:
            node, it = stack[-1]
            nxt = next((v for v in it if v not in seen), None)
            if nxt is None:
                stack.pop()
                out.append(node)
            else:
                seen.add(nxt)
                stack.append((nxt, iter(succ.get(nxt, ()))))
    dfs(entry)
    return out[::-1]


def dominators(succ: dict, entry: str) -> dict:
    """Immediate dominators (Cooper, Harvey and Kennedy's iterative algorithm)."""
    order = _rpo(succ, entry)
    index = {b: k for k, b in enumerate(order)}
    preds = {b: [] for b in order}
    for u in order:
        for v in succ.get(u, ()):
            if v in preds:
                preds[v].append(u)
    idom = {entry: entry}

    def intersect(a, b):
        while a != b:
            while index[a] > index[b]:
                a = idom[a]
            while index[b] > index[a]:
                b = idom[b]
        return a
    changed = True
    while changed:
        changed = False
        for b in order[1:]:
            ps = [p for p in preds[b] if p in idom]
            if not ps:
                continue
            new = ps[0]
            for p in ps[1:]:
                new = intersect(p, new)
            if idom.get(b) != new:
                idom[b] = new
                changed = True
    return idom


def post_dominators(fn: Function) -> dict:
    exit_ = "<exit>"
    rsucc = {exit_: []}
    for b in fn.order:
        rsucc.setdefault(b, [])
    for b in fn.order:
        blk = fn.blocks[b]
        targets = blk.succ if blk.succ else [exit_]
        for t in targets:
            rsucc.setdefault(t, []).append(b)
    return dominators(rsucc, exit_)


def _ancestors(idom, b):
    out = [b]
    while idom.get(b, b) != b:
        b = idom[b]
        out.append(b)
    return out


def side_blocks(fn: Function, entry: str, join: str) -> list:
    """Blocks reachable from entry without passing join, in reverse post-order."""
    sub = {}
    stack, seen = [entry], {entry}
    while stack:
        u = stack.pop()
        sub[u] = [v for v in fn.blocks[u].succ if v != join]
        for v in sub[u]:
            if v not in seen and v in fn.blocks:
                seen.add(v)
                stack.append(v)
    return [b for b in _rpo(sub, entry) if b in fn.blocks]


def histogram(ops) -> dict:
    h = {}
    for op in ops:
        if op in ("phi", "call.mark"):
            continue
        h[op] = h.get(op, 0) + 1
    return h


def block_latency(ops) -> int:
    return sum(latency(op) for op in ops if op not in ("phi", "call.mark"))


def mp_b(ops1, ops2) -> float:
    """Basic-block melding profitability."""
    h1, h2 = histogram(ops1), histogram(ops2)
    den = block_latency(ops1) + block_latency(ops2)
    if den == 0:
        return 0.0
    num = sum(min(h1[i], h2[i]) * latency(i) for i in h1 if i in h2)
    return num / den


def smith_waterman(a, b, score, gap):
    """Local alignment of sequences a and b: score(x, y) is the gain of aligning
    x with y (None: not alignable), gap the cost of leaving one unaligned.
    Returns (best score, aligned index pairs)."""
    n, m = len(a), len(b)
    H = [[0.0] * (m + 1) for _ in range(n + 1)]
    best, bi, bj = 0.0, 0, 0
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            s = score(a[i - 1], b[j - 1])
            diag = H[i - 1][j - 1] + s if s is not None else float("-inf")
            H[i][j] = max(0.0, diag, H[i - 1][j] - gap, H[i][j - 1] - gap)
            if H[i][j] > best:
                best, bi, bj = H[i][j], i, j
    pairs = []
    i, j = bi, bj
    while i > 0 and j > 0 and H[i][j] > 0:
        s = score(a[i - 1], b[j - 1])
        if s is not None and H[i][j] == H[i - 1][j - 1] + s:
            pairs.append((i - 1, j - 1))
            i, j = i - 1, j - 1
        elif H[i][j] == H[i - 1][j] - gap:
            i -= 1
        else:
            j -= 1
    return best, pairs[::-1]


def real_ops(ops):
    """The instructions of a block that execute (no phi nodes or side marks)."""
    return [op for op in ops if op not in ("phi", "call.mark")]


def _instr_score(x, y):
    """Instruction alignment score: same opcode class only, weighted by latency
    so that costly instructions are aligned first."""
    return float(latency(x)) if x == y else None


@dataclass
class RegionReport:
    kernel: str
    sides: tuple
    instances: int   # copies of the region in the function (unrolled loops)
    blocks: tuple    # blocks per side, summed over the copies
    lat: tuple       # static latency per side, summed over the copies
    mp_s: float      # subgraph melding profitability (latency-weighted over copies)
    saved: int       # latency of the aligned instructions
    gaps: int        # runs of unaligned instructions (a branch each)

    @property
    def saved_fraction(self) -> float:
        tot = self.lat[0] + self.lat[1]
        return self.saved / tot if tot else 0.0

    @property
    def melded_cost(self) -> int:
        return self.lat[0] + self.lat[1] - self.saved + GAP * self.gaps

    @property
    def predicted_speedup(self) -> float:
        """Cycles of a wave that runs both sides, divergent over melded."""
        return (self.lat[0] + self.lat[1]) / self.melded_cost if self.melded_cost else 0.0

    @property
    def profitable(self) -> bool:
        return self.mp_s >= THRESHOLD


THRESHOLD = 0.2  # the paper's default melding profitability threshold


def gap_runs(n: int, aligned) -> int:
    """Maximal runs of indices in [0, n) that are not in aligned."""
    runs, inside = 0, False
    for k in range(n):
        if k in aligned:
            inside = False
        elif not inside:
            runs, inside = runs + 1, True
    return runs


def align_sides(ops1, ops2):
    """Block alignment of two sides (Smith-Waterman on MP_B), then instruction
    alignment of every aligned block pair. Returns (MP_S numerator and
    denominator, saved latency, gap runs)."""
    _, bpairs = smith_waterman(ops1, ops2, mp_b, 0.05)
    num = den = 0.0
    saved = gaps = 0
    b1 = {i for i, _ in bpairs}
    b2 = {j for _, j in bpairs}
    for i, j in bpairs:
        w = block_latency(ops1[i]) + block_latency(ops2[j])
        num += mp_b(ops1[i], ops2[j]) * w
        den += w
        r1, r2 = real_ops(ops1[i]), real_ops(ops2[j])
        _, ipairs = smith_waterman(r1, r2, _instr_score, GAP)
        saved += sum(latency(r1[a]) for a, _ in ipairs)
        gaps += gap_runs(len(r1), {a for a, _ in ipairs})
        gaps += gap_runs(len(r2), {b for _, b in ipairs})
    # an unaligned block runs under its own branch
    gaps += sum(1 for k in range(len(ops1)) if k not in b1 and block_latency(ops1[k]))
    gaps += sum(1 for k in range(len(ops2)) if k not in b2 and block_latency(ops2[k]))
    return num, den, saved, gaps


def _depth(idom, b):
    return len(_ancestors(idom, b))


def region_of(fn: Function, idom: dict, ipdom: dict, e1: str, e2: str):
    """(branch, join, side 1 blocks, side 2 blocks) of the region whose sides
    start at e1 and e2."""
    anc1 = _ancestors(idom, e1)
    branch = next(b for b in _ancestors(idom, e2) if b in anc1)
    join = ipdom.get(branch, "<exit>")
    return branch, join, side_blocks(fn, e1, join), side_blocks(fn, e2, join)


def analyse_function(fn: Function, pairs=None) -> list:
    """One report per side pair present in fn, over all its copies; each copy
    of side 1 is paired with the copy of side 2 that branches off closest."""
    marks = {}
    for b in fn.order:
        for mk in fn.blocks[b].marks:
            marks.setdefault(mk, []).append(b)
    if not marks:
        return []
    idom = dominators({b: fn.blocks[b].succ for b in fn.order}, fn.order[0])
    ipdom = post_dominators(fn)
    out = []
    for n1, n2 in pairs or SIDE_PAIRS:
        e1s = [b for b in marks.get(n1, []) if b in idom]
        e2s = [b for b in marks.get(n2, []) if b in idom]
        if not e1s or not e2s:
            continue
        num = den = 0.0
        saved = gaps = nb1 = nb2 = l1 = l2 = count = 0
        free = set(e2s)
        pos = {b: k for k, b in enumerate(fn.order)}
        preds = {}
        for b in fn.order:
            for v in fn.blocks[b].succ:
                preds.setdefault(v, set()).add(b)
        for e1 in e1s:
            anc1 = set(_ancestors(idom, e1))

            def rank(e2):
                # a common predecessor (the branch of an if/else) first, then
                # the deepest common dominator, then the nearest block
                shared = bool(preds.get(e1, set()) & preds.get(e2, set()))
                ncd = next(b for b in _ancestors(idom, e2) if b in anc1)
                return (not shared, -_depth(idom, ncd), abs(pos[e1] - pos[e2]))
            cands = sorted(free, key=rank)
            if not cands:
                break
            e2 = cands[0]
            free.discard(e2)
            _, _, s1, s2 = region_of(fn, idom, ipdom, e1, e2)
            ops1 = [fn.blocks[b].ops for b in s1]
            ops2 = [fn.blocks[b].ops for b in s2]
            a, d, sv, g = align_sides(ops1, ops2)
            num, den, saved, gaps = num + a, den + d, saved + sv, gaps + g
            nb1, nb2 = nb1 + len(s1), nb2 + len(s2)
            l1 += sum(block_latency(o) for o in ops1)
            l2 += sum(block_latency(o) for o in ops2)
            count += 1
        out.append(RegionReport(fn.name, (n1, n2), count, (nb1, nb2), (l1, l2),
                                num / den if den else 0.0, saved, gaps))
    return out


# Side pairs of the library's divergent forms.
SIDE_PAIRS = (("ascending", "descending"), ("ascending batch", "descending batch"),
              ("ascending regs", "descending regs"), ("true", "false"), ("lower", "upper"),
              ("take a", "take b"), ("way 0", "way 1"), ("way 0", "way 2"), ("way 1", "way 2"))


def _emit(source: str, llvm: bool) -> str:
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.out")
        subprocess.check_call(
            [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{_INCLUDE}",
             f"-I{_CSRC}", "--offload-device-only", "-S"] + (["-emit-llvm"] if llvm else [])
            + [os.path.join(_CSRC, source), "-o", out], stderr=subprocess.DEVNULL)
        with open(out) as f:
            return f.read()


def emit_ir(source: str) -> str:
    """LLVM IR of one library source for gfx950 (built here, device code only)."""
    return _emit(source, True)


def resources(source: str) -> dict:
    """Per kernel of one library source: VGPRs, AGPRs, SGPRs, static LDS bytes
    and private (scratch) bytes, from the code-object metadata of its gfx950
    assembly."""
    out, cur = {}, {}
    for ln in _emit(source, False).split("\n"):
        m = re.match(r"\s*-?\s*\.(agpr_count|vgpr_count|sgpr_count|name|"
                     r"group_segment_fixed_size|private_segment_fixed_size):\s*(\S+)", ln)
        if not m:
            continue
        key, val = m.groups()
        if key == "agpr_count" and cur:  # first field of the next kernel's record
            if "name" in cur:
                out[cur["name"]] = cur
            cur = {}
        cur[key] = val if key == "name" else int(val)
    if "name" in cur:
        out[cur["name"]] = cur
    return out


def waves_per_simd(vgprs: int, agprs: int = 0) -> int:
    """Resident waves per SIMD that the register file allows: 512 registers
    per lane (VGPRs and AGPRs together, allocated in granules of 8), at most
    8 waves."""
    used = max(1, vgprs + agprs)
    return min(8, 512 // (-(-used // 8) * 8))


# Divergent kernels of the library, their melded counterparts, the side pairs
# of their regions and the bench.py figure that times the two forms.
KERNELS = (
    ("region.hip", r"region_divergent_kernel", r"region_melded_kernel", (("true", "false"),),
     ("region", "melded_vs_divergent", "0.5", "speedup")),
    ("region_variants.hip", r"region3_divergent_kernel", r"region3_melded_kernel",
     (("way 0", "way 1"), ("way 0", "way 2"), ("way 1", "way 2")),
     ("region", "region_variants", "three_way_thirds", "speedup")),
    ("region_variants.hip", r"region_lt_divergent_kernel", r"region_lt_melded_kernel",
     (("true", "false"),), ("region", "region_variants", "per_lane_trips_8_32_p0.5", "speedup")),
    ("bitonic_local_lds.hip", r"bitonic_sort_regs_kernelILb0ELi13ELb0ELb0E",
     r"bitonic_sort_regs_kernelILb0ELi13ELb1ELb1E",
     (("ascending batch", "descending batch"), ("ascending regs", "descending regs")),
     ("sort_keys_2^16", "lds", "local_sort_kernel", "speedup")),
    ("oddeven.hip", r"oddeven_bucket_kernelILi8ELi1024ELb0E", r"oddeven_bucket_kernelILi8ELi1024ELb1E",
     (("lower", "upper"),), ("oddeven_buckets", "buckets_2^13", "speedup")),
    ("mergesort.hip", r"merge_pass_kernelILb0E", r"merge_pass_kernelILb1E", (("take a", "take b"),),
     ("mergesort", "keys_2^24", "merge_passes_speedup")),
    ("segsort.hip", r"seg_sort_kernelILb0ELb0E", r"seg_sort_kernelILb1ELb1E",
     (("ascending", "descending"), ("ascending batch", "descending batch"),
      ("ascending regs", "descending regs")),
     ("segmented", "seed_1", "speedup_melded_lds_path")),
)


@dataclass
class KernelPlan:
    name: str
    key: tuple
    regions: list             # RegionReport per side pair
    divergent: dict           # resources of the divergent kernel
    melded: dict              # resources of the melded kernel

    @property
    def occupancy(self) -> tuple:
        return (waves_per_simd(self.divergent["vgpr_count"], self.divergent["agpr_count"]),
                waves_per_simd(self.melded["vgpr_count"], self.melded["agpr_count"]))


def _find(table: dict, pattern: str, source: str):
    hits = [v for name, v in table.items() if re.search(pattern, name)]
    if not hits:
        raise RuntimeError(f"no kernel matching {pattern} in {source}")
    return hits[0]


def plan(kernels=KERNELS) -> list:
    """A KernelPlan for every kernel of the table."""
    out, irs, res = [], {}, {}
    for source, div, mel, pairs, key in kernels:
        if source not in irs:
            irs[source] = parse_ir(emit_ir(source))
            res[source] = resources(source)
        fn = _find(irs[source], div, source)
        out.append(KernelPlan(re.sub(r"I.*", "", div), key, analyse_function(fn, pairs),
                              _find(res[source], div, source), _find(res[source], mel, source)))
    return out


def measured(bench, key):
    """The speedup a bench.py JSON line records under key, or None."""
    if bench is None or key is None:
        return None
    v = bench
    for part in key:
        if part is None:
            continue
        if not isinstance(v, dict) or part not in v:
            return None
        v = v[part]
    return v


def main(argv=None) -> int:
    import json
    argv = sys.argv[1:] if argv is None else argv
    bench = None
    if argv:
        with open(argv[0]) as f:
            bench = json.loads([ln for ln in f if ln.startswith("{")][-1])
    print(f"{'kernel':26s} {'sides':34s} {'n':>3s} {'lat/side':>11s} {'MP_S':>5s} "
          f"{'saved':>5s} {'pred':>5s} {'meld?':>5s} {'VGPR d/m':>8s} {'waves':>5s} "
          f"{'measured':>8s}")
    for kp in plan():
        meas = measured(bench, kp.key)
        vg = f"{kp.divergent['vgpr_count']}/{kp.melded['vgpr_count']}"
        occ = "%d/%d" % kp.occupancy
        for r in kp.regions:
            print(f"{kp.name[:26]:26s} {' / '.join(r.sides)[:34]:34s} {r.instances:3d} "
                  f"{r.lat[0]:5d},{r.lat[1]:<5d} {r.mp_s:5.3f} {r.saved_fraction:5.3f} "
                  f"{r.predicted_speedup:5.2f} {'yes' if r.profitable else 'no':>5s} "
                  f"{vg:>8s} {occ:>5s} {meas if meas is not None else '-':>8}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
