"""Count the VALU work of one event in a compiled ssa_kernel code object.

The kernel's event loop is the innermost loop that contains the Philox
multiplies (v_mad_u64_u32); one event is its lightest cycle through the block
holding the next event's Philox calls (see event_paths). Rare paths (snapshot
stores, trajectory completion, the selection fallback, refills) are excluded
by construction. Each VALU instruction on the path is weighted by its issue cost
in full-rate lane slots (one wave64 instruction on a 16-lane SIMD in 4 cycles
= 1), by rate class. The classes are the ones libssa_valu_peak.so measures on
MI355X at 8 waves per SIMD, relative to the full-rate classes (v_bitop3_b32,
v_mad_u64_u32, f64 add/mul/fma, v_cndmask_b32: 4.3-4.8 cycles at the nominal
2.4 GHz):
  0.5  f32 add / sub / mul / fma and 32-bit integer add / sub (2.4-2.8
       cycles with VGPR operands: the double-rate pipe; an SGPR operand makes
       some of them full rate, so 0.5 is the lower bound of their cost and
       the fraction of peak is never overstated);
  2    f32 transcendentals (v_rcp_f32: 8.5 cycles) and the SR conversions
       (v_cvt_sr_*: about 8 cycles);
  4    f64 transcendentals (v_rcp_f64: 16.6 cycles);
  1    everything else, including the 64-bit multiply-add Philox uses, which
       issues at the full rate on gfx950.

Usage: python -m paper_2605_00479_amd.csrc.valu_count <file.co>
"""
from __future__ import annotations

import re
import subprocess
import sys

OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"

_HALF = re.compile(r"^v_(mul_f32|fma_f32|fmac_f32|fmamk_f32|fmaak_f32|mac_f32|mad_f32|add_f32|sub_f32|subrev_f32|"
                   r"add_u32|sub_u32|subrev_u32)")
_TRANS64 = re.compile(r"^v_(rcp|rsq|sqrt)_f64")
_DOUBLE = re.compile(r"^v_(rcp_|rsq_|sqrt_|log_|exp_|sin_|cos_|rcp_iflag|cvt_sr_)")


def weight(op: str) -> float:
    """Issue cost of one VALU instruction in full-rate lane slots."""
    if _TRANS64.match(op):
        return 4.0
    if _DOUBLE.match(op):
        return 2.0
    if _HALF.match(op):
        return 0.5
    return 1.0

_LINE = re.compile(r"^\s+(\S+)(.*?)//\s*([0-9A-Fa-f]+):.*?(?:<(\w+)\+0x([0-9a-f]+)>)?\s*$")


def disassemble(co_path: str, func: str = "ssa_kernel"):
    out = subprocess.run([OBJDUMP, "-d", "--no-show-raw-insn", co_path], capture_output=True, text=True,
                         check=True).stdout
    insts, cur, base = [], None, None
    for line in out.splitlines():
        m = re.match(r"^([0-9a-f]+) <(\w+)>:", line)
        if m:
            cur = m.group(2)
            base = int(m.group(1), 16)
            continue
        if cur != func:
            continue
        m = _LINE.match(line)
        if not m:
            continue
        op, addr = m.group(1), int(m.group(3), 16)
        target = base + int(m.group(5), 16) if m.group(4) == func and m.group(5) else None
        insts.append((addr, op, target))
    return insts


def build_cfg(insts):
    leaders = {insts[0][0]}
    for i, (addr, op, tgt) in enumerate(insts):
        if op.startswith(("s_branch", "s_cbranch")):
            if tgt is not None:
                leaders.add(tgt)
            if i + 1 < len(insts):
                leaders.add(insts[i + 1][0])
        if op == "s_endpgm" and i + 1 < len(insts):
            leaders.add(insts[i + 1][0])
    blocks, order = {}, []
    cur = None
    for addr, op, tgt in insts:
        if addr in leaders:
            cur = addr
            blocks[cur] = []
            order.append(cur)
        blocks[cur].append((addr, op, tgt))
    succ = {}
    for i, b in enumerate(order):
        last_op, last_tgt = blocks[b][-1][1], blocks[b][-1][2]
        nxt = order[i + 1] if i + 1 < len(order) else None
        s = []
        if last_op.startswith("s_branch"):
            s = [last_tgt]
        elif last_op.startswith("s_cbranch"):
            s = [last_tgt, nxt]
        elif last_op == "s_endpgm":
            s = []
        else:
            s = [nxt]
        succ[b] = [x for x in s if x is not None]
    return blocks, order, succ


def dominators(nodes, succ, root):
    pred = {n: [] for n in nodes}
    for n in nodes:
        for s in succ.get(n, []):
            if s in pred:
                pred[s].append(n)
    dom = {n: set(nodes) for n in nodes}
    dom[root] = {root}
    changed = True
    while changed:
        changed = False
        for n in nodes:
            if n == root:
                continue
            ps = [dom[p] for p in pred[n]]
            new = ({n} | set.intersection(*ps)) if ps else {n}
            if new != dom[n]:
                dom[n] = new
                changed = True
    return dom


def reachable(succ, root, allowed):
    seen, stack = {root}, [root]
    while stack:
        n = stack.pop()
        for s in succ.get(n, []):
            if s in allowed and s not in seen:
                seen.add(s)
                stack.append(s)
    return seen


def _natural_loops(order, succ, dom):
    loops = []
    for u in order:
        for v in succ[u]:
            if v in dom[u]:
                body = {v}
                stack = [u]
                while stack:
                    n = stack.pop()
                    if n not in body:
                        body.add(n)
                        stack.extend(p for p in order if n in succ[p])
                loops.append((v, u, body))
    # one loop per header: the union of its back edges' bodies
    merged = {}
    for h, _, body in loops:
        merged[h] = merged.get(h, set()) | body
    return merged


def _is_mul(op):   # the Philox 32x32->64 multiplies (fused, or split into high/low halves)
    return op in ("v_mad_u64_u32", "v_mul_hi_u32")


def _slots(block):
    return sum(weight(op) for _, op, _ in block if op.startswith("v_"))


def _lightest_cycle(blocks, succ, body, B):
    """Cycle from B back to B inside `body` with the fewest VALU slots
    (Dijkstra with block weights; edges into B end at a sink)."""
    import heapq
    best = {B: _slots(blocks[B])}
    prev = {}
    heap = [(best[B], B)]
    while heap:
        c, n = heapq.heappop(heap)
        if c > best.get(n, float("inf")):
            continue
        if n == -1:
            path, m = [], prev[-1]
            while m != B:
                path.append(m)
                m = prev[m]
            path.append(B)
            return c, sorted(path)
        for t in succ[n]:
            if t not in body:
                continue
            nxt, nc = (-1, c) if t == B else (t, c + _slots(blocks[t]))
            if nc < best.get(nxt, float("inf")):
                best[nxt] = nc
                prev[nxt] = n
                heapq.heappush(heap, (nc, nxt))
    return None


def event_paths(co_path: str):
    """Lightest event of each copy of the event loop (the compiler may
    unswitch it). Every iteration of an innermost loop holding the Philox calls
    passes through the block with the next event's draw, so one event is the
    lightest cycle through some block holding Philox multiplies: the minimum,
    over those blocks, of the cycle through the block with the fewest VALU
    slots. Rare blocks (snapshot stores, status resolution, completion, the
    selection fallback, refills, extra random streams drawn only in rare
    cases) are off that cycle, and where a wave-uniform test picks one of two
    versions of a step, the lighter is counted, so the work derived from it is
    never overstated."""
    insts = disassemble(co_path)
    blocks, order, succ = build_cfg(insts)
    dom = dominators(order, succ, order[0])
    loops = _natural_loops(order, succ, dom)

    def n_mul(bs):
        return sum(1 for b in bs for _, op, _ in blocks[b] if _is_mul(op))

    cands = {h: body for h, body in loops.items() if n_mul(body) >= 18}
    # innermost: contains no other candidate's header
    inner = {h: body for h, body in cands.items() if not any(h2 != h and h2 in body for h2 in cands)}
    paths = []
    for h, body in inner.items():
        cycles = [_lightest_cycle(blocks, succ, body, b) for b in sorted(body) if n_mul([b]) >= 8]
        cycles = [cy for cy in cycles if cy is not None]
        if cycles:
            paths.append(min(cycles)[1])
    if not paths:
        raise RuntimeError("no event loop found in " + co_path)
    return blocks, paths


def event_path(co_path: str):
    """The lightest event over the event loop's copies."""
    blocks, paths = event_paths(co_path)
    return blocks, min(paths, key=lambda p: sum(_slots(blocks[b]) for b in p))


def count(co_path: str) -> dict:
    blocks, path = event_path(co_path)
    n_valu = n_salu = 0
    n_slots = 0.0
    multi = 0
    for b in path:
        for _, op, _ in blocks[b]:
            if op.startswith("v_"):
                w = weight(op)
                n_valu += 1
                n_slots += w
                multi += w > 1.0
            elif op.startswith("s_"):
                n_salu += 1
    return {"valu_insts": n_valu, "valu_slots": n_slots, "multi_cycle_insts": multi, "salu_insts": n_salu,
            "blocks": len(path)}


if __name__ == "__main__":
    print(count(sys.argv[1]))
