"""Static check of wave convergence in the library's device code.

The kernels keep one cell per wavefront and rely on every lane of the wave
taking part in each cross-lane operation (readlane / readfirstlane broadcasts,
ds_bpermute butterflies, wave barriers).  The compiler only guarantees that
where the control flow around such an operation does not depend on the lane.
Two shapes break it in practice:

* a loop whose exit or latch branch depends on the lane index (directly, or
  through a value that differs between lanes) and whose body holds a
  cross-lane operation -- lanes leave the loop in different iterations and
  the rest run the collective without them (this is how a lane-0 queue claim,
  threaded by the optimizer into the previous iteration's lane-0 block, left
  lanes 1..63 spinning on a stale index);
* an if-region on such a branch that holds a cross-lane operation.

The check compiles a HIP source to optimized device LLVM IR (the same flags as
the library build), marks every SSA value derived from the lane index, from a
cross-lane exchange (whose result is not bitwise identical across lanes) or
from a load at a lane-dependent address, and treats readlane / readfirstlane
broadcasts and ballot masks (the same bits on every lane) as uniform.  It then reports natural loops with a tainted exit that
contain a cross-lane operation, and tainted branches whose region up to the
immediate post-dominator contains one.

Test infrastructure only (CPU): it reads IR text, it runs no device code.
"""
import os
import re
import subprocess
from collections import defaultdict

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_18858_amd", "csrc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only", "-S", "-emit-llvm",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]

CROSS_LANE = re.compile(r"@llvm\.amdgcn\.(readfirstlane|readlane|ds\.bpermute|ds\.permute|"
                        r"update\.dpp|mov\.dpp|wave\.barrier|s\.barrier|ds\.swizzle|permlane)")
LANE_SOURCE = re.compile(r"@llvm\.amdgcn\.(workitem\.id|mbcnt|ds\.bpermute|ds\.permute|update\.dpp|"
                         r"mov\.dpp|ds\.swizzle|permlane)")
BROADCAST = re.compile(r"@llvm\.amdgcn\.(readfirstlane|readlane|ballot)")


def emit_ir(src, out):
    """Device IR of one HIP source; raises on a compiler error."""
    r = subprocess.run([HIPCC] + FLAGS + [src, "-o", out], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-2000:]}")
    return out


def functions(ir_text):
    return re.findall(r"^define[^\n]*@([\w.$]+)\(", ir_text, re.M)


def _blocks(ir_text, fname):
    m = re.search(r"^define[^\n]*@" + re.escape(fname) + r"\(.*?^\}", ir_text, re.S | re.M)
    body = m.group(0).split("\n")[1:-1]
    blocks, order, cur = {"<entry>": []}, ["<entry>"], "<entry>"
    for ln in body:
        mm = re.match(r"^([\w.]+):", ln)
        if mm:
            cur = mm.group(1)
            blocks[cur] = []
            order.append(cur)
        elif ln.strip():
            blocks[cur].append(ln.strip())
    return blocks, order


def _terminator(insts):
    k = len(insts) - 1
    while k > 0 and not re.match(r"(br |switch |ret|unreachable)", insts[k]):
        k -= 1
    return " ".join(insts[k:])


def _cond(term):
    m = re.match(r"br i1 %([\w.]+),", term) or re.match(r"switch \w+ %([\w.]+),", term)
    return m.group(1) if m else None


def check_function(ir_text, fname):
    """List of findings (strings) for one function."""
    blocks, order = _blocks(ir_text, fname)
    term = {b: _terminator(blocks[b]) for b in order}
    succ = {b: re.findall(r"label %([\w.]+)", term[b]) for b in order}
    pred = defaultdict(list)
    for b in order:
        for s in succ[b]:
            pred[s].append(b)
    # lane-dependent SSA values
    defs = {}
    for b in order:
        for i in blocks[b]:
            m = re.match(r"^%([\w.]+) = (.*)$", i)
            if m:
                defs[m.group(1)] = m.group(2)
    lane = set()
    changed = True
    while changed:
        changed = False
        for v, rhs in defs.items():
            if v in lane or BROADCAST.search(rhs):
                continue
            if LANE_SOURCE.search(rhs) or any(o in lane for o in re.findall(r"%([\w.]+)", rhs)):
                lane.add(v)
                changed = True
    # dominators / post-dominators (iterative)
    dom = {b: set(order) for b in order}
    dom[order[0]] = {order[0]}
    changed = True
    while changed:
        changed = False
        for b in order[1:]:
            ps = [dom[p] for p in pred[b]]
            nd = (set.intersection(*ps) if ps else set()) | {b}
            if nd != dom[b]:
                dom[b], changed = nd, True
    exits = [b for b in order if not succ[b]]
    pdom = {b: set(order) for b in order}
    for e in exits:
        pdom[e] = {e}
    changed = True
    while changed:
        changed = False
        for b in reversed(order):
            if b in exits:
                continue
            ss = [pdom[s] for s in succ[b]]
            nd = (set.intersection(*ss) if ss else set()) | {b}
            if nd != pdom[b]:
                pdom[b], changed = nd, True

    def n_cross(bs):
        return sum(1 for b in bs for i in blocks[b] if CROSS_LANE.search(i))

    findings = []
    for u in order:
        for h in succ[u]:
            if h not in dom[u]:
                continue
            body, stack = {h, u}, [u]
            while stack:
                x = stack.pop()
                if x == h:
                    continue
                for p in pred[x]:
                    if p not in body:
                        body.add(p)
                        stack.append(p)
            nc = n_cross(body)
            if not nc:
                continue
            bad = [b for b in body if (any(s not in body for s in succ[b]) or b == u)
                   and len(succ[b]) > 1 and _cond(term[b]) in lane]
            if bad:
                findings.append(f"{fname}: loop %{h} (latch %{u}, {nc} cross-lane ops) exits on "
                                f"lane-dependent %{_cond(term[bad[0]])} in %{bad[0]}")
    for b in order:
        c = _cond(term[b]) if len(succ[b]) > 1 else None
        if c not in lane:
            continue
        join, seen, queue = None, {b}, list(succ[b])
        while queue:
            x = queue.pop(0)
            if x in pdom[b] and x != b:
                join = x
                break
            if x not in seen:
                seen.add(x)
                queue.extend(succ[x])
        region, stack = set(), list(succ[b])
        while stack:
            x = stack.pop()
            if x in (join, b) or x in region:
                continue
            region.add(x)
            stack.extend(succ[x])
        nc = n_cross(region)
        if nc:
            findings.append(f"{fname}: region of lane-dependent branch %{b} on %{c} "
                            f"(join %{join}) holds {nc} cross-lane ops")
    return findings


def check_ir(ir_text):
    out = []
    for f in functions(ir_text):
        out += check_function(ir_text, f)
    return out
