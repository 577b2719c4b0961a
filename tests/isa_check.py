"""Structural checks on the AMD GPU assembly of a kernel built here (test
helper, no GPU needed).

A workgroup barrier (s_barrier) is safe only where every wave reaches it with
its lanes together.  Two compiled shapes break that:

* a loop whose exit is decided per lane: the compiler lowers it by masking off
  the lanes that leave (``s_andn2_b64 exec, exec, ...``) while the others keep
  iterating; if such a loop contains a barrier, the remaining lanes keep
  passing barriers while the lanes that left wait for them, and if those lanes
  are the ones that would end the loop (a ticket taken by lane 0 alone), the
  launch never finishes;
* a barrier inside a lane-masked region (between ``s_and_saveexec_b64 sX``
  and the ``s_or_b64 exec, exec, sX`` that closes it).

Loops are read from the compiler's own annotations of the assembly ("Loop
Header: Depth=k", "in Loop: Header=BBx", "Parent Loop BBy").
"""
from __future__ import annotations

import re


def function_lines(asm: str, symbol: str) -> list[str]:
    """Lines of one function, from its label to its end marker."""
    lines = asm.splitlines()
    start = next(i for i, ln in enumerate(lines) if ln.startswith(symbol + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    return lines[start:end]


def kernel_symbols(asm: str, fragment: str) -> list[str]:
    """Names of the functions whose label contains `fragment`."""
    return [m.group(1) for m in re.finditer(r"^(\S*" + re.escape(fragment) + r"\S*):", asm, re.M)]


def _blocks(lines):
    """(name, innermost loop header or None, instructions) per basic block.
    A block starts at a .LBB label or an '; %bb.' comment."""
    blocks = []
    name, loop, body = "entry", None, []
    parents = {}
    for ln in lines:
        lab = re.match(r"^\.L(BB\d+_\d+):(.*)$", ln)
        bbc = re.match(r"^; %bb\.(\d+):(.*)$", ln)
        if lab or bbc:
            blocks.append((name, loop, body))
            name = lab.group(1) if lab else "bb." + bbc.group(1)
            rest = lab.group(2) if lab else bbc.group(2)
            body = []
            loop = None
            h = re.search(r"Header=(BB\d+_\d+)", rest)
            if h:
                loop = h.group(1)
            if "Loop Header" in rest and lab:
                loop = name
            continue
        par = re.search(r"Parent Loop (BB\d+_\d+)", ln)
        if par and loop == name:
            parents[name] = par.group(1)
        ins = ln.split(";")[0].strip()
        if ins and not ins.startswith("."):
            body.append(ins)
    blocks.append((name, loop, body))
    return blocks, parents


def loops_with_divergent_barriers(lines) -> list[str]:
    """Headers of loops that contain a barrier (in themselves or a nested
    loop) and whose own blocks mask off exiting lanes."""
    blocks, parents = _blocks(lines)

    def ancestors(h):
        out = []
        while h is not None:
            out.append(h)
            h = parents.get(h)
        return out

    has_barrier, divergent = set(), set()
    for _, loop, body in blocks:
        if loop is None:
            continue
        if any(i.startswith("s_barrier") for i in body):
            has_barrier.update(ancestors(loop))
        if any(re.match(r"s_andn2_b64 exec, exec,", i) for i in body):
            divergent.add(loop)
    return sorted(has_barrier & divergent)


def barriers_in_masked_regions(lines) -> int:
    """Barriers met (in layout order) while a lane-masked region is open."""
    open_regions: list[str] = []
    count = 0
    for ln in lines:
        ins = ln.split(";")[0].strip()
        m = re.match(r"s_and_saveexec_b64 (s\[\d+:\d+\])", ins)
        if m:
            open_regions.append(m.group(1))
            continue
        m = re.match(r"s_or_b64 exec, exec, (s\[\d+:\d+\])", ins)
        if m and m.group(1) in open_regions:
            k = len(open_regions) - 1 - open_regions[::-1].index(m.group(1))
            del open_regions[k:]
            continue
        if ins.startswith("s_barrier") and open_regions:
            count += 1
    return count
