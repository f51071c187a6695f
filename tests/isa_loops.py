"""Loop structure of compiled gfx950 kernels, read from the assembly that hipcc
writes for code built here (`--cuda-device-only -S`).

A workgroup barrier inside a loop is only safe when every wave takes the
loop's back edge together.  The compiler annotates each basic block with its
innermost loop ("; in Loop: Header=BBf_n Depth=d") and each loop header with
its parents; from these the checker finds, for every loop that contains an
`s_barrier`, the blocks that jump (or fall through) back to its header, and
reports a latch whose decision is taken on the EXEC mask: such a loop lets
some lanes of a wave go round again while others leave, so the wave reaches
the barrier with part of its lanes and the lanes left behind never run again.
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field

_LABEL = re.compile(r"^(\.LBB\d+_\d+|; %bb\.\d+):")
_IN_LOOP = re.compile(r";\s+in Loop: Header=BB(\d+_\d+) Depth=(\d+)")
_HEADER = re.compile(r"=>\s*This (?:Inner )?Loop Header: Depth=(\d+)")
_PARENT = re.compile(r";\s+Parent Loop BB(\d+_\d+) Depth=(\d+)")
_BRANCH = re.compile(r"^\s*(s_branch|s_cbranch_\w+)\s+\.LBB(\d+_\d+)")


@dataclass
class Block:
    name: str                       # "BB2_11" or "bb.12" (unnamed fall-through block)
    loop: str | None = None         # innermost loop header ("BB2_11"), None outside loops
    lines: list = field(default_factory=list)

    def instructions(self):
        return [l.strip() for l in self.lines if l.strip() and not l.strip().startswith(";")]


def kernel_blocks(asm: str, symbol: str) -> list[Block]:
    lines = asm.split("\n")
    start = next(i for i, l in enumerate(lines) if l.startswith(symbol + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    blocks = [Block("entry")]
    for raw in lines[start + 1:end]:
        m = _LABEL.match(raw)
        if m:
            name = m.group(1)
            name = name[2:] if name.startswith(".LBB") else "bb." + name.split(".")[-1]
            blocks.append(Block(name))
        b = blocks[-1]
        mh = _HEADER.search(raw)
        if mh:
            b.loop = b.name                 # a header is in its own loop
        mi = _IN_LOOP.search(raw)
        if mi and b.loop is None:
            b.loop = "BB" + mi.group(1)
        b.lines.append(raw)
    return blocks


def loop_parents(asm: str, symbol: str) -> dict:
    """header -> parent header (None for outermost loops)."""
    lines = asm.split("\n")
    start = next(i for i, l in enumerate(lines) if l.startswith(symbol + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    parents, cur, chain = {}, None, []
    for raw in lines[start + 1:end]:
        m = _LABEL.match(raw)
        if m:                               # the label line may carry the first annotation
            cur, chain = m.group(1), []
        mp = _PARENT.search(raw)
        if mp:
            chain.append("BB" + mp.group(1))
        if _HEADER.search(raw) and cur is not None and cur.startswith(".LBB"):
            parents["BB" + cur[4:]] = chain[-1] if chain else None
    return parents


def _ancestors(h, parents):
    out = []
    while h is not None:
        out.append(h)
        h = parents.get(h)
    return out


def divergent_barrier_loops(asm: str, symbol: str) -> list[str]:
    """Loops of `symbol` that contain a barrier and have an EXEC-mask latch."""
    blocks = kernel_blocks(asm, symbol)
    parents = loop_parents(asm, symbol)
    # loops containing a barrier (the innermost loop of the barrier's block and its ancestors)
    with_barrier = set()
    for b in blocks:
        if b.loop and any(i.startswith("s_barrier") for i in b.instructions()):
            with_barrier.update(_ancestors(b.loop, parents))
    bad = []
    for h in sorted(with_barrier):
        body = {b.name for b in blocks if b.loop and h in _ancestors(b.loop, parents)}
        for k, b in enumerate(blocks):
            if b.name not in body:
                continue
            ins = b.instructions()
            targets = [m.group(2) for m in (_BRANCH.match(i) for i in ins) if m]
            jumps_back = ("BB" + t == h for t in targets)
            falls_into = (k + 1 < len(blocks) and blocks[k + 1].name == h and
                          not (ins and ins[-1].startswith("s_branch")))
            if not (any(jumps_back) or falls_into):
                continue
            # the latch decides on EXEC when it narrows EXEC and then tests it
            tail = ins[-4:]
            if any(i.startswith(("s_andn2_b64 exec, exec", "s_and_b64 exec, exec")) for i in tail) and \
                    any(i.startswith(("s_cbranch_execz", "s_cbranch_execnz")) for i in tail):
                bad.append(f"{h} (latch {b.name}: {' / '.join(tail)})")
    return bad


def kernel_symbols(asm: str, prefix: str) -> list[str]:
    return sorted({m.group(1) for m in re.finditer(r"^(" + re.escape(prefix) + r"\w*):", asm, re.M)})
