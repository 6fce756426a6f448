"""Build-time check of the gfx950 assembly of every kernel for one-sided
register copies in divergent control flow.

The structurized form of a per-lane if/else in AMDGPU code is

    s_and_saveexec_b64 S, cond   ; EXEC <- then-lanes
    s_xor_b64 S, exec, S         ; S    <- else-lanes
    ...then part...
  FLOW:
    ...flow part...              ; still under the then-lanes' EXEC
    s_or_saveexec_b64 D, S       ; (or s_andn2_saveexec_b64)
    s_xor_b64 exec, exec, D      ; EXEC <- else-lanes
    ...else part...
  END:
    s_or_b64 exec, exec, D       ; EXEC <- both

A copy made in the flow part reaches the then-lanes only.  When it copies a
value that the then part did not compute (a value live into the if/else,
defined for every lane), the else part does not write the destination, and
the destination is read after END, the else-lanes read whatever that
register (or spill slot) held before: a stale value from an earlier wave or
kernel.  The register allocator of the toolchain has been seen to place the
copies of a live-range split (moves into AGPRs, spill stores) exactly there
in the large boundary kernels; the results were wrong velocities, wrong
states and, when the stale value formed a store address, memory faults.

check(paths) scans assembly files and returns the offending copies;
main() exits non-zero when there are any.  The scan is linear over each
kernel's text and recognises the patterns above; it is a guard against that
miscompilation, not a general verifier.
"""
from __future__ import annotations

import re
import sys

_LABEL = re.compile(r'^(\.LBB\w+|; %bb\.\d+):')
_STORES = ('global_store', 'scratch_store', 'buffer_store', 'flat_store', 'ds_write', 'ds_store')


def _regs(tok: str) -> set:
    tok = tok.strip()
    m = re.match(r'^([va])\[(\d+):(\d+)\]$', tok)
    if m:
        return {'%s%d' % (m.group(1), r) for r in range(int(m.group(2)), int(m.group(3)) + 1)}
    if re.match(r'^[va]\d+$', tok):
        return {tok}
    return set()


def _is_code(t: str) -> bool:
    return bool(t) and not t.startswith((';', '.')) and not t.endswith(':')


def _dests(t: str) -> set:
    """Vector or accumulation registers an instruction writes."""
    if not _is_code(t):
        return set()
    op = t.split()[0]
    if op.startswith(_STORES) or op.startswith(('s_', 'v_cmp_', 'v_readlane', 'v_readfirstlane')):
        return set()
    return _regs(t[len(op):].split(',')[0])


def _sources(t: str) -> set:
    if not _is_code(t):
        return set()
    op = t.split()[0]
    if op.startswith('s_'):
        return set()
    parts = [x.strip() for x in t[len(op):].split(',')]
    cand = parts if op.startswith(_STORES) else parts[1:]
    out = set()
    for c in cand:
        c = c.split()[0] if c else c
        out |= _regs(c.lstrip('-|').rstrip('|'))
    return out


def _copy(t: str):
    """(destination, source registers) of a copy: a move into an AGPR, a
    register move, or a spill store."""
    m = re.match(r'v_accvgpr_write_b32 (a\d+), (v\d+)$', t)
    if m:
        return m.group(1), {m.group(2)}
    m = re.match(r'v_mov_b(?:32|64)_e(?:32|64) (v\S+), (v\S+)$', t)
    if m:
        return m.group(1), _regs(m.group(2))
    m = re.match(r'scratch_store_dword\w* off, (v[^,\s]+), off(?: offset:(\d+))?', t)
    if m:
        return 'scratch+%s' % (m.group(2) or '0'), _regs(m.group(1))
    return None


def _read_after(lines, k, dest) -> bool:
    """Is the first access of dest after line k (in layout order) a read?"""
    if dest.startswith('scratch+'):
        off = dest.split('+')[1]
        for t in lines[k + 1:]:
            if t.startswith('s_endpgm'):
                return False
            m = (re.match(r'scratch_(load|store)_dword\w* [^;]*?off, off(?: offset:(\d+))?', t)
                 or re.match(r'scratch_(load|store)_dword\w* off, [^,]+, off(?: offset:(\d+))?', t))
            if m and (m.group(2) or '0') == off:
                return m.group(1) == 'load'
        return False
    regs = _regs(dest)
    for t in lines[k + 1:]:
        if t.startswith('s_endpgm'):
            return False
        if not _is_code(t):
            continue
        if regs & _sources(t):
            return True
        if regs & _dests(t):
            return False
    return False


def _kernels(text: str):
    src = text.split('\n')
    heads = [(i, l.split(':')[0]) for i, l in enumerate(src) if re.match(r'^_Z\w+:', l)]
    for n, (s, name) in enumerate(heads):
        e = heads[n + 1][0] if n + 1 < len(heads) else len(src)
        yield name, [l.strip() for l in src[s:e]]


def check_kernel(L: list) -> list:
    found = []
    for i, t in enumerate(L):
        m = re.match(r's_(?:or|andn2)_saveexec_b64 (s\[\d+:\d+\]), (s\[\d+:\d+\])', t)
        if not m:
            continue
        D, S = m.group(1), m.group(2)
        j = i - 1
        while j >= 0 and not re.match(r's_and_saveexec_b64 ' + re.escape(S) + ',', L[j]):
            j -= 1
        if j < 0 or any(L[q].startswith('s_endpgm') for q in range(j, i)):
            continue
        f = i
        while f > j and not _LABEL.match(L[f]):
            f -= 1
        k = i + 1
        while k < len(L) and not re.match(r's_or_b64 exec, exec, ' + re.escape(D) + '$', L[k]):
            k += 1
        else_writes = set()
        for q in range(i + 1, k):
            c = _copy(L[q])
            if c:
                else_writes.add(c[0])
            else_writes |= _dests(L[q])
        for p in range(f, i):
            c = _copy(L[p])
            if not c:
                continue
            dest, srcs = c
            written = set()
            for q in range(j + 1, p):
                written |= _dests(L[q])
            if not srcs - written:
                continue  # a value of the then part
            dregs = _regs(dest) or {dest}
            later = set()
            for q in range(p + 1, i):
                later |= _dests(L[q])
            if dregs & later:
                continue  # overwritten before the join
            if dregs <= else_writes:
                continue  # the else part writes it too
            if _read_after(L, k, dest):
                found.append((p, L[p]))
    return found


def check(paths) -> list:
    bad = []
    for path in paths:
        with open(path) as fh:
            text = fh.read()
        for name, L in _kernels(text):
            for line, ins in check_kernel(L):
                bad.append((path, name, ins))
    return bad


def main(argv=None) -> int:
    paths = (argv if argv is not None else sys.argv[1:])
    bad = check(paths)
    for path, name, ins in bad:
        print('%s: %s: one-sided copy in a divergent flow block: %s' % (path, name, ins))
    print('%d kernel file(s) checked, %d one-sided copies' % (len(paths), len(bad)))
    return 1 if bad else 0


if __name__ == '__main__':
    sys.exit(main())
