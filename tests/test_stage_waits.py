"""Wait counts of the Legendre kernels' LDS pipelines (csrc/stage_waits.h).

Each stage of the analysis and synthesis kernels waits until at most n of
the wave's global->LDS copies are in flight, then meets the workgroup at a
barrier; the copies complete in issue order.  If n is too large, a stage
reads LDS that its copies have not filled yet.  That is a race the parity
tests would only catch by chance.  This test compiles stage_waits.h on the
host (it has no HIP dependency) and checks every count against a
simulation of one wave's copy queue.  The simulation replays the issue
order the kernels follow: the prologue, then every stage's copies D stages
ahead, plus the synthesis spectrum copies at part 1 of each row block.  It
covers the geometries the kernels instantiate and a wider sweep around
them.  A count above the simulated one is a race; the counts must also
equal the simulated ones, so no stage waits for more than it needs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_12144_amd", "csrc")

PARTS = (2, 3, 4, 6, 8, 12)
LPWS = (1, 2, 3, 4, 6, 8)
DEPTHS = (2, 3, 4)
NBS = (4, 8)
XSS = (0, 1, 2, 3, 4, 6)
STAGES = 48

CHECKER = r"""
#include <cstdio>
#include "stage_waits.h"
using namespace sht::waits;
int main() {
  const int parts[] = {%(parts)s}, lpws[] = {%(lpws)s}, ds[] = {%(ds)s}, nbs[] = {%(nbs)s}, xss[] = {%(xss)s};
  for (int p : parts) for (int l : lpws) for (int d : ds) for (int nb : nbs)
    for (int s = 0; s < %(st)d; ++s) std::printf("S %%d %%d %%d %%d %%d %%d %%d\n", p, l, d, nb, s, synthesis_behind(p, l, d, nb, s), spec_first(p) ? 1 : 0);
  for (int x : xss) for (int l : lpws) for (int d : ds)
    for (int g = 0; g < %(st)d; ++g) std::printf("A %%d %%d %%d %%d %%d\n", x, l, d, g, analysis_behind(x, l, d, g));
  return 0;
}
"""


def _values(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "waits.cpp"
    src.write_text(CHECKER % dict(parts=", ".join(map(str, PARTS)), lpws=", ".join(map(str, LPWS)),
                                  ds=", ".join(map(str, DEPTHS)), nbs=", ".join(map(str, NBS)),
                                  xss=", ".join(map(str, XSS)), st=STAGES))
    exe = tmp_path / "waits"
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    syn, ana = {}, {}
    for line in out.splitlines():
        f = line.split()
        if f[0] == "S":
            p, l, d, nb, s, n, sf = map(int, f[1:])
            syn[(p, l, d, nb, s)] = (n, bool(sf))
        else:
            x, l, d, g, n = map(int, f[1:])
            ana[(x, l, d, g)] = n
    return syn, ana


def _allowed(queue, need):
    """Copies issued after the last one of `need`: how many may stay in flight."""
    last = max(i for i, c in enumerate(queue) if c in need)
    return len(queue) - 1 - last


def simulate_synthesis(parts, lpw, d, nb, spec_first, stages):
    """Per stage: copies in flight the stage may leave (tables of stage s, and
    at part 0 the spectrum of its row block, complete)."""
    q = []

    def issue(v):  # stage v: table copies of stage v + d, spectrum at part 1
        at1 = v % parts == 1
        blk = v // parts + 1
        if spec_first and at1:
            q.extend([("s", blk)] * nb)
        q.extend([("t", v + d)] * lpw)
        if not spec_first and at1:
            q.extend([("s", blk)] * nb)

    if parts > d + 1:  # no prologue stage at part 1: row block 0 goes first
        q.extend([("s", 0)] * nb)
    for v in range(-d, 0):
        issue(v)
    out = []
    for s in range(stages):
        need = {("t", s)} | ({("s", s // parts)} if s % parts == 0 else set())
        out.append(_allowed(q, need))
        issue(s)
    return out


def simulate_analysis(xs, lpw, d, stages):
    q = []

    def issue(g):  # four copies of S / A per stage g < xs, lpw of table
        q.extend([g] * (4 if g < xs else lpw))

    for g in range(d):
        issue(g)
    out = []
    for g in range(stages):
        out.append(_allowed(q, {g}))
        issue(g + d)
    return out


def test_synthesis_waits_match_copy_queue(tmp_path):
    syn, _ = _values(tmp_path)
    for p in PARTS:
        for l in LPWS:
            for d in DEPTHS:
                for nb in NBS:
                    sf = syn[(p, l, d, nb, 0)][1]
                    assert sf == (p == 2)
                    sim = simulate_synthesis(p, l, d, nb, sf, STAGES)
                    got = [syn[(p, l, d, nb, s)][0] for s in range(STAGES)]
                    assert got == sim, (p, l, d, nb, got, sim)


def test_analysis_waits_match_copy_queue(tmp_path):
    _, ana = _values(tmp_path)
    for x in XSS:
        for l in LPWS:
            for d in DEPTHS:
                sim = simulate_analysis(x, l, d, STAGES)
                got = [ana[(x, l, d, g)] for g in range(STAGES)]
                assert got == sim, (x, l, d, got, sim)


def test_simulation_catches_a_wrong_order():
    """The simulation is not vacuous: with the spectrum copies issued after
    the table copies in a two-part row block, part 0 would have to wait for
    everything (no copy may stay in flight)."""
    sim = simulate_synthesis(2, 2, 2, 4, False, 8)
    assert sim[2] == 0 and sim[4] == 0
    assert simulate_synthesis(2, 2, 2, 4, True, 8)[2] == 2
