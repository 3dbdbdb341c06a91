// Copy counts behind the waits of the Legendre kernels' LDS pipelines.
//
// Every stage of the analysis and synthesis kernels starts by waiting until
// at most n global->LDS copies of the wave are still in flight (the copies
// complete in issue order), then a workgroup barrier.  The counts below are
// the largest n for which everything the stage reads has landed.  Plain
// constexpr C++ with no HIP dependency: tests/test_stage_waits.py compiles
// it on the host and checks every count against a simulation of each wave's
// copy queue.
//
// The pipelines: stage g's copies go into LDS buffer g % (D + 1) and are
// issued D stages ahead, at stage g - D (the prologue plays stages -D .. -1).
#pragma once

namespace sht {
namespace waits {

// Analysis: global stages g < xs bring the wave's K slice of S or A (four
// copies each), stage xs + s is table stage s (lpw copies each).  Behind the
// copies of stage gs come those of stages gs+1 .. gs+d-1.
constexpr int analysis_behind(int xs, int lpw, int d, int gs) {
  int n = 0;
  for (int i = 1; i < d; ++i) n += (gs + i < xs) ? 4 : lpw;
  return n;
}

// Synthesis: a row block takes `parts` stages; the stage at part 1 also
// issues the nb spectrum copies of the next row block (the block's B
// operands, read at its part 0).  Those go before the stage's table copies
// when a row block has two parts (part 0, the very next stage, then waits
// for all but one stage's copies instead of all of them), after them
// otherwise (the gathered spectrum then does not hold up the table copies).
constexpr bool spec_first(int parts) { return parts == 2; }

// Copies synthesis stage s may leave in flight.  Behind its table copies
// (issued at stage s-d) come the table copies of stages s+1 .. s+d-1 and
// the spectrum copies issued at part 1 by stages s-d+1 .. s-1, and by stage
// s-d too when they follow its table copies.  A stage at part 0 also needs
// the spectrum copies issued at part 1 of the previous row block; only the
// table copies of the parts-2 stages after that one, and of that stage
// itself when the spectrum went first, follow them.  (When no prologue stage
// is at part 1, row block 0's spectrum is issued before everything.)
constexpr int synthesis_behind(int parts, int lpw, int d, int nb, int s) {
  const bool sf = spec_first(parts);
  int n = (d - 1) * lpw;
  for (int j = sf ? s - d + 1 : s - d; j < s; ++j)
    if (((j % parts) + parts) % parts == 1) n += nb;
  const int ns = (sf ? parts - 1 : parts - 2) * lpw;
  if (s % parts == 0 && ns < n) n = ns;
  return n;
}

}  // namespace waits
}  // namespace sht
