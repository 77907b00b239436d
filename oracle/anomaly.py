"""Attack candidates read off the factor R (the online detection of the
paper's application section, Section 5, "CTD at work").

TEST INFRASTRUCTURE ONLY, like the rest of this package: only tests/, the
package smoke check and the CPU baseline leg of the benchmark may use it.

R holds actual mode-alpha fibers, so each kept fiber names its coordinates
in the other modes (for a source x destination x time traffic tensor
decomposed along the source mode: a destination host and a time step).  The
readout, in the order of the paper's description:
  1. kept fibers with the same coordinate in the grouping mode (the
     destination) stand for the same major activity;
  2. the first such fiber in R, in order of acceptance, represents it;
  3. the representatives whose norm ||x_f|| is above the average over all
     representatives are the candidates.

Readings: "the first fiber" is the earliest accepted one (R grows by
appending, so this is also the earliest in time for CTD-D); "above the
average" is strict; the average is the arithmetic mean of the norms (not of
the squared norms).
"""
from __future__ import annotations

import math


def group_coordinate(fid: int, dims, mode: int, group_mode: int) -> int:
    """Coordinate in `group_mode` of the mode-`mode` fiber with column index
    `fid` (column-major over the other modes in increasing order).  The last
    of the other modes is not reduced modulo its length, so that fibers of a
    stream, whose time index grows past the initial length, decode too."""
    if group_mode == mode:
        raise ValueError("the grouping mode must differ from the decomposition mode")
    others = [m for m in range(len(dims)) if m != mode]
    stride = 1
    for m in others:
        if m == group_mode:
            q = fid // stride
            return q if m == others[-1] else q % int(dims[m])
        stride *= int(dims[m])
    raise ValueError("group_mode out of range")


def attack_candidates(accepted, norms, dims, mode, group_mode):
    """Steps 1-3 above.

    accepted: fiber ids of R in order of acceptance; norms: ||x_f|| of each.
    Returns (candidates, representatives, mean): positions into `accepted`
    (ascending) and the mean norm of the representatives.
    """
    first = {}
    for a, f in enumerate(accepted):
        g = group_coordinate(int(f), dims, mode, group_mode)
        if g not in first:
            first[g] = a
    reps = sorted(first.values())
    if not reps:
        return [], [], 0.0
    mean = math.fsum(float(norms[a]) for a in reps) / len(reps)
    cands = [a for a in reps if float(norms[a]) > mean]
    return cands, reps, mean
