"""CPU oracle for the virtual-rank collectives (ring / double-binary-tree
AllReduce, ring ReduceScatter, AllGather, Broadcast and Reduce).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The library itself
never calls it, and it shares no code with the library: it re-derives the
channel partition, the ring and tree topologies and every step of every
schedule from the paper's description, in plain numpy, slowly and visibly.

What it computes (each module cites the passage it follows):

* ``elementwise``  -- the reduction operators per element type (int32 wrap,
  IEEE fp32 add, bf16 add as fp32 add then round-to-nearest-even, max with
  a fixed +0/-0 rule).
* ``partition``    -- channel regions (workOffset / channelCount), outer
  loops and elementary-step chunks (Section V-C, Fig. 3).
* ``topology``     -- ring successor/predecessor and the double binary tree
  (Section II-C).
* ``simulate``     -- each rank's primitive sequence per loop iteration
  (Tables of Section V-E) executed against explicit bounded FIFOs, one per
  connection; detects deadlock; returns outputs and a step trace.
* ``definitions``  -- the plain mathematical definitions of the five
  collectives (brute force) and an fp64 reference with its error bound.
* ``protocol``     -- LL and LL128 line formats and slot geometry (Section III).
* ``folds``        -- closed-form association order of every float sum the
  schedules produce, derived independently of the simulator.

Pins: see tests/test_oracle_*.py (brute force, closed forms, the paper's
step tables and buffer geometry under tests/golden/, library conversions).
"""
from . import elementwise, partition, topology, simulate, definitions, folds, protocol  # noqa: F401
