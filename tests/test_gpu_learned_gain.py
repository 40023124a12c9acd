"""What the trained network gains over the plain criterion (GPU, about 15 s).

The held-out evaluation case (wind seed 0, the 1500 km/s cone CME aimed at
the sample point), relaxed 14 days on the stretched base grid, then 1.5 days
with 5 levels and regrids every 10 steps: plain criterion with the buffer
against learned flags (the shipped network at its stored threshold, judged
by the plain criterion every 10th regrid) without the buffer.  The learned
run must reach the same shock arrival at (1 AU, 90 deg, 0 deg) within
0.25 h with fewer leaf-block-steps.
"""
import os

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_learned_flags_cost_less_at_equal_arrival():
    from paper_2211_12867_amd import IC_SOURCE_LEARNED_JUDGED, IC_SOURCE_PLAIN, forecast as F
    net, meta = F.load_network(os.path.join(HERE, "..", "paper_2211_12867_amd", "flags_net.npz"))
    grid, wind, cme, amr, _ = F._workload_parts("learned_flags", max_level=5)
    cme = dict(cme, t_start_s=14 * F.DAY)
    st = F.relax(grid, wind, cme, 14 * F.DAY, chunk_s=7 * F.DAY, log=None)
    t_end = 15.5 * F.DAY
    plain = F.cme_run(grid, wind, cme, dict(amr, source=IC_SOURCE_PLAIN, buffer_blocks=1), st, t_end,
                      chunk_s=F.DAY / 2, log=None)
    learned = F.cme_run(grid, wind, cme, dict(amr, source=IC_SOURCE_LEARNED_JUDGED, buffer_blocks=0,
                                               learned_threshold=meta["threshold"]), st, t_end, network=net,
                        chunk_s=F.DAY / 2, log=None)
    print("plain+buffer: arrival %.3f h, %d leaf-block-steps; learned: arrival %.3f h, %d leaf-block-steps, %s"
          % (plain["arrival_h"], plain["leaf_block_steps"], learned["arrival_h"], learned["leaf_block_steps"],
             learned["regrid_stats"]))
    assert plain["arrival_h"] == plain["arrival_h"], "no arrival within the run"
    assert abs(learned["arrival_h"] - plain["arrival_h"]) <= 0.25
    assert learned["leaf_block_steps"] < plain["leaf_block_steps"]
    assert learned["regrid_stats"]["learned"] > 0 and learned["regrid_stats"]["judged"] > 0
