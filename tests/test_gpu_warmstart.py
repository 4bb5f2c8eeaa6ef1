"""What the trained surrogate gains over the plain method: the network is trained on the
GPU (BF16 matrix cores) from the stored periodic states of the training draws (seeds 1,
3 to 9) that the batched PIC produced, then two held-out seed-2 discharges run from a uniform start (the
plain method) and from the predicted state, side by side in one batch.  Both must reach
the steady-state criterion; the warm start in at most half the RF periods, and its final
profiles within 3 % of the cold start's (the cold PIC run decides the error)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import log
from paper_1608_04601_amd import warmstart as WS

pytestmark = pytest.mark.gpu

HELD_OUT = [6, 15]   # positions in the seed-2 draw of 16


def test_warm_start_reaches_the_periodic_state_in_fewer_periods():
    data = WS.load_data()
    keep = WS.training_mask(data)
    net, norm, loss = WS.train(data["params"][keep], data["profiles"][keep], steps=4000)
    log(f"surrogate trained on {keep.sum()} periodic states: loss {loss:.3e}")
    params = W.surrogate_params(16, 2)[HELD_OUT]
    rows = WS.evaluate(net, norm, params, 2, 400, log=log, index=HELD_OUT)
    for r in rows:
        log(f"  {r['params']}: cold {r['cold_steady_at']} periods, warm {r['warm_steady_at']}, "
            f"warm vs cold {max(r['warm_vs_cold']):.3f}, prediction vs cold {max(r['prediction_vs_cold']):.3f}")
        assert not r["extinct"]
        assert r["cold_steady_at"] is not None and r["warm_steady_at"] is not None
        assert 2 * r["warm_steady_at"] <= r["cold_steady_at"]
        assert max(r["warm_vs_cold"]) <= 0.03
    net.close()
