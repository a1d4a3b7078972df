"""What the trained network gains: a reduced-size run of the learned-start pipeline.

Family A(theta) = A0 + sum_k theta_k B_k at n = 32 (8 parameters), network 8 -> 256 -> 256 -> 32^2,
trained on 4096 solves of the batched FP64 path, evaluated on 24 held-out parameters.  Asserted:
every solve (learned start with fallback, learned start always accepted, FP32 start, plain) meets
the acceptance bar; training lowers the loss; the trained network's start is closer to diagonal
than both the untrained network's and no start at all (A itself), and started from it Jacobi needs
no more sweeps than plain Jacobi.  The comparison with the FP32 start is printed, not asserted:
how far a learned start gets is what this run measures.
"""
import json

import numpy as np
import pytest
import torch

from paper_2211_03339_amd import jacobi
from paper_2211_03339_amd import learned
from paper_2211_03339_amd import testmats as tm

pytestmark = pytest.mark.gpu


def test_learned_start_gain_small_family():
    n, hidden = 32, 256
    A0, B = learned.family(n)
    th_train = tm.param_thetas(4096, learned.THETA_TRAIN_SEED)
    th_eval = tm.param_thetas(24, learned.THETA_EVAL_SEED)
    print("[learned] data", flush=True)
    theta, T, data = learned.make_dataset(A0, B, th_train)
    assert data["unconverged"] == 0
    net = jacobi.Mlp(8, hidden, n, 256, seed=3)
    before = learned.evaluate(net, A0, B, th_eval, check=False, forced=False)
    print("[learned] train", flush=True)
    tr = learned.train(net, theta, T, epochs=40, batch=256, lr=2e-3, weight_decay=1e-4)
    print("[learned] eval", flush=True)
    ev = learned.evaluate(net, A0, B, th_eval)
    print(json.dumps({"data": data, "loss": tr["loss_per_epoch"][::8] + tr["loss_per_epoch"][-1:],
                      "before": before["learned_start"], "after": ev}), flush=True)
    assert tr["loss_per_epoch"][-1] < 0.5 * tr["loss_per_epoch"][0]
    for m in ("mlp", "mlp_forced", "fp32", "plain"):
        assert ev[m]["max_res"] <= 1e-13, (m, ev[m])
        assert ev[m]["max_orth"] <= 1e-13, (m, ev[m])
    ls = ev["learned_start"]
    assert ls["mean_start_resid"] < before["learned_start"]["mean_start_resid"]
    assert ls["mean_start_resid"] < ls["mean_identity_start_resid"]
    assert ev["mlp_forced"]["mean_sweeps"] <= ev["plain"]["mean_sweeps"]
    net.close()
