"""The batched form at the size the benchmark times: 4096 random networks
(M log-uniform on [3, 2048], N = M / 4, 64 trajectories each), the networks
above 512 channels in the lazy form, the others with the autotuned plan, the
benchmark's firing cap -- one captured launch.

Checks: per class, trajectories of items spread over the class's queue are
recomputed by the oracle (lazy items by its lazy form) and must match bit for
bit; Eq. 5 (X_final = x0 + sum_k n_k v_k) on every one of the 262,144
trajectories; the launch's firing count equals the sum of n; every OK or
ABSORBED trajectory's last sample (at t_end) equals its final state.
"""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from paper_2103_00405_amd import workloads as W

pytestmark = pytest.mark.gpu


def _nu_dense(spec):
    """Net change v_k (Eq. 5) of every reaction, [M][N], from the CSR lists."""
    nu = np.zeros((spec.M, spec.N), np.int64)
    rp, pp = np.asarray(spec.react_ptr), np.asarray(spec.prod_ptr)
    rows_r = np.repeat(np.arange(spec.M), np.diff(rp))
    rows_p = np.repeat(np.arange(spec.M), np.diff(pp))
    np.subtract.at(nu, (rows_r, np.asarray(spec.react_species)), np.asarray(spec.react_sigma))
    np.add.at(nu, (rows_p, np.asarray(spec.prod_species)), np.asarray(spec.prod_mult))
    return nu


def _np(t):
    return t.cpu().numpy()


def test_full_batch_configuration_against_oracle():
    import bench
    from paper_2103_00405_amd import api
    wl = W.batch_networks(4096)
    jobs = bench.batch_jobs(api, wl)
    want = ("samples", "n", "T", "x_final", "status", "tie_step")
    cap = bench.BATCH_MAX_FIRINGS
    b0 = api.Batch(jobs, want=want, max_firings=cap)
    with tempfile.TemporaryDirectory() as d:
        plan = os.path.join(d, "plan.txt")
        api.autotune(b0, plan, samples=16)
        del b0
        b = api.Batch(jobs, want=want, max_firings=cap, plan_path=plan)
    st = b.run(seed=1)
    torch.cuda.synchronize()
    classes = b.classes()
    print("classes:", [(c["mapping"], c["lanes"], c["items"]) for c in classes], flush=True)
    assert len(classes) >= 6
    assert any(c["mapping"] == api.MAP_WAVE and c["lanes"] == 64 and c["max_M"] > 512
               for c in classes)                      # the lazy class

    # Eq. 5 and the firing count on every trajectory
    total = 0
    for w, o in zip(wl, b.outputs):
        n = _np(o["n"]).view(np.uint32).astype(np.int64)
        total += int(n.sum())
        pred = w.x0.astype(np.int64)[None, :] + n @ _nu_dense(w.net)
        assert np.array_equal(pred, _np(o["x_final"]).astype(np.int64)), w.net_id
        good = o["status"] <= 1
        assert torch.equal(o["samples"][good][:, -1, :], o["x_final"][good]), w.net_id
    assert st["firings"] == total

    # per class: four items spread over the queue, two trajectories each
    checked = 0
    for ci, c in enumerate(classes):
        members = b.class_items(ci)
        picks = sorted({members[0], members[len(members) // 3], members[(2 * len(members)) // 3],
                        members[-1]})
        for i in picks:
            w, j, o = wl[i], jobs[i], b.outputs[i]
            lazy = j["method"] == api.METHOD_LAZY
            for r in (0, 41):
                ref = oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, 1, 1, net_id=w.net_id,
                                      traj_offset=r, max_firings=cap, lazy=lazy)
                sl = slice(r, r + 1)
                assert np.array_equal(_np(o["samples"][sl]), ref["samples"]), (i, r)
                assert np.array_equal(_np(o["n"][sl]).view(np.uint32), ref["n"]), (i, r)
                assert np.array_equal(_np(o["T"][sl]).view(np.uint64),
                                      ref["T"].view(np.uint64)), (i, r)
                assert np.array_equal(_np(o["x_final"][sl]), ref["x_final"]), (i, r)
                assert np.array_equal(_np(o["status"][sl]), ref["status"]), (i, r)
                assert np.array_equal(_np(o["tie_step"][sl]).view(np.uint32),
                                      ref["tie_step"]), (i, r)
                checked += 1
    assert checked >= 2 * 4 * len(classes) - 8        # small classes may repeat an item
