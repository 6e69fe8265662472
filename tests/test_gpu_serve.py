"""Serving on the GPU: requests answered by continuous batching over two
launch slots match the FP64 oracle (reconciled at the parity tolerances) and
equal the same requests run alone (bitwise); the run really batched (several
requests per launch, requests on one volume sharing a launch) and really
overlapped (both slots busy at once)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import dvl, random_amr
from parity import reconcile

pytestmark = pytest.mark.gpu

KEYS = ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


def test_served_results_match_oracle_and_alone():
    import synth
    from paper_2306_11612_amd.serve import GpuEngine, Scheduler, make_requests, run_open_loop
    D = dvl()
    vols = {"a": synth.make_amr(16, (0.4, 0.3, 0.2), 4, 501, octaves=3, field_octaves=2),
            "b": random_amr(502, 8, 3, 0.4, n_fields=4),
            "c": random_amr(503, 12, 2, 0.3, n_fields=4)}
    Vs, sorted_inputs = {}, {}
    for k, v in vols.items():
        d = v.to("cuda")
        Vs[k] = D.build_order(d.x, d.y, d.z, d.level, d.fields)
        _, perm = Vs[k].export_order()
        p = perm.cpu().numpy().view(np.uint32)
        F = np.stack([f.numpy()[p] for f in v.fields]).astype(np.float32)
        sorted_inputs[k] = (v.level.numpy()[p], F, *oracle.default_windows(F))
    eng = GpuEngine(Vs, n_slots=2)
    try:
        jobs = make_requests(sorted(Vs), {k: V.m for k, V in Vs.items()}, rate=5000.0, duration=0.01,
                             max_requests=60, seed=synth.SEED + 77, widths=(64, 1024, 1920), tf_pool=8)
        sched = Scheduler(eng, budget_bytes=1 << 30, max_batch=16, keep_outputs=True)
        res = run_open_loop(sched, jobs)
        print(f"[serve] {res}", flush=True)
        assert res["requests"] == len(jobs)
        assert res["mean_batch"] > 1.0, "no request was batched with another"
        assert res["max_requests_on_one_volume"] > 1, "no launch shared a volume's reads"
        assert res["max_running_slots"] == 2, "the two launch slots never ran at once"
        torch.cuda.synchronize()
        moved = 0
        for j in sched.completed:
            V = Vs[j.volume]
            got = V.read_bins(j.out)
            # what the client received: the pinned host copy made on the slot's stream
            h = j.out.host
            assert np.array_equal(h.first.numpy().view(np.uint32), got["first"])
            assert np.array_equal(h.last.numpy().view(np.uint32), got["last"])
            for k, key in enumerate(("mean", "vmin", "vmax", "y")):
                assert h.stats[k].numpy().tobytes() == got[key].tobytes(), key
            # the FP64 oracle on the same sorted inputs, TFs and width
            lev, F, lo, hi = sorted_inputs[j.volume]
            ob = oracle.update(lev, F, j.alpha, lo, hi, j.n_bins, keep_cells=True)
            rep = reconcile(got, ob, F, j.alpha, lo, hi, j.n_bins)
            assert abs(got["f_total"] - ob.f_total) <= 1e-5 * ob.f_total
            moved += rep.edges_moved
            # the same request alone
            for m in range(V.m):
                V.set_tf(m, j.alpha[m])
            b = D.Bins(j.n_bins, V.m)
            V.update(b)
            ref = V.read_bins(b)
            for key in KEYS:
                x, y = np.asarray(got[key]), np.asarray(ref[key])
                assert x.tobytes() == y.tobytes(), f"request {j.rid} ({j.volume}, W={j.n_bins}): {key}"
        print(f"[serve] {len(sched.completed)} results reconciled with the oracle; edges moved {moved}",
              flush=True)
        eng.release(sched.completed)
    finally:
        eng.close()
        for V in Vs.values():
            V.close()
