"""Serving on the GPU: requests answered by continuous batching over two
launch slots equal the same requests run alone (bitwise)."""
import numpy as np
import pytest
import torch

from gpu_cases import dvl, random_amr

pytestmark = pytest.mark.gpu

KEYS = ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


def test_served_results_equal_alone():
    import synth
    from paper_2306_11612_amd.serve import GpuEngine, Scheduler, make_requests, run_open_loop
    D = dvl()
    vols = {"a": synth.make_amr(16, (0.4, 0.3, 0.2), 4, 501, octaves=3, field_octaves=2),
            "b": random_amr(502, 8, 3, 0.4, n_fields=4),
            "c": random_amr(503, 12, 2, 0.3, n_fields=4)}
    Vs = {}
    for k, v in vols.items():
        d = v.to("cuda")
        Vs[k] = D.build_order(d.x, d.y, d.z, d.level, d.fields)
    eng = GpuEngine(Vs, n_slots=2)
    try:
        jobs = make_requests(sorted(Vs), {k: V.m for k, V in Vs.items()}, rate=5000.0, duration=0.01,
                             max_requests=60, seed=synth.SEED + 77, widths=(64, 1024, 1920), tf_pool=8)
        sched = Scheduler(eng, budget_bytes=1 << 30, max_batch=16, keep_outputs=True)
        res = run_open_loop(sched, jobs)
        print(f"[serve] {res}", flush=True)
        assert res["requests"] == len(jobs)
        torch.cuda.synchronize()
        for j in sched.completed:
            V = Vs[j.volume]
            got = V.read_bins(j.out)
            for m in range(V.m):
                V.set_tf(m, j.alpha[m])
            b = D.Bins(j.n_bins, V.m)
            V.update(b)
            ref = V.read_bins(b)
            for key in KEYS:
                x, y = np.asarray(got[key]), np.asarray(ref[key])
                assert x.tobytes() == y.tobytes(), f"request {j.rid} ({j.volume}, W={j.n_bins}): {key}"
        eng.release(sched.completed)
    finally:
        eng.close()
        for V in Vs.values():
            V.close()
