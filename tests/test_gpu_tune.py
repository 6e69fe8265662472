"""The layout autotuner on the GPU: it measures candidate layouts of a small
volume, caches the winner for the shape class, and a volume built with the
tuned layout reconciles against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import dvl, tfs
from parity import reconcile

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


def test_tune_then_build_tuned_matches_oracle(tmp_path, monkeypatch):
    import synth
    from paper_2306_11612_amd import tune
    monkeypatch.setenv("DVL_TUNE_CACHE", str(tmp_path / "tune.json"))
    D = dvl()
    vol = synth.make_amr(16, (0.4, 0.3, 0.2), 4, 921, octaves=3, field_octaves=2)
    d = vol.to("cuda")
    W = 1920
    res = tune.tune(d.x, d.y, d.z, d.level, d.fields, W, candidates=[(16, 0), (8, 0), (32, 16)], steps=2)
    assert len(res["all"]) == 3 and all(r["ms"] > 0 for r in res["all"])
    assert res["ms"] == min(r["ms"] for r in res["all"])
    lay = tune.best_layout(d.x, d.y, d.z, d.level, d.fields, W)       # tunes the full list, then caches
    assert tune._load()[tune.shape_key(vol.n, vol.m, torch.float32, W)] == lay
    V = tune.build_tuned(d.x, d.y, d.z, d.level, d.fields, W)
    try:
        A = tfs(921, vol.m)
        _, perm = V.export_order()
        p = perm.cpu().numpy().view(np.uint32)
        F = np.stack([f.numpy()[p] for f in vol.fields]).astype(np.float32)
        lo, hi = oracle.default_windows(F)
        for m in range(vol.m):
            D.set_tf(V, m, A[m], float(lo[m]), float(hi[m]))
        b = D.Bins(W, vol.m)
        V.update(b)
        g = V.read_bins(b)
        ob = oracle.update(vol.level.numpy()[p], F, A, lo, hi, W, keep_cells=True)
        rep = reconcile(g, ob, F, A, lo, hi, W)
        print(f"[tune] layout {lay}: edges moved {rep.edges_moved}", flush=True)
    finally:
        V.close()
