"""GPU test of one volume updated from two streams in turn (dvl_update,
Eqs. 1-4 and section Projecting Cells to 1D): its executor's descriptor
block and workspace are shared by both streams and its TF entry cache is
built on one stream and read on the other, so each launch must wait for the
previous one on the other stream.  Every output must be bitwise the same as
the same update run alone on the default stream."""
import numpy as np
import pytest
import torch

from gpu_cases import dvl, tfs

pytestmark = pytest.mark.gpu

KEYS = ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


def test_update_alternating_streams():
    import synth
    D = dvl()
    vol = synth.make_amr(16, (0.4, 0.3, 0.2), 4, 83, octaves=3, field_octaves=2).to("cuda")
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    try:
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        # (TF seed, W, parameters); the windows stay the data ranges, so the
        # entry cache is built on the second update and read from then on
        specs = [(1, 1920, {}), (2, 1920, {}), (3, 64, dict(exponent=2.0)), (4, 3840, {}),
                 (5, 777, dict(scan_mode=1)), (6, 1920, {}), (7, 1, {}), (8, 2048, dict(min_importance=0.1))]
        outs = []
        for i, (seed, W, kw) in enumerate(specs):
            A = tfs(seed, V.m)
            for m in range(V.m):
                V.set_tf(m, A[m])
            b = D.Bins(W, V.m)
            V.update(b, stream=streams[i % 2], **kw)
            outs.append(b)
        torch.cuda.synchronize()
        got = [V.read_bins(b) for b in outs]
        print(f"[streams] {len(specs)} updates on 2 streams, n={V.n}, cache={V.entry_cache_info() is not None}",
              flush=True)
        for i, (seed, W, kw) in enumerate(specs):
            A = tfs(seed, V.m)
            for m in range(V.m):
                V.set_tf(m, A[m])
            b = D.Bins(W, V.m)
            V.update(b, **kw)
            ref = V.read_bins(b)
            for k in KEYS:
                assert np.asarray(got[i][k]).tobytes() == np.asarray(ref[k]).tobytes(), f"update {i}: {k} differs"
    finally:
        V.close()
