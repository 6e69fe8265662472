"""GPU test of the carry hand-off inside the fused carry-and-classification
kernel (Eq. 4 across runs; section Projecting Cells to 1D): with the wait
bound at 0 every classifying workgroup computes its requests' carries itself
instead of reading them from the scan workgroups, and every output must be
bitwise the same as with the default bounded wait, for a single update and
for a batch whose classifying workgroups span several requests."""
import numpy as np
import pytest
import torch

from gpu_cases import dvl, random_amr, tfs

pytestmark = pytest.mark.gpu

KEYS = ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


def _same(a, b, label):
    for k in KEYS:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        assert x.tobytes() == y.tobytes(), f"{label}: {k} differs"


def _runs(D, fn):
    """fn() with the default wait, then with every workgroup computing the carry."""
    try:
        D.set_carry_wait(D.CARRY_WAIT_DEFAULT)
        ref = fn()
        D.set_carry_wait(0)
        got = fn()
    finally:
        D.set_carry_wait(D.CARRY_WAIT_DEFAULT)
    return ref, got


def test_carry_fallback_single_update():
    import synth
    D = dvl()
    vol = synth.make_amr(16, (0.4, 0.3, 0.2), 4, 81, octaves=3, field_octaves=2).to("cuda")
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    try:
        A = tfs(81, V.m)
        for m in range(V.m):
            V.set_tf(m, A[m])
        for kw in (dict(), dict(scan_mode=1), dict(exponent=2.0, min_importance=0.0)):
            def run():
                b = D.Bins(1920, V.m)
                V.update(b, **kw)
                return V.read_bins(b)
            ref, got = _runs(D, run)
            print(f"[carry] single update {kw}: n={V.n}", flush=True)
            _same(got, ref, f"single {kw}")
    finally:
        V.close()


def test_carry_fallback_batch():
    D = dvl()
    vols = [random_amr(90 + i, 6, 3, 0.4, n_fields=4) for i in range(5)]
    Vs = []
    for v in vols:
        d = v.to("cuda")
        Vs.append(D.build_order(d.x, d.y, d.z, d.level, list(d.fields)))
    try:
        specs = [(i % len(Vs), 10 + i, W) for i, W in enumerate((1920, 64, 777, 3840, 1, 300, 2048))]
        reqs = [D.Request(Vs[vi], tfs(seed, Vs[vi].m), D.Bins(W, Vs[vi].m)) for vi, seed, W in specs]
        ex = D.Executor()
        try:
            def run():
                ex.update_batch(reqs)
                torch.cuda.synchronize()
                return [r.vol.read_bins(r.bins) for r in reqs]
            ref, got = _runs(D, run)
            print(f"[carry] batch of {len(reqs)} requests on {len(Vs)} volumes", flush=True)
            for i in range(len(reqs)):
                _same(got[i], ref[i], f"request {i}")
        finally:
            ex.close()
    finally:
        for V in Vs:
            V.close()
