"""GPU tests of batched updates (dvl_update_batch) and captured batches
(dvl_graph_*): every request's outputs must be bitwise equal to the same
update run alone through dvl_update, whatever else shares the launch, and
one request of each batch is also reconciled against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import dvl, random_amr, tfs

pytestmark = pytest.mark.gpu

KEYS = ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


def _build(vol, dtype=torch.float32, **opt):
    D = dvl()
    dev = vol.to("cuda")
    return D.build_order(dev.x, dev.y, dev.z, dev.level, [f.to(dtype) for f in dev.fields], **opt)


def _alone(V, alpha, W, lo=None, hi=None, **kw):
    """The same request through dvl_update on the volume's own TF state."""
    D = dvl()
    for m in range(V.m):
        if lo is None:
            V.set_tf(m, alpha[m])
        else:
            D.set_tf(V, m, alpha[m], float(lo[m]), float(hi[m]))
    b = D.Bins(W, V.m)
    V.update(b, **kw)
    return V.read_bins(b)


def _same(a, b, label):
    for k in KEYS:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        assert x.dtype == y.dtype and x.shape == y.shape and x.tobytes() == y.tobytes(), f"{label}: {k} differs"


def _vols():
    import synth
    v1 = synth.make_amr(16, (0.4, 0.3, 0.2), 4, 71, octaves=3, field_octaves=2)
    v2 = random_amr(72, 8, 3, 0.4, n_fields=4)
    v3 = random_amr(73, 6, 4, 0.5, n_fields=4)
    return v1, v2, v3


def _oracle_check(V, vol, alpha, W, **kw):
    from parity import reconcile, to_np
    _, perm_t = V.export_order()
    perm = perm_t.cpu().numpy().view(np.uint32)
    F = np.stack([to_np(f)[perm] for f in vol.fields]).astype(np.float32)
    lo, hi = oracle.default_windows(F)
    for m in range(F.shape[0]):
        if not hi[m] > lo[m]:
            hi[m] = np.nextafter(lo[m], np.float32(np.inf))
    return F, lo, hi, perm


def test_batch_alone_vs_mix():
    """Three volumes, seven requests with different TFs, widths, exponents
    and max(V) modes in one batch; each equals its update alone."""
    D = dvl()
    vols = _vols()
    Vs = [_build(v) for v in vols]
    try:
        specs = [  # (volume, tf seed, W, kwargs)
            (0, 1, 1920, dict()),
            (0, 2, 64, dict(exponent=2.0)),
            (1, 3, 777, dict(vmax_mode=2)),
            (0, 4, 3840, dict(exponent=0.5, min_importance=0.1)),
            (2, 5, 1, dict()),
            (1, 6, 300, dict(level_scale=3, clamp_mode=1)),
            (2, 7, 2048, dict(scan_mode=1, vmax_mode=1)),
        ]
        reqs = []
        for vi, seed, W, kw in specs:
            A = tfs(seed, Vs[vi].m)
            reqs.append(D.Request(Vs[vi], A, D.Bins(W, Vs[vi].m), **kw))
        print(f"[batch] {len(reqs)} requests on {len(Vs)} volumes", flush=True)
        ex = D.Executor()
        try:
            ex.update_batch(reqs)
            torch.cuda.synchronize()
            got = [r.vol.read_bins(r.bins) for r in reqs]
            for i, (vi, seed, W, kw) in enumerate(specs):
                ref = _alone(Vs[vi], reqs[i].alpha, W, **kw)
                _same(got[i], ref, f"request {i}")
            # and the first request against the oracle
            from parity import reconcile
            F, lo, hi, perm = _oracle_check(Vs[0], vols[0], reqs[0].alpha, 1920)
            ob = oracle.update(vols[0].level.numpy()[perm], F, reqs[0].alpha, lo, hi, 1920, keep_cells=True)
            reconcile(got[0], ob, F, reqs[0].alpha, lo, hi, 1920)
        finally:
            ex.close()
    finally:
        for V in Vs:
            V.close()


def test_batch_mixed_field_counts():
    """Volumes with 1, 2, 3 and 4 fields in one batch (the general kernel
    variant): each request equals its update alone."""
    D = dvl()
    vols = [random_amr(60 + m, 6, 3, 0.4, n_fields=m) for m in (1, 2, 3, 4)]
    Vs = [_build(v) for v in vols]
    ex = D.Executor()
    try:
        reqs = [D.Request(V, tfs(200 + i, V.m), D.Bins(333 + 100 * i, V.m), exponent=1.5)
                for i, V in enumerate(Vs)]
        ex.update_batch(reqs)
        for i, r in enumerate(reqs):
            _same(r.vol.read_bins(r.bins), _alone(r.vol, r.alpha, r.bins.n_bins, exponent=1.5), f"M={r.vol.m}")
    finally:
        ex.close()
        for V in Vs:
            V.close()


def test_batch_more_requests_than_a_job_holds():
    """Eleven requests on one volume: split into jobs of at most eight that
    share the volume's reads; each equals its update alone."""
    D = dvl()
    vol = random_amr(81, 8, 3, 0.4, n_fields=3)
    V = _build(vol)
    try:
        reqs = [D.Request(V, tfs(100 + i, 3), D.Bins(100 + 37 * i, 3), exponent=1.0 + (i % 3))
                for i in range(11)]
        ex = D.Executor()
        try:
            ex.update_batch(reqs)
            got = [V.read_bins(r.bins) for r in reqs]
            for i, r in enumerate(reqs):
                _same(got[i], _alone(V, r.alpha, r.bins.n_bins, exponent=1.0 + (i % 3)), f"request {i}")
        finally:
            ex.close()
    finally:
        V.close()


def test_batch_explicit_windows_and_reuse():
    """Explicit windows, and the executor reused for a second, different
    batch (workspaces grown and reused)."""
    D = dvl()
    vols = _vols()
    Vs = [_build(v) for v in vols]
    ex = D.Executor()
    try:
        lo = np.array([0.5, 0.2, 0.1, 0.0], np.float32)
        hi = np.array([3.0, 2.0, 5.0, 1.0], np.float32)
        r1 = [D.Request(Vs[1], tfs(9, 4), D.Bins(500, 4), lo=lo, hi=hi)]
        ex.update_batch(r1)
        g1 = Vs[1].read_bins(r1[0].bins)
        _same(g1, _alone(Vs[1], r1[0].alpha, 500, lo=lo, hi=hi), "explicit windows")
        r2 = [D.Request(Vs[i], tfs(20 + i, 4), D.Bins(1024, 4)) for i in (2, 0, 1)]
        ex.update_batch(r2)
        for i, r in enumerate(r2):
            _same(r.vol.read_bins(r.bins), _alone(r.vol, r.alpha, 1024), f"second batch {i}")
        assert ex.nbytes > 0
    finally:
        ex.close()
        for V in Vs:
            V.close()


def test_graph_replays_follow_tf_changes():
    """A captured batch replayed with new TFs between launches, with other
    device work in between: every replay equals the eager batch."""
    D = dvl()
    vols = _vols()
    Vs = [_build(v) for v in vols]
    try:
        reqs = [D.Request(Vs[0], tfs(31, 4), D.Bins(1920, 4)),
                D.Request(Vs[1], tfs(32, 4), D.Bins(256, 4), exponent=2.0),
                D.Request(Vs[0], tfs(33, 4), D.Bins(48, 4), vmax_mode=2),
                D.Request(Vs[2], tfs(34, 4), D.Bins(999, 4))]
        g = D.Graph(reqs)
        ex = D.Executor()
        try:
            for rep in range(4):
                if rep:
                    new = [tfs(1000 * rep + i, 4) for i in range(len(reqs))]
                    for r, A in zip(reqs, new):
                        r.alpha = np.ascontiguousarray(A)
                    if rep % 2:
                        g.set_tf_all(new)                    # one call for every request
                    else:
                        for i, A in enumerate(new):
                            g.set_tf(i, A)
                print(f"[graph] replay {rep}", flush=True)
                g.launch()
                junk = torch.randn(1 << 20, device="cuda").cumsum(0)     # unrelated eager work
                torch.cuda.synchronize()
                got = [r.vol.read_bins(r.bins) for r in reqs]
                eager = [D.Request(r.vol, r.alpha, D.Bins(r.bins.n_bins, 4), **kw)
                         for r, kw in zip(reqs, (dict(), dict(exponent=2.0), dict(vmax_mode=2), dict()))]
                ex.update_batch(eager)
                torch.cuda.synchronize()
                for i, (a, e) in enumerate(zip(got, eager)):
                    _same(a, e.vol.read_bins(e.bins), f"replay {rep} request {i}")
                del junk
        finally:
            ex.close()
            g.close()
    finally:
        for V in Vs:
            V.close()


@pytest.mark.parametrize("tile_steps,run_waves", [(8, 0), (32, 0), (16, 64), (8, 5000)])
def test_build_options_parity(tile_steps, run_waves):
    """Other tile sizes and run counts: same oracle parity."""
    import synth
    from parity import reconcile
    vol = synth.make_amr(16, (0.4, 0.3, 0.2), 4, 91, octaves=3, field_octaves=2)
    V = _build(vol, tile_steps=tile_steps, run_waves=run_waves)
    try:
        A = tfs(91, 4)
        F, lo, hi, perm = _oracle_check(V, vol, A, 1920)
        for W in (1920, 16):
            g = _alone(V, A, W, exponent=2.0)
            ob = oracle.update(vol.level.numpy()[perm], F, A, lo, hi, W, 2.0, keep_cells=True)
            reconcile(g, ob, F, A, lo, hi, W)
    finally:
        V.close()


def test_batch_errors():
    D = dvl()
    vol = random_amr(95, 4, 2, n_fields=2)
    V32 = _build(vol)
    V16 = _build(vol, dtype=torch.float16)
    ex = D.Executor()
    try:
        r = [D.Request(V32, tfs(1, 2), D.Bins(16, 2)), D.Request(V16, tfs(2, 2), D.Bins(16, 2))]
        with pytest.raises(D.DvlError) as e:
            ex.update_batch(r)
        assert e.value.status == 1 and "mixes" in str(e.value)
        with pytest.raises(D.DvlError) as e:
            ex.update_batch([D.Request(V32, tfs(1, 2), D.Bins(16, 2), exponent=-1.0)])
        assert e.value.status == 1 and "request 0" in str(e.value)
        with pytest.raises(D.DvlError) as e:
            ex.update_batch([D.Request(V32, tfs(1, 2), D.Bins(16, 2), lo=[1.0, 1.0], hi=[1.0, 2.0])])
        assert e.value.status == 1
        with pytest.raises(D.DvlError) as e:
            D.build_order(*[t.cuda() for t in (vol.x, vol.y, vol.z, vol.level)], [f.cuda() for f in vol.fields],
                          tile_steps=12)
        assert e.value.status == 1
    finally:
        ex.close()
        V32.close()
        V16.close()
