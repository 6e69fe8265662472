"""The C ABI's memory and data-change contract on the GPU: device memory
through a caller's allocator (PyTorch's caching allocator from Python), no
leak when an allocation fails at any point, and a rejected data change that
leaves the volume as it was."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import dvl, random_amr, tfs
from parity import reconcile

pytestmark = pytest.mark.gpu

KEYS = ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


class Counting:
    """Allocator over PyTorch's caching allocator that records every block
    and refuses the allocation with index `fail_at` (and every later one)."""

    def __init__(self, fail_at=None):
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}
        D = dvl()
        self.allocator = D.Allocator(self._alloc, self._release)

    def _alloc(self, nbytes, stream):
        k = self.calls
        self.calls += 1
        if self.fail_at is not None and k >= self.fail_at:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes)
        self.live[p] = nbytes
        return p

    def _release(self, ptr, stream):
        assert ptr in self.live, f"release of a pointer the allocator never gave out: {ptr:#x}"
        del self.live[ptr]
        torch.cuda.caching_allocator_delete(ptr)


def _update(V, alpha, W, **kw):
    D = dvl()
    for m in range(V.m):
        V.set_tf(m, alpha[m])
    b = D.Bins(W, V.m)
    V.update(b, **kw)
    return V.read_bins(b)


def test_torch_allocator_holds_the_volume_and_gives_it_back():
    D = dvl()
    vol = random_amr(31, 6, 3, 0.4, n_fields=4).to("cuda")
    A = tfs(31, 4)
    ref = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    try:
        want = _update(ref, A, 96)
    finally:
        ref.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    alloc = D.torch_allocator()
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields, allocator=alloc)
    try:
        held = torch.cuda.memory_allocated() - before
        assert held >= V.nbytes > 0, (held, V.nbytes)
        got = _update(V, A, 96)
        for k in KEYS:
            assert np.asarray(got[k]).tobytes() == np.asarray(want[k]).tobytes(), k
    finally:
        V.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_failed_allocation_at_every_point_leaks_nothing():
    D = dvl()
    vol = random_amr(32, 4, 3, 0.4, n_fields=3).to("cuda")
    probe = Counting()
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields, allocator=probe.allocator)
    V.close()
    total = probe.calls
    assert total >= 10 and not probe.live
    for k in range(total):
        c = Counting(fail_at=k)
        with pytest.raises(D.DvlError) as e:
            D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields, allocator=c.allocator)
        assert e.value.status == D.E_NOMEM, (k, e.value)
        assert not c.live, f"allocation {k} failing left {len(c.live)} blocks behind"


def test_update_workspace_growth_failure_is_not_sticky():
    """An update whose workspace cannot grow fails with DVL_E_NOMEM and the
    volume keeps working for updates that fit."""
    D = dvl()
    vol = random_amr(33, 16, 3, 0.4, n_fields=4)     # about 50 k cells, 13 tiles
    dev = vol.to("cuda")
    c = Counting()
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields, allocator=c.allocator, entry_cache=2)
    try:
        A = tfs(33, 4)
        for _ in range(4):             # every descriptor slot of the volume's executor in use once
            _update(V, A, 2)
        c.fail_at = c.calls            # nothing more may be allocated
        for m in range(4):
            V.set_tf(m, A[m])
        big = D.Bins(4096, 4)          # dense bins: the update also stores f (4 B per cell)
        with pytest.raises(D.DvlError) as e:
            V.update(big)
        assert e.value.status == D.E_NOMEM
        g = _update(V, A, 2)           # fits the workspace made at build time
        _, perm = V.export_order()
        p = perm.cpu().numpy().view(np.uint32)
        F = np.stack([f.numpy()[p] for f in vol.fields])
        lo, hi = oracle.default_windows(F)
        ob = oracle.update(vol.level.numpy()[p], F, A, lo, hi, 2, keep_cells=True)
        reconcile(g, ob, F, A, lo, hi, 2)
    finally:
        V.close()
    assert not c.live


def test_executor_allocator():
    D = dvl()
    vol = random_amr(34, 6, 3, 0.4, n_fields=4).to("cuda")
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    c = Counting()
    ex = D.Executor(allocator=c.allocator)
    try:
        A = tfs(34, 4)
        alone = _update(V, A, 200)
        r = D.Request(V, A, D.Bins(200, 4))
        ex.update_batch([r])
        assert c.live and ex.nbytes == sum(c.live.values())
        got = V.read_bins(r.bins)
        for k in KEYS:
            assert np.asarray(got[k]).tobytes() == np.asarray(alone[k]).tobytes(), k
    finally:
        ex.close()
        V.close()
    assert not c.live


def test_set_field_with_nan_leaves_the_volume_unchanged():
    D = dvl()
    vol = random_amr(35, 6, 3, 0.4, n_fields=3)
    dev = vol.to("cuda")
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields)
    try:
        A = tfs(35, 3)
        before = _update(V, A, 64)
        ranges = [V.field_range(m) for m in range(3)]
        bad = dev.fields[1] * 2.0
        bad[vol.n // 2] = float("nan")
        with pytest.raises(D.DvlError) as e:
            V.set_field(1, bad)
        assert e.value.status == D.E_RANGE
        assert [V.field_range(m) for m in range(3)] == ranges
        after = _update(V, A, 64)      # the volume is not in a failed state
        for k in KEYS:
            assert np.asarray(after[k]).tobytes() == np.asarray(before[k]).tobytes(), k
        lv, fs = V.export_sorted()
        _, perm = V.export_order()
        p = perm.cpu().numpy().view(np.uint32)
        assert np.array_equal(fs[1].cpu().numpy(), vol.fields[1].numpy()[p])
    finally:
        V.close()
