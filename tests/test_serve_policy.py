"""Admission and batching policy of the server, with the GPU launch and
completion replaced by a fake (CPU)."""
import collections

import pytest


class FakeSlot:
    def __init__(self):
        self.batch = None
        self.event = self
        self.ticks = 0

    def query(self):
        self.ticks -= 1
        return self.ticks <= 0


def make_server(slots=2, max_batch=3):
    from paper_2006_00816_amd import serve
    srv = serve.HogServer.__new__(serve.HogServer)
    srv.max_batch, srv.cap, srv.thresh, srv.iou = max_batch, 4, 0.0, 0.5
    srv.slots = [FakeSlot() for _ in range(slots)]
    srv.pending = collections.OrderedDict(((240, 320), collections.deque()) for _ in range(1))
    srv.pending[(480, 640)] = collections.deque()
    srv.completed = []
    srv.batches = 0
    srv.limit = {}
    launched = []

    def launch(slot, reqs):
        slot.batch = reqs
        slot.ticks = 2
        srv.batches += 1
        launched.append([r.rid for r in reqs])

    srv._launch = launch
    return srv, launched


def test_batches_by_resolution_oldest_first_and_never_drops(monkeypatch):
    pytest.importorskip("torch")
    from paper_2006_00816_amd import serve
    import numpy as np
    srv, launched = make_server()
    # completion copies results from pinned buffers; fake them
    for s in srv.slots:
        s.h_n = np.zeros(16, np.int32)
        s.h_dets = __import__("torch").zeros((16, 4, 10), dtype=__import__("torch").int32)
    shapes = [(240, 320), (480, 640), (240, 320), (240, 320), (480, 640), (240, 320), (240, 320), (240, 320)]
    for i, s in enumerate(shapes):
        srv.submit(serve.Request(i, s, None, float(i)))
    t = [0.0]

    def now():
        t[0] += 1.0
        return t[0]

    for _ in range(50):
        srv.pump(now)
    # first slot: oldest resolution first (rid 0 is 240x320), up to 3 frames of it
    assert launched[0] == [0, 2, 3]
    assert launched[1] == [1, 4]
    assert sorted(r.rid for r in srv.completed) == list(range(len(shapes)))
    assert all(len(b) <= 3 for b in launched)
    for b in launched:
        assert len({shapes[i] for i in b}) == 1


def test_admission_by_batch_bytes(monkeypatch):
    """A batch takes only as many frames of its resolution as the slab's
    bytes hold (the per-resolution limit), the rest wait for the next slot."""
    pytest.importorskip("torch")
    from paper_2006_00816_amd import serve
    import numpy as np
    srv, launched = make_server(slots=2, max_batch=3)
    srv.limit = {(240, 320): 3, (480, 640): 1}
    for s in srv.slots:
        s.h_n = np.zeros(16, np.int32)
        s.h_dets = __import__("torch").zeros((16, 4, 10), dtype=__import__("torch").int32)
    shapes = [(480, 640)] * 3 + [(240, 320)] * 4
    for i, s in enumerate(shapes):
        srv.submit(serve.Request(i, s, None, float(i)))
    t = [0.0]

    def now():
        t[0] += 1.0
        return t[0]

    for _ in range(50):
        srv.pump(now)
    assert sorted(r.rid for r in srv.completed) == list(range(len(shapes)))
    for b in launched:
        assert len(b) <= (1 if shapes[b[0]] == (480, 640) else 3)
    assert [b for b in launched if shapes[b[0]] == (480, 640)] == [[0], [1], [2]]


def test_batch_limits_follow_workspace_bytes():
    """The limits come from hog_workspace_bytes: a 64 MiB slab holds 16
    frames of 320x240, 10 of 640x480 and 3 of 1280x720 with 5 filters."""
    from paper_2006_00816_amd import serve
    lim = {s: serve.batch_limit(*s, 5, 64 << 20, 16) for s in ((240, 320), (480, 640), (720, 1280))}
    assert lim == {(240, 320): 16, (480, 640): 10, (720, 1280): 3}
    for (h, w), n in lim.items():
        assert serve.batch_bytes(h, w, n, 5) <= 64 << 20
        if n < 16:
            assert serve.batch_bytes(h, w, n + 1, 5) > 64 << 20

