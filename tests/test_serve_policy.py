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
