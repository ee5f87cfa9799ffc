"""A stand-in for the serving executor: every query is answered by the CPU
oracle, BFS sessions advance one level per step exactly as the device sessions
do (a query's alive bit is set while its BFS reaches new vertices), and jobs
finish after a fixed number of scheduler rounds.  Used with a fake clock to
test the scheduler's admission, batching and cancellation on the CPU."""
import numpy as np

import oracle as orc

UNR = 0xFFFFFFFF


class FakeClock:
    """Returns `now`; each reading also advances it by `tick` (0: time stands
    still unless slept)."""

    def __init__(self, tick=0.0):
        self.now = 0.0
        self.tick = tick

    def __call__(self):
        t = self.now
        self.now += self.tick
        return t

    def sleep(self, dt):
        self.now += max(dt, 0.0)


class _Session:
    def __init__(self, g):
        self.g = g
        self.steps = 0
        self.slots = {}   # slot -> (levels, step at join)
        self.alive = 0
        self.steps_with = []  # number of busy slots at each step


class _Future:
    def __init__(self, fn, ticks):
        self.fn, self.left, self.value = fn, ticks, None

    def done(self):
        self.left -= 1
        return self.left <= 0

    def result(self):
        if self.value is None:
            self.value = self.fn()
        return self.value


class FakeExecutor:
    def __init__(self, graphs, job_ticks=3, session_bytes=None):
        self.graphs = graphs
        self.job_ticks = job_ticks
        self._sess_bytes = session_bytes
        self.opened = self.closed = 0
        self.sessions = []
        self.jobs_run = []

    def graph_n(self, g):
        return self.graphs[g].n

    def session_bytes(self, g):
        return self._sess_bytes if self._sess_bytes is not None else 280 * self.graphs[g].n + 1024

    def job_bytes(self, kind, g):
        return 0 if kind == "tc" else 12 * self.graphs[g].n

    def result_bytes(self, kind, g):
        return 8 if kind == "tc" else 4 * self.graphs[g].n

    def open_session(self, g):
        self.opened += 1
        s = _Session(g)
        self.sessions.append(s)
        return s

    def join(self, h, slot, source):
        assert slot not in h.slots
        h.slots[slot] = (orc.bfs(self.graphs[h.g], source), h.steps)

    def step(self, h):
        h.steps += 1
        h.steps_with.append(len(h.slots))
        h.alive = 0
        for slot, (lv, start) in h.slots.items():
            if np.any(lv == h.steps - start):
                h.alive |= 1 << slot

    def ready(self, h):
        return True

    def alive(self, h):
        return h.alive

    def extract(self, h, slot):
        lv, _ = h.slots.pop(slot)
        return lv

    def token_ready(self, token):
        return True

    def token_result(self, token):
        return token

    def cancel(self, h, slot):
        h.slots.pop(slot)

    def close_session(self, h):
        assert not h.slots
        self.closed += 1

    def submit(self, kind, g, source):
        self.jobs_run.append((kind, g, source))
        G = self.graphs[g]
        fn = {"sssp": lambda: orc.sssp_unit(G, source), "cc": lambda: orc.cc(G), "tc": lambda: orc.tc(G)}[kind]
        return _Future(fn, self.job_ticks)
