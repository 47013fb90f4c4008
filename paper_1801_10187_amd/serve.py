"""Serving many independent SRD simulations on one GPU.

A `Server` runs requests (a box, its particles, a step count) concurrently:
each admitted request gets its own context and HIP stream, so the kernels of
requests in flight overlap on the device. Requests are admitted in arrival
order (first in, first out) as soon as a worker thread is free and the
device memory their contexts need fits in the budget beside the requests
already running; a request larger than the whole budget runs alone. The
result of a request is its cell-averaged velocity field, and it is the same
bit for bit whether the request ran alone or among others: every context has
its own random-number key (its seed) and its own memory.
"""
import collections
import concurrent.futures
import threading

from . import binding

def footprint(n_particles, n_cells, precision=binding.FP32, steps=1):
    """Device bytes a request's context takes at its peak (mpcd_footprint:
    the library's own allocation rules, host arrays uploaded and the
    velocity field read back)."""
    peak, _ = binding.footprint(n_cells, n_particles, nsteps=steps, precision=precision,
                                host_arrays=True)
    return peak


class Request:
    """One simulation: `make()` returns its (pos, vel) arrays (called in the
    worker, so particle generation overlaps other requests' GPU work); the
    keyword arguments go to `Sim` (seed, kT, thermostat, ...)."""

    def __init__(self, n_cells, n_particles, steps, make, precision=binding.FP32, **sim_kw):
        self.n_cells = tuple(int(x) for x in n_cells)
        self.n_particles = int(n_particles)
        self.steps = int(steps)
        self.make = make
        self.precision = precision
        self.sim_kw = sim_kw
        self.bytes = footprint(self.n_particles, self.n_cells, precision, self.steps)


def run_request(req):
    """Run one request in a context of its own: create, step, read the
    cell-averaged velocity field (u, mass), destroy."""
    pos, vel = req.make()
    sim = binding.Sim(pos, vel, req.n_cells, precision=req.precision, **req.sim_kw)
    try:
        sim.step(req.steps)
        return sim.velocity_field()
    finally:
        sim.close()


class Server:
    """FIFO admission of requests by worker slot and device-memory budget.

    workers        requests in flight at most (one host thread each)
    memory_budget  device bytes the requests in flight may hold together
                   (default: 90 % of the device memory free at start)
    runner         function running one request (default `run_request`)
    """

    def __init__(self, workers=8, memory_budget=None, runner=run_request):
        if memory_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            memory_budget = int(0.9 * free)
        self.budget = int(memory_budget)
        self.runner = runner
        self._queue = collections.deque()
        self._cv = threading.Condition()
        self._inflight_bytes = 0
        self._inflight = 0
        self._closed = False
        self.max_inflight_bytes = 0
        self.max_inflight = 0
        self.admitted = []          # request order of admission
        self._threads = [threading.Thread(target=self._work, daemon=True) for _ in range(workers)]
        for t in self._threads:
            t.start()

    def submit(self, req):
        fut = concurrent.futures.Future()
        with self._cv:
            if self._closed:
                raise RuntimeError("server is closed")
            self._queue.append((req, fut))
            self._cv.notify_all()
        return fut

    def _fits(self, req):
        return self._inflight == 0 or self._inflight_bytes + req.bytes <= self.budget

    def _work(self):
        while True:
            with self._cv:
                while not (self._closed and not self._queue) and \
                        not (self._queue and self._fits(self._queue[0][0])):
                    self._cv.wait()
                if not self._queue:
                    return
                req, fut = self._queue.popleft()
                self._inflight += 1
                self._inflight_bytes += req.bytes
                self.max_inflight = max(self.max_inflight, self._inflight)
                self.max_inflight_bytes = max(self.max_inflight_bytes, self._inflight_bytes)
                self.admitted.append(req)
            try:
                if fut.set_running_or_notify_cancel():
                    fut.set_result(self.runner(req))
            except BaseException as e:  # the caller sees the request's own error
                fut.set_exception(e)
            finally:
                with self._cv:
                    self._inflight -= 1
                    self._inflight_bytes -= req.bytes
                    self._cv.notify_all()

    def close(self):
        """Serve what is queued, then stop the workers."""
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
