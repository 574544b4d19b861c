"""A simulated device for testing the serving logic on the CPU.

Counts come from the CPU oracle (so results are exact); the time a batch
takes is simulated as the sum of per-query costs (cost_fn) scaled to
seconds, and a query whose cost exceeds its deadline is reported as DNF.
Live device memory is tracked so tests can check that admission never
over-commits it."""
import threading
import time


class FakeGraph:
    def __init__(self, row_ptr, col, nbytes):
        self.row_ptr = row_ptr
        self.col = col
        self.n = len(row_ptr) - 1
        self.nbytes = nbytes


class FakeBackend:
    def __init__(self, oracle, cost_fn, seconds_per_cost=1e-3, pool_bytes=0, mem_limit=None,
                 estimate_fn=None, pivot_cost_fn=None):
        self.oracle = oracle
        self.pivot_cost_fn = pivot_cost_fn
        self.pivot_calls = []
        if estimate_fn is not None:
            self.estimate = estimate_fn
        self.cost_fn = cost_fn
        self.scale = seconds_per_cost
        self.lock = threading.Lock()
        self.live = pool_bytes
        self.peak = pool_bytes
        self.mem_limit = mem_limit
        self.active = 0
        self.max_active = 0
        self.calls = []

    def orient(self, row_ptr, col, slot):
        from paper_2502_00317_amd.serve import oriented_bytes
        b = oriented_bytes(len(row_ptr) - 1, len(col) // 2)
        with self.lock:
            self.live += b
            self.peak = max(self.peak, self.live)
            if self.mem_limit is not None:
                assert self.live <= self.mem_limit, "device memory over-committed"
        return FakeGraph(row_ptr, col, b)

    def free(self, g):
        with self.lock:
            self.live -= g.nbytes

    def count_all(self, slot, g, kmax, budget_ms):
        """Every k <= kmax in one simulated pass of pivot_cost_fn(g, kmax)."""
        c = self.pivot_cost_fn(g, kmax)
        self.pivot_calls.append((slot, g.n, kmax))
        if budget_ms and c * self.scale * 1e3 > budget_ms:
            time.sleep(budget_ms / 1e3)
            return None, "dnf"
        res = [(0, 0)] + [self.oracle.count(g.row_ptr, g.col, k, nthreads=1) for k in range(1, kmax + 1)]
        time.sleep(c * self.scale)
        return res, "ok"

    def count_one(self, slot, g, k, budget_ms):
        res, st, _ = self.count_batch(slot, [g], [k], [budget_ms])
        return res[0], st[0]

    def count_batch(self, slot, graphs, ks, deadlines_ms, on_done=None, costs=None):
        """Runs the pairs one after another, cheapest first; with on_done
        each pair is reported as soon as its simulated time has passed.  A
        pair's budget runs from its own start."""
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.calls.append((slot, len(graphs), time.perf_counter()))
        n = len(graphs)
        res, st = [None] * n, [None] * n
        costs = [self.cost_fn(g, k) for g, k in zip(graphs, ks)]
        total = 0.0
        for i in sorted(range(n), key=lambda i: costs[i]):
            g, k, dl, c = graphs[i], ks[i], deadlines_ms[i], costs[i]
            if dl and c * self.scale * 1e3 > dl:
                res[i], st[i] = (0, 0), "dnf"
                dt = dl / 1e3
            else:
                cnt, fp = self.oracle.count(g.row_ptr, g.col, k, nthreads=1)
                res[i], st[i] = (cnt, fp), ("overflow" if cnt >= 1 << 64 else "ok")
                dt = c * self.scale
            total += dt
            if on_done is not None:
                time.sleep(dt)
                on_done(i, res[i][0], res[i][1], st[i], dt * 1e3)
        if on_done is None:
            time.sleep(total)
        with self.lock:
            self.active -= 1
        return res, st, total * 1e3
