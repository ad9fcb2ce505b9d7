"""Comparison helpers shared by the GPU parity tests, smoke() and the bench:
the acceptance metric (max error normalised to the peak oracle power), the
paper's rRMSE, and the tie-aware top-k rule."""
from __future__ import annotations

import heapq

import numpy as np

FP32_TOL = 1e-4      # max |P_gpu - P_ref| / max P_ref for the float32 path
MIXED_TOL = 2e-3     # the same for the 16-bit plans (FP16 storage)
TOPK = 16


class PlaneStats:
    """Streams row blocks of (gpu, oracle) power and accumulates the metrics."""

    def __init__(self, k: int = TOPK):
        self.k = k
        self.max_abs = 0.0
        self.max_ref = 0.0
        self.sq_err = 0.0
        self.sq_ref = 0.0
        self.gpu_heap = []    # min-heap of (P, -t, -i) keeping the k largest
        self.ref_heap = []
        self.gpu_vals = {}    # (t, i) -> gpu power of candidates
        self.ref_rows = {}    # (t, i) -> oracle power of candidates

    def _push(self, heap, vals, rows_t, block):
        k = self.k
        flat = block.reshape(-1)
        if flat.size == 0:
            return
        take = min(k, flat.size)
        idx = np.argpartition(flat, flat.size - take)[flat.size - take:]
        # include every cell tied with the smallest kept value
        thr = flat[idx].min()
        idx = np.nonzero(flat >= thr)[0]
        n = block.shape[1]
        for c in idx.tolist():
            t, i = rows_t[c // n], c % n
            item = (float(flat[c]), -int(t), -int(i))
            if len(heap) < k:
                heapq.heappush(heap, item)
            elif item > heap[0]:
                heapq.heapreplace(heap, item)

    def add(self, rows_t, gpu_block, ref_block):
        gpu_block = np.asarray(gpu_block, dtype=np.float64)
        ref_block = np.asarray(ref_block, dtype=np.float64)
        d = np.abs(gpu_block - ref_block)
        self.max_abs = max(self.max_abs, float(d.max()) if d.size else 0.0)
        self.max_ref = max(self.max_ref, float(ref_block.max()) if ref_block.size else 0.0)
        self.sq_err += float(np.sum(d * d))
        self.sq_ref += float(np.sum(ref_block * ref_block))
        rows_t = list(rows_t)
        self._push(self.gpu_heap, None, rows_t, gpu_block)
        self._push(self.ref_heap, None, rows_t, ref_block)
        # remember both powers of every cell that is (or was) a candidate on either side
        n = gpu_block.shape[1]
        for heap in (self.gpu_heap, self.ref_heap):
            for _, mt, mi in heap:
                t, i = -mt, -mi
                if t in rows_t:
                    r = rows_t.index(t)
                    self.gpu_vals[(t, i)] = float(gpu_block[r, i])
                    self.ref_rows[(t, i)] = float(ref_block[r, i])
        del n

    @property
    def norm_err(self) -> float:
        return self.max_abs / self.max_ref if self.max_ref > 0 else self.max_abs

    @property
    def rrmse(self) -> float:
        return float(np.sqrt(self.sq_err / self.sq_ref)) if self.sq_ref > 0 else 0.0

    def topk(self, which: str):
        heap = self.gpu_heap if which == "gpu" else self.ref_heap
        return [(-mt, -mi, p) for p, mt, mi in sorted(heap, reverse=True)]

    def topk_agree(self, tol: float = FP32_TOL):
        """Top-k sets equal, except cells whose oracle power lies within
        tol * max(P_ref) of the oracle's k-th value may swap."""
        ref = self.topk("ref")
        gpu = self.topk("gpu")
        if not ref:
            return True, []
        kth = ref[-1][2]
        slack = tol * self.max_ref
        ref_set = {(t, i) for t, i, _ in ref}
        gpu_set = {(t, i) for t, i, _ in gpu}
        bad = []
        for c in gpu_set - ref_set:
            if c not in self.ref_rows or self.ref_rows[c] < kth - slack:
                bad.append(("extra", c, self.ref_rows.get(c)))
        for c in ref_set - gpu_set:
            if self.ref_rows[c] > kth + slack:
                bad.append(("missing", c, self.ref_rows[c]))
        return not bad, bad

    def summary(self) -> dict:
        ok, bad = self.topk_agree()
        return {"norm_err": self.norm_err, "rrmse": self.rrmse, "max_ref": self.max_ref,
                "topk_ok": ok, "topk_mismatch": bad[:4]}


def check_against_plane(t, b, p, ref_plane, k, tol=FP32_TOL):
    """GPU top-k list of one array against its FP64 oracle plane."""
    m, n = ref_plane.shape
    cells = m * n
    import oracle
    want = oracle.topk(ref_plane, k)
    maxref = float(ref_plane.max()) if cells else 0.0
    if cells < k:
        assert np.all(t[cells:] == -1) and np.all(b[cells:] == -1) and np.all(p[cells:] == -1.0)
    got = [(int(t[r]), int(b[r]), float(p[r])) for r in range(min(k, cells))]
    # each reported power is the oracle's power at that cell
    for tt, bb, pp in got:
        assert 0 <= tt < m and 0 <= bb < n
        assert abs(pp - ref_plane[tt, bb]) <= tol * maxref + 1e-30
    # ordered by (P desc, t asc, bin asc)
    for r in range(len(got) - 1):
        a_, c_ = got[r], got[r + 1]
        assert a_[2] > c_[2] or (a_[2] == c_[2] and (a_[0], a_[1]) < (c_[0], c_[1]))
    # same set as the oracle's, up to swaps within the tolerance of the k-th value
    kth = want[-1][2]
    gs = {(a_, b_) for a_, b_, _ in got}
    ws = {(a_, b_) for a_, b_, _ in want}
    for c in gs - ws:
        assert ref_plane[c] >= kth - tol * maxref, ("extra", c)
    for c in ws - gs:
        assert ref_plane[c] <= kth + tol * maxref, ("missing", c)


class OracleTopk:
    """The FP64 oracle's top-k cells of one array's whole power plane,
    computed in blocks of rows so that no plane is held whole: the k largest
    cells by (P desc, t asc, i asc), the plane's maximum, and every cell tied
    with or above the running k-th value (so the k-th value is exact)."""

    def __init__(self, x, taps, tap_len, k: int = TOPK, rows_per_block: int = 8, nthreads: int = 0):
        import oracle
        self.k = k
        m = taps.shape[0]
        cand = []                    # (P, t, i) of every cell that may still be in the top k
        thr = -np.inf
        self.maxref = 0.0
        self.n = int(np.asarray(x).shape[0])
        for r0 in range(0, m, rows_per_block):
            rows = list(range(r0, min(m, r0 + rows_per_block)))
            blk = oracle.power(x, taps, tap_len, rows=rows, nthreads=nthreads)
            self.maxref = max(self.maxref, float(blk.max()) if blk.size else 0.0)
            flat = blk.reshape(-1)
            if len(cand) < k:           # fewer than k cells so far: this block's k largest
                take = min(k, flat.size)
                sel = np.flatnonzero(flat >= np.partition(flat, flat.size - take)[flat.size - take])
            else:
                sel = np.flatnonzero(flat >= thr)
            n = blk.shape[1]
            for c in sel.tolist():
                cand.append((float(flat[c]), rows[c // n], c % n))
            cand.sort(key=lambda e: (-e[0], e[1], e[2]))
            if len(cand) >= k:
                thr = cand[k - 1][0]
                cand = [e for e in cand if e[0] >= thr]
        self.top = [(t, i, p) for p, t, i in cand[:k]]
        self.kth = self.top[-1][2] if self.top else 0.0
        # every cell at or above the k-th value (ties included)
        self.above = {(t, i): p for p, t, i in cand}

    def check(self, x, taps, tap_len, t, b, p, tol=FP32_TOL):
        """GPU top-k list (t, b, p arrays) of this array against the oracle's,
        with the near-tie rule: each reported power equals the oracle's power
        at that cell within tol * max P; the list is ordered; and the cell
        sets agree except for cells within tol * max P of the k-th value."""
        import oracle
        k = self.k
        cells = taps.shape[0] * self.n
        got = [(int(t[r]), int(b[r]), float(p[r])) for r in range(min(k, cells))]
        if cells < k:
            assert np.all(t[cells:] == -1) and np.all(b[cells:] == -1) and np.all(p[cells:] == -1.0)
        slack = tol * self.maxref
        for tt, bb, _ in got:
            assert 0 <= tt < taps.shape[0] and 0 <= bb < self.n, (tt, bb)
        ref_at = oracle.power_at(x, taps, tap_len, [g[0] for g in got], [g[1] for g in got])
        for (tt, bb, pp), rv in zip(got, ref_at):
            assert abs(pp - rv) <= slack + 1e-30, ("power", tt, bb, pp, rv)
        for r in range(len(got) - 1):
            a_, c_ = got[r], got[r + 1]
            assert a_[2] > c_[2] or (a_[2] == c_[2] and (a_[0], a_[1]) < (c_[0], c_[1])), ("order", r)
        gs = {(a_, b_): rv for (a_, b_, _), rv in zip(got, ref_at)}
        ws = {(a_, b_) for a_, b_, _ in self.top}
        for c, rv in gs.items():
            if c not in ws:
                assert rv >= self.kth - slack, ("extra", c, rv, self.kth)
        for c in ws - set(gs):
            assert self.above[c] <= self.kth + slack, ("missing", c, self.above[c], self.kth)
        return max((abs(pp - rv) for (_, _, pp), rv in zip(got, ref_at)), default=0.0) / max(self.maxref, 1e-300)
