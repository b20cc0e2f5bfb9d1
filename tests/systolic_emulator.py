"""CPU model of the systolic schedule (test code; no GPU, no library).

It reproduces, with numpy float32 arithmetic on whole boxes, the data flow of
the persistent systolic kernel: the tile plan, the per-tile slot box that
moves one cell along the x-y-z-t diagonal per step, the faces ("trails")
published to the field arrays (x and y faces) and to a per-ticket z-face ring,
the forward-shell loads, the neighbour progress counters and the waits on them,
the band starts and ends, and the ring-slot reuse waits.  Tickets run as
coroutines that yield at every wait; a seeded scheduler interleaves up to
``resident`` of them at random (tickets are dequeued in order, as by the
kernel's atomic ticket counter).  A missing or misplaced wait shows up as a
read of stale data, so the result stops matching the FP32 oracle.

Skewed frame: during the tau-th step of a call (tau = 1..nsteps) the tile with
index (a, b, c) updates B_tau = [a*Wx + tau, a*Wx + tau + Wx - 1] x ... and
keeps the slot box R = B_tau plus one layer below on every axis.  All axes
must be PEC: cells outside the domain are ghosts that read as zero.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def plan(shape, W, K, nsteps):
    """Tickets in dequeue order and per-band tile ranges.

    Returns (tickets, ranges, ticket_of) with tickets = [(band, a, b, c)],
    ranges[band] = ((alo, ahi), (blo, bhi), (clo, chi)), and ticket_of a dict
    (band, a, b, c) -> ticket index.  Within a band, tiles are ordered by
    depth below the most upwind corner (upwind first): every tile appears
    after its seven upwind neighbours."""
    tickets, ranges = [], []
    nb = (nsteps + K - 1) // K
    for band in range(nb):
        t0, t1 = band * K, min(nsteps, (band + 1) * K)
        rg = []
        for n, w in zip(shape, W):
            lo = -((w - 1 + t1) // w)          # ceil((1 - w - t1) / w)
            hi = (n - 2 - t0) // w
            rg.append((lo, hi))
        ranges.append(tuple(rg))
        tiles = [(a, b, c) for a in range(rg[0][0], rg[0][1] + 1)
                 for b in range(rg[1][0], rg[1][1] + 1)
                 for c in range(rg[2][0], rg[2][1] + 1)]
        tiles.sort(key=lambda p: ((rg[0][1] - p[0]) + (rg[1][1] - p[1]) + (rg[2][1] - p[2]), p))
        tickets += [(band,) + p for p in tiles]
    ticket_of = {t: i for i, t in enumerate(tickets)}
    return tickets, ranges, ticket_of


def ring_depth(tickets, ticket_of):
    """Smallest ring size R such that the consumer of ticket t (its -z
    neighbour in the same band) has index < t + R."""
    R = 1
    for i, (band, a, b, c) in enumerate(tickets):
        j = ticket_of.get((band, a, b, c - 1))
        if j is not None:
            R = max(R, j - i + 1)
    return R


class Machine:
    def __init__(self, fields, cE, cH, shape, W, K, nsteps, sources=(), step0=0,
                 ring_slack=0):
        self.f = [np.array(x, dtype=F32) for x in fields]
        self.cE = [np.asarray(x, dtype=F32) for x in cE]
        self.cH = F32(cH)
        self.shape = tuple(shape)
        self.W = tuple(W)
        self.K = K
        self.nsteps = nsteps
        self.sources = list(sources)
        self.step0 = step0
        self.tickets, self.ranges, self.ticket_of = plan(shape, W, K, nsteps)
        self.R = ring_depth(self.tickets, self.ticket_of) + ring_slack
        Wx, Wy, Wz = W
        # ring: [slot][local step][9 values][Wx][Wy]; values: Ex Ey Ez Hx Hy Hz cEx cEy cEz
        self.ring = np.full((self.R, K, 9, Wx, Wy), np.nan, dtype=F32)
        self.progress = {}
        self.reads_before_ready = 0

    # ---- geometry ---------------------------------------------------------
    def exists(self, band, a, b, c):
        rg = self.ranges[band]
        return rg[0][0] <= a <= rg[0][1] and rg[1][0] <= b <= rg[1][1] and rg[2][0] <= c <= rg[2][1]

    def _box_index(self, lo, size):
        """Index arrays for a box with lower corner lo and given size, plus an
        in-domain mask."""
        ax = [np.arange(l, l + s) for l, s in zip(lo, size)]
        inb = [(x >= 0) & (x < n) for x, n in zip(ax, self.shape)]
        mask = inb[0][:, None, None] & inb[1][None, :, None] & inb[2][None, None, :]
        cl = [np.clip(x, 0, n - 1) for x, n in zip(ax, self.shape)]
        return np.ix_(*cl), mask

    def load_box(self, arr, lo, size):
        idx, mask = self._box_index(lo, size)
        return np.where(mask, arr[idx], F32(0)).astype(F32)

    def store_box(self, arr, lo, vals):
        """Store the in-domain part of a box; ghost cells are dropped."""
        dst, src = [], []
        for l, s, n in zip(lo, vals.shape, self.shape):
            a, b = max(l, 0), min(l + s, n)
            if a >= b:
                return
            dst.append(slice(a, b))
            src.append(slice(a - l, b - l))
        arr[tuple(dst)] = vals[tuple(src)]

    # ---- coroutine for one ticket ------------------------------------------
    def wait(self, tile, target):
        while self.progress.get(tile, 0) < target:
            yield "wait"

    def run_ticket(self, t):
        band, a, b, c = self.tickets[t]
        K, (Wx, Wy, Wz) = self.K, self.W
        t0, t1 = band * K, min(self.nsteps, (band + 1) * K)
        ups = [(a + dx, b + dy, c + dz) for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)
               if (dx, dy, dz) != (0, 0, 0)]
        me = (a, b, c)
        # band start: this tile and its upwind neighbours finished the previous band
        if band > 0:
            for u in [me] + ups:
                if self.exists(band - 1, *u):
                    yield from self.wait(u, 2 * t0)
        # ring slot reuse: the previous occupant of the slot has finished
        # writing it and its consumer (the -z neighbour) has finished reading it
        slot = t % self.R
        if t >= self.R:
            pb, pa, pbb, pc = self.tickets[t - self.R]
            pend = 2 * min(self.nsteps, (pb + 1) * K)
            yield from self.wait((pa, pbb, pc), pend)
            cons = (pa, pbb, pc - 1)
            if self.exists(pb, *cons):
                yield from self.wait(cons, pend)
        ox, oy, oz = a * Wx, b * Wy, c * Wz
        # slot box of step t0 + 1: lower corner (ox + t0, ...), size W + 1
        lo = (ox + t0, oy + t0, oz + t0)
        P = (Wx + 1, Wy + 1, Wz + 1)
        S = [self.load_box(self.f[q], lo, P) for q in range(6)]
        C = [self.load_box(self.cE[q], lo, P) for q in range(3)]
        cH = self.cH
        for tau in range(t0 + 1, t1 + 1):
            # box lower corner at the start of step tau is (o + tau - 1)
            blo = (ox + tau, oy + tau, oz + tau)          # B_tau lower corner
            Ex, Ey, Ez, Hx, Hy, Hz = S
            cx, cy, cz = C
            i, j, k = slice(1, None), slice(1, None), slice(1, None)
            bb = (i, j, k)
            # E half-step on B = box[1:,1:,1:], backward neighbours at index - 1
            ex = (Ex[bb] + cx[bb] * (Hz[bb] - Hz[1:, :-1, 1:])) - cx[bb] * (Hy[bb] - Hy[1:, 1:, :-1])
            ey = (Ey[bb] + cy[bb] * (Hx[bb] - Hx[1:, 1:, :-1])) - cy[bb] * (Hz[bb] - Hz[:-1, 1:, 1:])
            ez = (Ez[bb] + cz[bb] * (Hy[bb] - Hy[:-1, 1:, 1:])) - cz[bb] * (Hx[bb] - Hx[1:, :-1, 1:])
            Ex[bb], Ey[bb], Ez[bb] = ex, ey, ez
            # sources on cells of B
            s = self.step0 + tau - 1
            for src in self.sources:
                m = s - src["first_step"]
                if m < 0 or m >= len(src["waveform"]):
                    continue
                p = (src["i"] - blo[0], src["j"] - blo[1], src["k"] - blo[2])
                if all(0 <= p[d] < self.W[d] for d in range(3)):
                    arr = S[src["comp"]]
                    q = (p[0] + 1, p[1] + 1, p[2] + 1)
                    arr[q] = F32(arr[q] + F32(src["waveform"][m]))
            # publish E of the first layer of B: x and y faces to the field
            # arrays, z face to the ring
            self._publish(S, C, blo, slot, tau - t0 - 1, comps=(0, 1, 2))
            self.progress[me] = 2 * tau - 1
            yield "E"
            for u in ups:
                if self.exists(band, *u):
                    yield from self.wait(u, 2 * tau - 1)
            # shift the box by one on every axis; load the forward shell's E
            S = [self._shift(x) for x in S]
            C = [self._shift(x) for x in C]
            nlo = (ox + tau, oy + tau, oz + tau)
            self._load_forward(S, C, nlo, band, (a, b, c), tau - t0 - 1, comps=(0, 1, 2))
            Ex, Ey, Ez, Hx, Hy, Hz = S
            hb = (slice(0, -1), slice(0, -1), slice(0, -1))   # B_tau in the new box
            hx = (Hx[hb] - cH * (Ez[:-1, 1:, :-1] - Ez[hb])) + cH * (Ey[:-1, :-1, 1:] - Ey[hb])
            hy = (Hy[hb] - cH * (Ex[:-1, :-1, 1:] - Ex[hb])) + cH * (Ez[1:, :-1, :-1] - Ez[hb])
            hz = (Hz[hb] - cH * (Ey[1:, :-1, :-1] - Ey[hb])) + cH * (Ex[:-1, 1:, :-1] - Ex[hb])
            Hx[hb], Hy[hb], Hz[hb] = hx, hy, hz
            # publish H (and the coefficients, for the ring) of the first layer
            self._publish_shifted(S, C, blo, slot, tau - t0 - 1)
            if tau == t1:
                # band end: the whole B goes back to the field arrays
                for q in range(6):
                    self.store_box(self.f[q], blo, S[q][hb])
            self.progress[me] = 2 * tau
            yield "H"
            if tau < t1:
                for u in ups:
                    if self.exists(band, *u):
                        yield from self.wait(u, 2 * tau)
                self._load_forward(S, C, nlo, band, (a, b, c), tau - t0 - 1, comps=(3, 4, 5),
                                   coef=True)

    @staticmethod
    def _shift(x):
        y = np.full_like(x, np.nan)
        y[:-1, :-1, :-1] = x[1:, 1:, 1:]
        return y

    def _publish(self, S, C, blo, slot, ls, comps):
        """E of the first layer of B (box index 1 on each axis, before the shift)."""
        for q in comps:
            B = S[q][1:, 1:, 1:]
            # x face: x = blo[0], all (y, z) of B
            self.store_box(self.f[q], blo, B[0:1, :, :])
            # y face: y = blo[1]
            self.store_box(self.f[q], blo, B[:, 0:1, :])
            # z face -> ring
            self.ring[slot, ls, q] = B[:, :, 0]

    def _publish_shifted(self, S, C, blo, slot, ls):
        """H of the first layer of B after the shift (box index 0 on each axis)."""
        for q in (3, 4, 5):
            B = S[q][:-1, :-1, :-1]
            self.store_box(self.f[q], blo, B[0:1, :, :])
            self.store_box(self.f[q], blo, B[:, 0:1, :])
            self.ring[slot, ls, q] = B[:, :, 0]
        for q in range(3):
            self.ring[slot, ls, 6 + q] = C[q][:-1, :-1, 0]

    def _load_forward(self, S, C, nlo, band, tile, ls, comps, coef=False):
        """Load the forward shell of the box whose lower corner is nlo."""
        Wx, Wy, Wz = self.W
        a, b, c = tile
        X, Y, Z = nlo[0] + Wx, nlo[1] + Wy, nlo[2] + Wz
        arrs = [(S[q], self.f[q], q) for q in comps]
        if coef:
            arrs += [(C[q], self.cE[q], 6 + q) for q in range(3)]
        zt = (band, a, b, c + 1)
        zslot = self.ticket_of[zt] % self.R if zt in self.ticket_of else None
        for box, src, q in arrs:
            # x plane: all (y, z) of the box at x = X
            box[-1:, :, :] = self.load_box(src, (X, nlo[1], nlo[2]), (1, Wy + 1, Wz + 1))
            # y plane: x < X, y = Y
            box[:-1, -1:, :] = self.load_box(src, (nlo[0], Y, nlo[2]), (Wx, 1, Wz + 1))
            # z plane: x < X, y < Y, z = Z, from the +z neighbour's ring slot
            if zslot is None:
                vals = np.zeros((Wx, Wy), F32)
            else:
                vals = self.ring[zslot, ls, q]
            _, mask = self._box_index((nlo[0], nlo[1], Z), (Wx, Wy, 1))
            box[:-1, :-1, -1] = np.where(mask[:, :, 0], vals, F32(0))

    # ---- scheduler --------------------------------------------------------
    def run(self, resident=4, seed=0):
        rng = np.random.default_rng(seed)
        nxt = 0
        live = []
        guard = 0
        while nxt < len(self.tickets) or live:
            while len(live) < resident and nxt < len(self.tickets):
                live.append((nxt, self.run_ticket(nxt)))
                nxt += 1
            order = rng.permutation(len(live))
            progressed = False
            for idx in order:
                t, g = live[idx]
                try:
                    r = next(g)
                    if r != "wait":
                        progressed = True
                except StopIteration:
                    live[idx] = None
                    progressed = True
                    break
                if progressed:
                    break
            live = [x for x in live if x is not None]
            guard = 0 if progressed else guard + 1
            if guard > 100000:
                raise RuntimeError("emulated schedule deadlocked")
        return self.f
