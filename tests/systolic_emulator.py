"""CPU model of the systolic schedule (test code; no GPU, no library).

It reproduces, with numpy float32 arithmetic on whole boxes, the data flow of
the persistent systolic kernel: the tile plan, the per-tile slot box that
moves one cell along the x-y-z-t diagonal per step, the faces ("trails")
published to per-ticket face rings (one per face orientation), the
forward-shell loads that assemble each face from up to four producers (edges
and corners come from the diagonal neighbours), the neighbour progress
counters and the waits on them, the band starts and ends (the only accesses
of the field arrays), and the ring-slot reuse waits.  Tickets run as
coroutines that yield at every wait; a seeded scheduler interleaves up to
``resident`` of them at random (tickets are dequeued in order, as by the
kernel's atomic ticket counter).  A missing or misplaced wait shows up as a
read of stale data, so the result stops matching the FP32 oracle.

Skewed frame: during the tau-th step of a call (tau = 1..nsteps) the tile with
index (a, b, c) updates B_tau = [a*Wx + tau, a*Wx + tau + wx - 1] x ... and
keeps the slot box R = B_tau plus one layer below on every axis.  On a PEC
axis cells outside the domain are ghosts that read as zero and the tile range
of each band covers the domain; on a periodic axis positions wrap modulo n,
the L = ceil(n / W) tiles form a ring whose last tile is ragged (width
n - W (L - 1)), and the tiles of a ring depend on each other in a cycle that
only time breaks: they must be resident together and advance in lock-step.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def ring_tiles(shape, W, bc):
    """Tiles per periodic axis (None on PEC axes)."""
    return [-(-n // w) if p else None for n, w, p in zip(shape, W, bc)]


def plan(shape, W, K, nsteps, bc=(0, 0, 0)):
    """Tickets in dequeue order and per-band tile ranges.

    Returns (tickets, ranges, ticket_of) with tickets = [(band, a, b, c)],
    ranges[band] = ((alo, ahi), (blo, bhi), (clo, chi)), and ticket_of a dict
    (band, a, b, c) -> ticket index.  Within a band, tiles are ordered by
    depth below the most upwind corner along the PEC axes (upwind first), and
    the tiles that differ only along periodic axes (one ring group) are
    consecutive: every tile appears after its upwind neighbours outside its
    group."""
    tickets, ranges = [], []
    L = ring_tiles(shape, W, bc)
    nb = (nsteps + K - 1) // K
    for band in range(nb):
        t0, t1 = band * K, min(nsteps, (band + 1) * K)
        rg = []
        for n, w, l in zip(shape, W, L):
            if l is not None:
                rg.append((0, l - 1))
                continue
            lo = -((w - 1 + t1) // w)          # ceil((1 - w - t1) / w)
            hi = (n - 2 - t0) // w
            rg.append((lo, hi))
        ranges.append(tuple(rg))
        tiles = [(a, b, c) for a in range(rg[0][0], rg[0][1] + 1)
                 for b in range(rg[1][0], rg[1][1] + 1)
                 for c in range(rg[2][0], rg[2][1] + 1)]

        def key(p):
            pec = tuple(p[d] for d in range(3) if L[d] is None)
            depth = sum(rg[d][1] - p[d] for d in range(3) if L[d] is None)
            return (depth, pec, p)
        tiles.sort(key=key)
        tickets += [(band,) + p for p in tiles]
    ticket_of = {t: i for i, t in enumerate(tickets)}
    return tickets, ranges, ticket_of


def wrap_tile(t, L):
    """Tile coordinates with the periodic axes wrapped onto their rings."""
    return tuple(x % l if l is not None else x for x, l in zip(t, L))


# offsets of the seven downwind (consumer) and upwind (producer) neighbours
DOWN = [(-dx, -dy, -dz) for dx in (0, 1) for dy in (0, 1) for dz in (0, 1) if (dx, dy, dz) != (0, 0, 0)]


def ring_depth(tickets, ticket_of, L=(None, None, None)):
    """Smallest ring size R such that every consumer of ticket t (its
    downwind neighbours in the same band) has index < t + R."""
    R = 1
    for i, (band, a, b, c) in enumerate(tickets):
        for d in DOWN:
            j = ticket_of.get((band,) + wrap_tile((a + d[0], b + d[1], c + d[2]), L))
            if j is not None:
                R = max(R, j - i + 1)
    return R


class Machine:
    def __init__(self, fields, cE, cH, shape, W, K, nsteps, sources=(), step0=0,
                 ring_slack=0, bc=(0, 0, 0)):
        self.f = [np.array(x, dtype=F32) for x in fields]
        self.cE = [np.asarray(x, dtype=F32) for x in cE]
        self.cH = F32(cH)
        self.shape = tuple(shape)
        self.W = tuple(W)
        self.K = K
        self.nsteps = nsteps
        self.sources = list(sources)
        self.step0 = step0
        self.per = tuple(bool(p) for p in bc)
        for n, w, p in zip(shape, W, self.per):
            if p and n <= w:
                raise ValueError("a periodic axis needs at least two tiles")
        self.L = ring_tiles(shape, W, self.per)
        self.tickets, self.ranges, self.ticket_of = plan(shape, W, K, nsteps, self.per)
        # a slot is reused R tickets later, after its previous occupant and that
        # occupant's consumers have finished their band; with R beyond the ring
        # depth plus one ring group, all lie in groups before the reuser's own
        self.group = int(np.prod([l for l in self.L if l is not None]))
        self.R = ring_depth(self.tickets, self.ticket_of, self.L) + self.group - 1 + ring_slack
        Wx, Wy, Wz = W
        # face rings per [slot][local step][value]: x face [Wy][Wz] and y face
        # [Wx][Wz] of Ex Ey Ez Hx Hy Hz; z face [Wx][Wy] of those and cEx cEy cEz
        self.xring = np.full((self.R, K, 6, Wy, Wz), np.nan, dtype=F32)
        self.yring = np.full((self.R, K, 6, Wx, Wz), np.nan, dtype=F32)
        self.ring = np.full((self.R, K, 9, Wx, Wy), np.nan, dtype=F32)
        self.progress = {}
        self.reads_before_ready = 0

    # ---- geometry ---------------------------------------------------------
    def tile(self, band, a, b, c):
        """The tile (a, b, c) wrapped onto the periodic rings, or None if the
        band has no such tile."""
        t = wrap_tile((a, b, c), self.L)
        rg = self.ranges[band]
        if all(rg[d][0] <= t[d] <= rg[d][1] for d in range(3)):
            return t
        return None

    def exists(self, band, a, b, c):
        return self.tile(band, a, b, c) is not None

    def widths(self, tile):
        """Updated cells per axis of a tile (the last tile of a ring is ragged)."""
        return tuple(n - w * (l - 1) if l is not None and x == l - 1 else w
                     for x, n, w, l in zip(tile, self.shape, self.W, self.L))

    def _box_index(self, lo, size):
        """Index arrays for a box with lower corner lo and given size, plus an
        in-domain mask (periodic axes wrap and are always in the domain)."""
        ax = [np.arange(l, l + s) for l, s in zip(lo, size)]
        inb = [np.ones(len(x), bool) if p else (x >= 0) & (x < n)
               for x, n, p in zip(ax, self.shape, self.per)]
        mask = inb[0][:, None, None] & inb[1][None, :, None] & inb[2][None, None, :]
        cl = [x % n if p else np.clip(x, 0, n - 1) for x, n, p in zip(ax, self.shape, self.per)]
        return np.ix_(*cl), mask

    def load_box(self, arr, lo, size):
        idx, mask = self._box_index(lo, size)
        return np.where(mask, arr[idx], F32(0)).astype(F32)

    def store_box(self, arr, lo, vals):
        """Store the in-domain part of a box; ghost cells are dropped."""
        dst, src = [], []
        for l, s, n, p in zip(lo, vals.shape, self.shape, self.per):
            if p:
                assert s <= n
                dst.append(np.arange(l, l + s) % n)
                src.append(np.arange(s))
                continue
            a, b = max(l, 0), min(l + s, n)
            if a >= b:
                return
            dst.append(np.arange(a, b))
            src.append(np.arange(a - l, b - l))
        arr[np.ix_(*dst)] = vals[np.ix_(*src)]

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
        wx, wy, wz = self.widths(me)
        # band start: this tile and its upwind neighbours finished the previous band
        if band > 0:
            for u in [me] + ups:
                u = self.tile(band - 1, *u)
                if u is not None:
                    yield from self.wait(u, 2 * t0)
        # ring slot reuse: the previous occupant of the slot has finished
        # writing it and its consumers (its downwind neighbours) have finished
        # reading it
        slot = t % self.R
        if t >= self.R:
            pb, pa, pbb, pc = self.tickets[t - self.R]
            pend = 2 * min(self.nsteps, (pb + 1) * K)
            yield from self.wait((pa, pbb, pc), pend)
            for d in DOWN:
                cons = self.tile(pb, pa + d[0], pbb + d[1], pc + d[2])
                if cons is not None:
                    yield from self.wait(cons, pend)
        ox, oy, oz = a * Wx, b * Wy, c * Wz
        # slot box of step t0 + 1: lower corner (ox + t0, ...), size W + 1
        lo = (ox + t0, oy + t0, oz + t0)
        P = (wx + 1, wy + 1, wz + 1)
        S = [self.load_box(self.f[q], lo, P) for q in range(6)]
        C = [self.load_box(self.cE[q], lo, P) for q in range(3)]
        cH = self.cH
        for tau in range(t0 + 1, t1 + 1):
            if self._below(me, tau):
                # before the tile's first cell crosses the lower wall of a PEC
                # axis the box holds ghosts only (+0, loaded so and never
                # changed), which reach no grid cell: no update and no faces.
                # The last such step still takes the forward shells, which
                # carry the first grid cells into the box.
                last = tau < t1 and not self._below(me, tau + 1)
                self.progress[me] = 2 * tau - 1
                yield "E"
                if last:
                    for u in ups:
                        u = self.tile(band, *u)
                        if u is not None:
                            yield from self.wait(u, 2 * tau - 1)
                    S = [self._shift(x) for x in S]
                    C = [self._shift(x) for x in C]
                    nlo = (ox + tau, oy + tau, oz + tau)
                    self._load_forward(S, C, nlo, band, (a, b, c), tau - t0 - 1, comps=(0, 1, 2))
                self.progress[me] = 2 * tau
                yield "H"
                if last:
                    for u in ups:
                        u = self.tile(band, *u)
                        if u is not None:
                            yield from self.wait(u, 2 * tau)
                    self._load_forward(S, C, nlo, band, (a, b, c), tau - t0 - 1, comps=(3, 4, 5),
                                       coef=True)
                continue
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
                p = [src["i"] - blo[0], src["j"] - blo[1], src["k"] - blo[2]]
                p = [x % n if per else x for x, n, per in zip(p, self.shape, self.per)]
                if all(0 <= p[d] < (wx, wy, wz)[d] for d in range(3)):
                    arr = S[src["comp"]]
                    q = (p[0] + 1, p[1] + 1, p[2] + 1)
                    arr[q] = F32(arr[q] + F32(src["waveform"][m]))
            # publish E of the first layer of B to the face rings
            self._publish(S, C, blo, slot, tau - t0 - 1, comps=(0, 1, 2))
            self.progress[me] = 2 * tau - 1
            yield "E"
            for u in ups:
                u = self.tile(band, *u)
                if u is not None:
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
            if tau < t1 and self._gone(me, tau + 1):
                # every cell of B_{tau+1} (and later boxes) lies past a PEC
                # wall: nothing the tile would compute reaches a grid cell, and
                # its consumers read those positions as ghosts (+0).  The
                # band-end level releases everything that waits on it.
                self.progress[me] = 2 * t1
                return
            if tau < t1:
                for u in ups:
                    u = self.tile(band, *u)
                    if u is not None:
                        yield from self.wait(u, 2 * tau)
                self._load_forward(S, C, nlo, band, (a, b, c), tau - t0 - 1, comps=(3, 4, 5),
                                   coef=True)

    def _below(self, tile, tau):
        """True if B_tau of the tile lies wholly below the lower wall of a PEC
        axis (its cells there are o + tau .. o + tau + W - 1), on a grid with
        no periodic axis (the kernel variant for periodic grids runs such
        steps in full)."""
        if any(self.per):
            return False
        return any(o * w + tau + w - 1 < 0 for o, w in zip(tile, self.W))

    def _gone(self, tile, tau):
        """True if B_tau of the tile lies wholly past the upper wall of a PEC
        axis (its lower corner is o + tau on every axis)."""
        return any(not p and o * w + tau >= n
                   for o, w, n, p in zip(tile, self.W, self.shape, self.per))

    @staticmethod
    def _shift(x):
        y = np.full_like(x, np.nan)
        y[:-1, :-1, :-1] = x[1:, 1:, 1:]
        return y

    def _faces(self, B, slot, ls, q):
        """The three first-layer faces of B (shape wx, wy, wz) into the rings."""
        wx, wy, wz = B.shape
        self.xring[slot, ls, q, :wy, :wz] = B[0, :, :]
        self.yring[slot, ls, q, :wx, :wz] = B[:, 0, :]
        self.ring[slot, ls, q, :wx, :wy] = B[:, :, 0]

    def _publish(self, S, C, blo, slot, ls, comps):
        """E of the first layer of B (box index 1 on each axis, before the shift)."""
        for q in comps:
            self._faces(S[q][1:, 1:, 1:], slot, ls, q)

    def _publish_shifted(self, S, C, blo, slot, ls):
        """H of the first layer of B after the shift (box index 0 on each axis)."""
        for q in (3, 4, 5):
            self._faces(S[q][:-1, :-1, :-1], slot, ls, q)
        for q in range(3):
            cq = C[q][:-1, :-1, 0]
            self.ring[slot, ls, 6 + q, :cq.shape[0], :cq.shape[1]] = cq

    def _slot(self, band, a, b, c):
        t = self.tile(band, a, b, c)
        return self.ticket_of[(band,) + t] % self.R if t is not None else None

    def _load_forward(self, S, C, nlo, band, tile, ls, comps, coef=False):
        """Load the forward shell of the box whose lower corner is nlo: E and
        H from the producers' face rings, the coefficients from their arrays."""
        Wx, Wy, Wz = self.widths(tile)
        a, b, c = tile
        X, Y, Z = nlo[0] + Wx, nlo[1] + Wy, nlo[2] + Wz
        _, mx = self._box_index((X, nlo[1], nlo[2]), (1, Wy + 1, Wz + 1))
        _, my = self._box_index((nlo[0], Y, nlo[2]), (Wx, 1, Wz + 1))
        _, mz = self._box_index((nlo[0], nlo[1], Z), (Wx, Wy, 1))
        # the +x neighbours: own rows and columns from (a+1, b, c); the
        # forward row, column and corner from the first row / column of the
        # +x+y, +x+z and +x+y+z neighbours
        parts_x = [((0, 0), slice(0, Wy), slice(0, Wz), slice(0, Wy), slice(0, Wz)),
                   ((1, 0), slice(Wy, Wy + 1), slice(0, Wz), slice(0, 1), slice(0, Wz)),
                   ((0, 1), slice(0, Wy), slice(Wz, Wz + 1), slice(0, Wy), slice(0, 1)),
                   ((1, 1), slice(Wy, Wy + 1), slice(Wz, Wz + 1), slice(0, 1), slice(0, 1))]
        parts_y = [(0, slice(0, Wz), slice(0, Wz)), (1, slice(Wz, Wz + 1), slice(0, 1))]
        zslot = self._slot(band, a, b, c + 1)
        for q in comps:
            box = S[q]
            vx = np.zeros((Wy + 1, Wz + 1), F32)
            for (dy, dz), ry, rz, sy, sz in parts_x:
                sl = self._slot(band, a + 1, b + dy, c + dz)
                if sl is not None:
                    vx[ry, rz] = self.xring[sl, ls, q, sy, sz]
            box[-1, :, :] = np.where(mx[0], vx, F32(0))
            vy = np.zeros((Wx, Wz + 1), F32)
            for dz, rz, sz in parts_y:
                sl = self._slot(band, a, b + 1, c + dz)
                if sl is not None:
                    vy[:, rz] = self.yring[sl, ls, q, :Wx, sz]
            box[:-1, -1, :] = np.where(my[:, 0, :], vy, F32(0))
            vz = self.ring[zslot, ls, q, :Wx, :Wy] if zslot is not None else np.zeros((Wx, Wy), F32)
            box[:-1, :-1, -1] = np.where(mz[:, :, 0], vz, F32(0))
        if coef:
            for q in range(3):
                box = C[q]
                box[-1:, :, :] = self.load_box(self.cE[q], (X, nlo[1], nlo[2]), (1, Wy + 1, Wz + 1))
                box[:-1, -1:, :] = self.load_box(self.cE[q], (nlo[0], Y, nlo[2]), (Wx, 1, Wz + 1))
                vz = (self.ring[zslot, ls, 6 + q, :Wx, :Wy] if zslot is not None
                      else np.zeros((Wx, Wy), F32))
                box[:-1, :-1, -1] = np.where(mz[:, :, 0], vz, F32(0))

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
