"""Oracle values of one cell computed on a crop around it (test helper).

After n steps a cell depends only on cells within n of it on each axis, so a
crop of half-width n+2 reproduces it.  A crop that ends at the grid's upper
wall gets an artificial PEC plane at its own lower end (tangential E zeroed)
so that its periodic wrap reproduces the wall; crops that start at the lower
wall keep the real wall; interior crops wrap periodically.  Every artificial
boundary is more than n cells from the cell and cannot reach it.

With FP16 storage on the systolic scheme the grid is rounded once per band,
cell by cell, so the crop takes the same rounding at the same steps.
"""
import numpy as np

import oracle

PEC, PER = 0, 1


def crop_oracle(w, p, nsteps, fp16_band=None):
    """FP32 oracle values of all six components at cell p after nsteps (with
    fp16_band: the FP16-storage systolic schedule with that band length)."""
    r = nsteps + 2
    lo, hi, bc, art = [], [], [], []
    for a in range(3):
        n = w.shape[a]
        l, h = max(0, p[a] - r), min(n, p[a] + r + 1)
        lo.append(l)
        hi.append(h)
        if l == 0 or h == n:
            bc.append(PEC)
            art.append(l > 0)          # crop ends at the upper wall only
        else:
            bc.append(PER)
            art.append(False)
    sl = tuple(slice(l, h) for l, h in zip(lo, hi))
    eps = np.ascontiguousarray(w.eps[sl])
    fields = [np.ascontiguousarray(f[sl]) for f in w.fields_or_zeros()]
    for c in range(3):                 # artificial lower walls: tangential E = +0
        for a in range(3):
            if a != c and art[a]:
                idx = [slice(None)] * 3
                idx[a] = 0
                fields[c][tuple(idx)] = 0.0
    srcs = []
    for s in w.sources:
        q = (s["i"] - lo[0], s["j"] - lo[1], s["k"] - lo[2])
        if all(0 <= q[a] < hi[a] - lo[a] for a in range(3)):
            srcs.append(dict(s, i=q[0], j=q[1], k=q[2]))
    if fp16_band:
        from oracle import f16
        cE16 = f16.coeff_E16([eps] * 3, tuple(bc), w.dt, w.dx)
        out = f16.run_systolic(fields, cE16, np.float32(w.dt / w.dx), [nsteps], [fp16_band],
                               sources=srcs)
    else:
        out = oracle.run(fields, [eps] * 3, tuple(bc), w.dt, w.dx, nsteps, sources=srcs,
                         dtype=np.float32)
    loc = tuple(p[a] - lo[a] for a in range(3))
    return np.array([o[loc] for o in out], dtype=np.float32)
