// Host-side plan of the systolic launch (see plan.h).
#include "plan.h"

#include <algorithm>

namespace fdtd {
namespace plan {

namespace {

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

}  // namespace

bool build(const int N[3], const int per_in[3], const int W[3], int nsteps, int K, Plan* out,
           std::string* err, const Order& order)
{
    for (int d = 0; d < 3; ++d)
        if (order.w[d] < 1 || order.w[d] > 64) {
            *err = "systolic: order weights must lie in [1, 64]";
            return false;
        }
    int per[3], L[3], group = 1;
    for (int d = 0; d < 3; ++d) {
        per[d] = per_in[d] ? 1 : 0;
        L[d] = per[d] ? (N[d] + W[d] - 1) / W[d] : 0;
        if (per[d]) group *= L[d];
    }
    const int nb = (nsteps + K - 1) / K;
    std::vector<int> band((size_t)kBandRec * nb);
    size_t ntot = 0;
    for (int bb = 0; bb < nb; ++bb) {
        const int t0 = bb * K, t1 = std::min(nsteps, t0 + K);
        size_t cnt = 1;
        for (int d = 0; d < 3; ++d) {
            // tiles whose subdomain meets the grid at some step of the band
            // (a periodic axis always holds its whole ring)
            const int lo = per[d] ? 0 : -floordiv(W[d] - 1 + t1, W[d]);
            const int hi = per[d] ? L[d] - 1 : floordiv(N[d] - 2 - t0, W[d]);
            band[(size_t)kBandRec * bb + 2 * d] = lo;
            band[(size_t)kBandRec * bb + 2 * d + 1] = hi;
            cnt *= (size_t)(hi - lo + 1);
        }
        band[(size_t)kBandRec * bb + 6] = (int)ntot;
        band[(size_t)kBandRec * bb + 7] = 0;
        ntot += cnt;
        if (ntot > (size_t)1 << 30) {
            *err = "systolic: too many tickets";
            return false;
        }
    }
    std::vector<Ticket> tickets(ntot);
    std::vector<int> tix(ntot), depth(ntot);
    size_t pos = 0;
    for (int bb = 0; bb < nb; ++bb) {
        const int* bi = &band[(size_t)kBandRec * bb];
        const int n3[3] = {bi[1] - bi[0] + 1, bi[3] - bi[2] + 1, bi[5] - bi[4] + 1};
        // sort key: weighted depth below the most upwind corner along the
        // PEC axes, under an optional slab index along one PEC axis
        int kmax = 0;
        for (int d = 0; d < 3; ++d)
            if (!per[d]) kmax += order.w[d] * (n3[d] - 1);
        const int sa = order.slab_axis;
        const bool slabs = sa >= 0 && sa < 3 && !per[sa] && order.slab > 0;
        const int nslab = slabs ? (n3[sa] + order.slab - 1) / order.slab : 1;
        const int maxd = nslab * (kmax + 1) - 1;
        // loop order: PEC axes outside, periodic axes inside, so that the
        // tiles of one ring group are enumerated (and so stored) together
        int ax[3], k = 0;
        for (int d = 0; d < 3; ++d)
            if (!per[d]) ax[k++] = d;
        for (int d = 0; d < 3; ++d)
            if (per[d]) ax[k++] = d;
        auto depth_of = [&](const int* i3) {
            int dd = 0;
            for (int d = 0; d < 3; ++d)
                if (!per[d]) dd += order.w[d] * (n3[d] - 1 - i3[d]);
            if (slabs) dd += (nslab - 1 - i3[sa] / order.slab) * (kmax + 1);
            return dd;
        };
        // counting sort by depth (upwind first), stable in the loop order
        std::vector<size_t> count((size_t)maxd + 2, 0);
        int i3[3];
        for (i3[ax[0]] = 0; i3[ax[0]] < n3[ax[0]]; ++i3[ax[0]])
            for (i3[ax[1]] = 0; i3[ax[1]] < n3[ax[1]]; ++i3[ax[1]])
                for (i3[ax[2]] = 0; i3[ax[2]] < n3[ax[2]]; ++i3[ax[2]]) count[(size_t)depth_of(i3) + 1]++;
        for (int d = 1; d <= maxd + 1; ++d) count[d] += count[d - 1];
        for (i3[ax[0]] = 0; i3[ax[0]] < n3[ax[0]]; ++i3[ax[0]])
            for (i3[ax[1]] = 0; i3[ax[1]] < n3[ax[1]]; ++i3[ax[1]])
                for (i3[ax[2]] = 0; i3[ax[2]] < n3[ax[2]]; ++i3[ax[2]]) {
                    const int dd = depth_of(i3);
                    const size_t t = pos + count[dd]++;
                    tickets[t] = Ticket{bb, bi[0] + i3[0], bi[2] + i3[1], bi[4] + i3[2]};
                    depth[t] = dd;
                    tix[(size_t)bi[6] + ((size_t)i3[0] * n3[1] + i3[1]) * n3[2] + i3[2]] = (int)t;
                }
        pos += (size_t)n3[0] * n3[1] * n3[2];
    }
    out->nsteps = nsteps;
    out->K = K;
    out->wx = W[0];
    out->nt = (int)ntot;
    out->nbands = nb;
    for (int d = 0; d < 3; ++d) {
        out->per[d] = per[d];
        out->L[d] = L[d];
    }
    out->group = group;
    out->tickets.swap(tickets);
    out->tix.swap(tix);
    out->band.swap(band);
    out->depth.swap(depth);
    return true;
}

bool merge(const Plan* const* plans, int n, Merged* out, std::string* err)
{
    std::vector<size_t> base(n + 1, 0), tix_base(n + 1, 0), band_base(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        base[i + 1] = base[i] + plans[i]->tickets.size();
        tix_base[i + 1] = tix_base[i] + plans[i]->tix.size();
        band_base[i + 1] = band_base[i] + plans[i]->band.size();
    }
    const size_t nt = base[n];
    if (nt > (size_t)1 << 30 || tix_base[n] > (size_t)1 << 30) {
        *err = "systolic: too many tickets";
        return false;
    }
    std::vector<int> sim(nt), order(nt);
    for (int i = 0; i < n; ++i)
        for (size_t q = base[i]; q < base[i + 1]; ++q) sim[q] = i;
    for (size_t q = 0; q < nt; ++q) order[q] = (int)q;
    if (n > 1)
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const Plan* px = plans[sim[x]];
            const Plan* py = plans[sim[y]];
            const size_t lx = x - base[sim[x]], ly = y - base[sim[y]];
            // band start step (grids may have different band lengths)
            const long long bx = (long long)px->tickets[lx].band * px->K;
            const long long by = (long long)py->tickets[ly].band * py->K;
            if (bx != by) return bx < by;
            return sim[x] < sim[y];
        });
    std::vector<int> pos(nt);  // concatenated index -> merged position
    for (size_t q = 0; q < nt; ++q) pos[order[q]] = (int)q;
    out->tickets.assign(nt, Ticket{0, 0, 0, 0});
    out->tsim.assign(nt, 0);
    out->tix.assign(tix_base[n], 0);
    out->band.assign(band_base[n], 0);
    for (int i = 0; i < n; ++i) {
        const Plan* pi = plans[i];
        for (size_t q = 0; q < pi->tickets.size(); ++q) {
            out->tickets[pos[base[i] + q]] = pi->tickets[q];
            out->tsim[pos[base[i] + q]] = i;
        }
        for (size_t q = 0; q < pi->tix.size(); ++q) out->tix[tix_base[i] + q] = pos[base[i] + pi->tix[q]];
        for (size_t q = 0; q < pi->band.size(); ++q)
            out->band[band_base[i] + q] = pi->band[q] + (q % kBandRec == 6 ? (int)tix_base[i] : 0);
    }
    // largest distance (in tickets) from a face producer to one of its
    // consumers (the downwind neighbours), and the largest ring group
    int D = 1, group = 1;
    for (int i = 0; i < n; ++i) group = std::max(group, plans[i]->group);
    for (size_t t = 0; t < nt; ++t) {
        const Plan* pi = plans[out->tsim[t]];
        const Ticket q = out->tickets[t];
        const int* bi = &out->band[band_base[out->tsim[t]] + (size_t)kBandRec * q.band];
        const int nbb = bi[3] - bi[2] + 1, nc = bi[5] - bi[4] + 1;
        for (int d = 1; d < 8; ++d) {
            int v[3] = {q.a - (d & 1), q.b - ((d >> 1) & 1), q.c - ((d >> 2) & 1)};
            bool in = true;
            for (int k = 0; k < 3; ++k) {
                if (pi->per[k]) v[k] = ((v[k] % pi->L[k]) + pi->L[k]) % pi->L[k];
                in = in && v[k] >= bi[2 * k] && v[k] <= bi[2 * k + 1];
            }
            if (!in) continue;
            const int j = out->tix[(size_t)bi[6] + ((size_t)(v[0] - bi[0]) * nbb + (v[1] - bi[2])) * nc +
                                  (v[2] - bi[4])];
            D = std::max(D, j - (int)t + 1);
        }
    }
    out->band_off.assign(band_base.begin(), band_base.end() - 1);
    out->D = D;
    out->group = group;
    return true;
}

double band_cost(const int N[3], const int per[3], const int W[3], int K)
{
    // Per cell update, a band of K steps costs the tile-steps that cover its
    // skewed space-time region, prod_d (n_d + K/2 + 30) / n_d on PEC axes
    // (tiles that leave through an upper wall stop once wholly outside, so
    // half of the K term remains; tiles below a lower wall skip their
    // updates but keep a workgroup) and W_d L_d / n_d on periodic rings, times
    // (1 + beta / K) for the band's start and end (box load, state
    // write-back, the refill behind each tile's band start).  beta = 10 steps.
    constexpr double kBeta = 10.0;
    double f = 1.0 + kBeta / K;
    for (int d = 0; d < 3; ++d) {
        const double slots = per[d] ? (double)W[d] * ((N[d] + W[d] - 1) / W[d]) : (double)N[d] + 0.5 * K + 30.0;
        f *= slots / N[d];
    }
    return f;
}

}  // namespace plan
}  // namespace fdtd
