// Checks of the systolic launch plan (paper_2502_20610_amd/csrc/plan.cpp),
// built for the host alone with AddressSanitizer and UndefinedBehavior-
// Sanitizer by tests/test_sanitizers_cpu.py.  Exits non-zero on the first
// violated property:
//   - every band holds each tile of its range exactly once, and the tile ->
//     ticket table inverts the ticket list;
//   - the tiles of a band cover every cell of the grid at every step of it;
//   - along PEC axes every upwind neighbour's ticket comes earlier (the
//     deadlock-freedom of the dequeue order), and on periodic axes the tiles
//     of a ring group are contiguous;
//   - a merged launch keeps every grid's own order, and every consumer of a
//     producer lies within D - 1 tickets after it.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "plan.h"

using fdtd::plan::Plan;
using fdtd::plan::Merged;
using fdtd::plan::Ticket;
using fdtd::plan::kBandRec;

static int g_fail = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);               \
            fprintf(stderr, "\n");                      \
            g_fail = 1;                                 \
            return false;                               \
        }                                               \
    } while (0)

static int wrap(const Plan& p, int d, int v) { return p.per[d] ? ((v % p.L[d]) + p.L[d]) % p.L[d] : v; }

static bool check_plan(const int N[3], const int per[3], const int W[3], int nsteps, int K, Plan* out,
                       const fdtd::plan::Order& order = fdtd::plan::Order())
{
    Plan& p = *out;
    std::string err;
    CHECK(fdtd::plan::build(N, per, W, nsteps, K, &p, &err, order), "build failed: %s", err.c_str());
    CHECK(p.nbands == (nsteps + K - 1) / K, "band count");
    CHECK((int)p.tickets.size() == p.nt && (int)p.tix.size() == p.nt && (int)p.depth.size() == p.nt, "sizes");
    CHECK((int)p.band.size() == kBandRec * p.nbands, "band records");
    std::vector<int> seen(p.nt, 0);
    size_t off = 0;
    for (int b = 0; b < p.nbands; ++b) {
        const int* bi = &p.band[(size_t)kBandRec * b];
        CHECK(bi[6] == (int)off, "tix offset of band %d", b);
        const int n3[3] = {bi[1] - bi[0] + 1, bi[3] - bi[2] + 1, bi[5] - bi[4] + 1};
        for (int d = 0; d < 3; ++d) CHECK(n3[d] >= 1, "empty range");
        // coverage of every cell at every step of the band
        const int t0 = b * K, t1 = std::min(nsteps, t0 + K);
        for (int tau = t0 + 1; tau <= t1; ++tau)
            for (int d = 0; d < 3; ++d) {
                if (per[d]) {
                    CHECK(bi[2 * d] == 0 && bi[2 * d + 1] == p.L[d] - 1, "ring range");
                    continue;
                }
                std::vector<char> cov(N[d], 0);
                for (int a = bi[2 * d]; a <= bi[2 * d + 1]; ++a)
                    for (int x = a * W[d] + tau; x < a * W[d] + tau + W[d]; ++x)
                        if (x >= 0 && x < N[d]) cov[x] = 1;
                for (int x = 0; x < N[d]; ++x) CHECK(cov[x], "cell %d of axis %d uncovered at step %d", x, d, tau);
            }
        for (int i = 0; i < n3[0]; ++i)
            for (int j = 0; j < n3[1]; ++j)
                for (int k = 0; k < n3[2]; ++k) {
                    const size_t q = off + ((size_t)i * n3[1] + j) * n3[2] + k;
                    const int t = p.tix[q];
                    CHECK(t >= 0 && t < p.nt, "ticket index range");
                    const Ticket tk = p.tickets[t];
                    CHECK(tk.band == b && tk.a == bi[0] + i && tk.b == bi[2] + j && tk.c == bi[4] + k,
                          "tix does not invert the ticket list");
                    seen[t]++;
                }
        off += (size_t)n3[0] * n3[1] * n3[2];
    }
    for (int t = 0; t < p.nt; ++t) CHECK(seen[t] == 1, "ticket %d listed %d times", t, seen[t]);
    // bands in order, topological order along PEC axes, contiguous ring groups
    std::set<std::tuple<int, int, int, int>> done_groups;
    std::tuple<int, int, int, int> cur_group{-1, 0, 0, 0};
    for (int t = 0; t < p.nt; ++t) {
        const Ticket tk = p.tickets[t];
        if (t) CHECK(p.tickets[t - 1].band <= tk.band, "bands out of order");
        const int* bi = &p.band[(size_t)kBandRec * tk.band];
        const int n3[3] = {bi[1] - bi[0] + 1, bi[3] - bi[2] + 1, bi[5] - bi[4] + 1};
        auto ticket_at = [&](int a, int b, int c) -> int {
            if (a < bi[0] || a > bi[1] || b < bi[2] || b > bi[3] || c < bi[4] || c > bi[5]) return -1;
            return p.tix[(size_t)bi[6] + ((size_t)(a - bi[0]) * n3[1] + (b - bi[2])) * n3[2] + (c - bi[4])];
        };
        for (int d = 1; d < 8; ++d) {
            const int ua = wrap(p, 0, tk.a + (d & 1)), ub = wrap(p, 1, tk.b + ((d >> 1) & 1)),
                      uc = wrap(p, 2, tk.c + ((d >> 2) & 1));
            const int u = ticket_at(ua, ub, uc);
            if (u < 0) continue;
            const bool along_pec = (!per[0] && (d & 1)) || (!per[1] && (d & 2)) || (!per[2] && (d & 4));
            if (along_pec) CHECK(u < t, "upwind neighbour after its consumer (ticket %d, dir %d)", t, d);
        }
        // ring group key: band and the PEC coordinates
        std::tuple<int, int, int, int> g{tk.band, per[0] ? 0 : tk.a, per[1] ? 0 : tk.b, per[2] ? 0 : tk.c};
        if (g != cur_group) {
            CHECK(!done_groups.count(g), "ring group split (ticket %d)", t);
            if (std::get<0>(cur_group) >= 0) done_groups.insert(cur_group);
            cur_group = g;
        }
    }
    return true;
}

static bool check_merge(std::vector<Plan>& plans)
{
    std::vector<const Plan*> pp;
    for (auto& p : plans) pp.push_back(&p);
    Merged m;
    std::string err;
    CHECK(fdtd::plan::merge(pp.data(), (int)pp.size(), &m, &err), "merge failed: %s", err.c_str());
    size_t total = 0;
    for (auto& p : plans) total += p.tickets.size();
    CHECK(m.tickets.size() == total && m.tsim.size() == total, "merged sizes");
    // every grid's order is kept
    std::vector<size_t> next(plans.size(), 0);
    for (size_t t = 0; t < total; ++t) {
        const int g = m.tsim[t];
        CHECK(g >= 0 && g < (int)plans.size(), "grid index");
        const Ticket a = m.tickets[t], b = plans[g].tickets[next[g]++];
        CHECK(a.band == b.band && a.a == b.a && a.b == b.b && a.c == b.c, "grid order changed");
    }
    // consumers within D - 1 tickets of their producer, through the merged tables
    for (size_t t = 0; t < total; ++t) {
        const Plan& p = plans[m.tsim[t]];
        const Ticket q = m.tickets[t];
        const int* bi = &m.band[m.band_off[m.tsim[t]] + (size_t)kBandRec * q.band];
        const int nb = bi[3] - bi[2] + 1, nc = bi[5] - bi[4] + 1;
        for (int d = 1; d < 8; ++d) {
            const int v[3] = {wrap(p, 0, q.a - (d & 1)), wrap(p, 1, q.b - ((d >> 1) & 1)), wrap(p, 2, q.c - ((d >> 2) & 1))};
            if (v[0] < bi[0] || v[0] > bi[1] || v[1] < bi[2] || v[1] > bi[3] || v[2] < bi[4] || v[2] > bi[5]) continue;
            const size_t q2 = (size_t)bi[6] + ((size_t)(v[0] - bi[0]) * nb + (v[1] - bi[2])) * nc + (v[2] - bi[4]);
            CHECK(q2 < m.tix.size(), "merged tix range");
            const int j = m.tix[q2];
            CHECK(m.tsim[j] == m.tsim[t], "consumer in another grid");
            CHECK(j - (int)t + 1 <= m.D, "consumer beyond D");
        }
    }
    int group = 1;
    for (auto& p : plans) group = std::max(group, p.group);
    CHECK(m.group == group, "largest group");
    return true;
}

int main()
{
    struct Case {
        int N[3], per[3], W[3], nsteps, K;
    };
    const Case cases[] = {
        {{8, 8, 8}, {0, 0, 0}, {15, 15, 15}, 5, 5},
        {{40, 36, 34}, {0, 0, 0}, {15, 15, 15}, 20, 8},
        {{1, 6, 11}, {0, 0, 0}, {15, 15, 15}, 7, 3},
        {{31, 47, 29}, {0, 0, 0}, {11, 15, 15}, 33, 16},
        {{16, 20, 50}, {1, 0, 1}, {15, 15, 15}, 21, 8},
        {{30, 30, 30}, {1, 1, 1}, {15, 15, 15}, 17, 6},
        {{46, 16, 45}, {0, 1, 0}, {11, 15, 15}, 12, 12},
        {{64, 64, 64}, {0, 0, 0}, {15, 15, 15}, 100, 24},
        {{256, 256, 256}, {1, 1, 0}, {15, 15, 15}, 64, 48},
        {{128, 96, 80}, {0, 0, 0}, {15, 15, 15}, 128, 64},
        // the 19-wide tile: PEC, a 256^3 grid periodic in x and y (ring groups
        // of 14 x 18 tiles, a ragged width-9 x tile), every axis periodic
        {{83, 45, 52}, {0, 0, 0}, {19, 15, 15}, 60, 24},
        {{256, 256, 256}, {1, 1, 0}, {19, 15, 15}, 64, 64},
        {{40, 33, 36}, {1, 1, 1}, {19, 15, 15}, 60, 32},
    };
    std::vector<Plan> plans;
    for (const Case& c : cases) {
        Plan p;
        if (!check_plan(c.N, c.per, c.W, c.nsteps, c.K, &p)) {
            fprintf(stderr, "case N=%dx%dx%d per=%d%d%d K=%d nsteps=%d\n", c.N[0], c.N[1], c.N[2], c.per[0],
                    c.per[1], c.per[2], c.K, c.nsteps);
            return 1;
        }
        const double cost = fdtd::plan::band_cost(c.N, c.per, c.W, c.K);
        if (!(cost >= 1.0 && isfinite(cost))) {
            fprintf(stderr, "band cost %g\n", cost);
            return 1;
        }
        // other dequeue orders: weighted depth keys and slabs along each axis
        const int orders[][5] = {{1, 1, 3, -1, 0}, {4, 4, 1, -1, 0}, {1, 1, 1, 1, 2}, {2, 1, 1, 0, 1}, {1, 3, 2, 2, 3}};
        for (const auto& o : orders) {
            fdtd::plan::Order ord;
            for (int d = 0; d < 3; ++d) ord.w[d] = o[d];
            ord.slab_axis = o[3];
            ord.slab = o[4];
            Plan q;
            if (!check_plan(c.N, c.per, c.W, c.nsteps, c.K, &q, ord)) {
                fprintf(stderr, "order %d,%d,%d slab %d:%d\n", o[0], o[1], o[2], o[3], o[4]);
                return 1;
            }
        }
        if (c.N[0] <= 64) plans.push_back(std::move(p));
    }
    if (!check_merge(plans)) return 1;
    std::vector<Plan> one(1);
    one[0] = plans[1];
    if (!check_merge(one)) return 1;
    printf("plan checks passed (%zu cases)\n", sizeof(cases) / sizeof(cases[0]));
    return g_fail;
}
