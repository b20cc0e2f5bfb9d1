// Host-side plan of the systolic scheme's persistent launch: which (band,
// tile) tickets exist, the order in which workgroups take them, and the
// tables the kernel uses to find a neighbour's ticket.  Plain C++ (no HIP
// types), so that it also builds for the host alone (sanitizer checks).
//
// Traversal (paper, Section 3): tiles move one cell along the x-y-z-t
// diagonal per step, so every dependency between tiles points upwind (+x,
// +y, +z).  A call of nsteps steps is cut into bands of K steps; within a
// band each tile is one ticket, and tickets are ordered by band, then by
// depth below the most upwind corner along the PEC axes (upwind first), with
// the tiles that differ only along periodic axes (a ring group) contiguous.
#pragma once

#include <stddef.h>

#include <string>
#include <vector>

namespace fdtd {
namespace plan {

// One ticket: band index and tile coordinates (the layout of a HIP int4).
struct Ticket {
    int band, a, b, c;
};

// Band record layout: alo ahi blo bhi clo chi tix_off pad (tile ranges of the
// band; tix_off = offset of the band's tile -> ticket table).
constexpr int kBandRec = 8;

struct Plan {
    int nsteps = -1, K = -1, wx = -1;  // call length, band, tile width along x
    int nt = 0, nbands = 0;
    int per[3] = {0, 0, 0};  // periodic axes
    int L[3] = {0, 0, 0};    // tiles of the ring on periodic axes
    int group = 1;           // tiles of one ring group (must be co-resident)
    std::vector<Ticket> tickets;  // in dequeue order
    std::vector<int> tix;         // per band, tile -> ticket
    std::vector<int> band;        // kBandRec ints per band
    std::vector<int> depth;       // per ticket: depth below the upwind corner (PEC axes)
};

// Dequeue order of the tiles of a band.  Tiles are sorted (stably, ring
// groups staying whole) by the key
//     slab-major:  (slabs - 1 - i_s / slab) * (kmax + 1) + sum_d w[d] (n_d - 1 - i_d)
// where i_d is the tile's index in the band's range along PEC axis d, n_d
// the range's length, and the slab term applies when slab_axis names a PEC
// axis (slab > 0).  Any positive weights keep every upwind neighbour (along
// PEC axes) earlier, and so does cutting one axis into slabs taken from its
// upwind end: w = (1, 1, 1) without slabs is the plain depth below the most
// upwind corner.
struct Order {
    int w[3] = {1, 1, 1};
    int slab_axis = -1;
    int slab = 0;
};

// Build the plan of one grid: N cells per axis, per[d] = 1 on periodic axes,
// W updated cells per tile and axis, a call of nsteps steps in bands of K.
// Returns false (with *err) when the plan would exceed 2^30 tickets.
bool build(const int N[3], const int per[3], const int W[3], int nsteps, int K, Plan* out,
           std::string* err, const Order& order = Order());

// The plans of several grids merged into one launch order: tickets by band
// start step, then by grid, each grid keeping its own order.  D = the largest
// producer -> consumer ticket distance (consumers are the seven downwind
// neighbours); group = the largest ring group.
struct Merged {
    std::vector<Ticket> tickets;
    std::vector<int> tsim;          // grid of each ticket
    std::vector<int> tix;           // per grid and band, tile -> merged ticket
    std::vector<int> band;          // band records, tix_off into the merged table
    std::vector<size_t> band_off;   // per grid: offset of its band records
    int D = 1, group = 1;
};

bool merge(const Plan* const* plans, int n, Merged* out, std::string* err);

// Band-length cost model: relative cost per cell update of bands of K steps
// on a grid (tile-steps covering the band's skewed space-time region, times
// the band's start and end), see the definition.
double band_cost(const int N[3], const int per[3], const int W[3], int K);

}  // namespace plan
}  // namespace fdtd
