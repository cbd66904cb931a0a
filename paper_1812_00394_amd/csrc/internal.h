// Internal declarations shared by the host preprocessing and the device library.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fvlbm.h"

namespace fvlbm {

// An error carrying the status the C ABI returns.
struct Error : std::runtime_error {
    fvlbm_status status;
    Error(fvlbm_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

void set_last_error(const std::string &msg);

constexpr int kSlots = 4;               // at most four edges per cell (triangles and quads)
constexpr int kTile = 256;              // cells per tile of the fused stage kernels (one workgroup)
constexpr double kNoWallDistance = 1e30;

}  // namespace fvlbm

// Host-side mesh after preprocessing.  Everything is in the internal (renumbered) cell order;
// per-edge ("slot") arrays are structure-of-arrays [kSlots][n] so that one thread per cell reads
// them coalesced.  Slot s of cell c:
//   nbr  >= 0  : internal index of the neighbour across the edge
//        == -1 : unused slot (triangle)
//        <= -2 : boundary edge number b = -2 - nbr in the internal boundary-edge list
//   nl   outward normal times edge length
//   rf   edge midpoint minus the cell centroid
//   d    stencil point minus the cell centroid: neighbour centroid (periodic image) or edge midpoint
//   c    weighted least-squares coefficient: grad phi_c = sum_s c_s (phi_s - phi_c)
struct fvlbm_mesh {
    int64_t n = 0;
    int64_t n_nodes = 0;
    int32_t n_groups = 0;
    int32_t kinds[FVLBM_MAX_GROUPS] = {};
    int64_t n_bfaces_user = 0;
    int64_t n_interior_edges = 0;
    int64_t n_boundary_edges = 0;
    int32_t max_faces = 0;
    std::vector<int64_t> perm;   // internal -> user
    std::vector<int64_t> iperm;  // user -> internal
    std::vector<double> area, xc, yc, wdist;
    std::vector<int32_t> nbr;
    std::vector<int8_t> rev;     // [kSlots][n]: slot of the neighbour that points back (interior slots)
    std::vector<double> nlx, nly, rfx, rfy, dx, dy, cx, cy;
    std::vector<double> mi00, mi01, mi11;   // [n] inverse of the weighted least-squares matrix
    std::vector<double> tri_p;              // [6][n] triangle vertices minus the centroid (x0, y0, x1, y1, x2, y2)
    std::vector<int32_t> bfirst;            // [n] first boundary edge of the cell, -1 if none
    // boundary edges (periodic ones excluded), ordered by internal owner cell then slot
    std::vector<int32_t> b_cell, b_group, b_kind;
    std::vector<int64_t> b_user;  // index into the caller's boundary-edge arrays
    std::vector<double> b_nx, b_ny, b_l, b_dperp, b_xfx, b_xfy;
    // tiles of kTile consecutive internal cells: the halo of tile t (interior neighbours of its
    // cells that lie outside it, ascending) is halo_cell[halo_ptr[t] .. halo_ptr[t+1]); lnb[s][c]
    // is the tile-local index of slot s's neighbour: c' - tile start inside the tile, kTile + its
    // position in the halo outside it; -1 for an unused slot, -2 - k for the cell's k-th boundary
    // edge (edge number bfirst[c] + k)
    int32_t n_tiles = 0, halo_max = 0;
    std::vector<int32_t> halo_ptr, halo_cell;
    std::vector<int16_t> lnb;
    // extended halo of tile t: ext_cell[ext_ptr[t] .. ext_ptr[t+1]) lists ring 1 (the halo above,
    // ext_n1[t] cells) then ring 2 (interior neighbours of ring-1 cells outside the tile and ring 1,
    // ascending); ext_lnb[s][e] is the tile-local column of slot s's neighbour of ring-1 entry e
    // (tile cells c - tile start, ext entry j kTile + j; -1 unused, -2 - k the k-th boundary edge)
    int32_t ext_max = 0;
    std::vector<int32_t> ext_ptr, ext_n1, ext_cell;
    std::vector<int16_t> ext_lnb;
};
