// D2Q9 lattice and the device-side building blocks of the FVLBM step.
//
// Distribution functions are stored as deviations from the rest state, d_a = f_a - w_a rho0, in
// the storage type T (double, or float for the FP32-deviation mode); the equilibrium, the ghost
// states and the stage collision are written for deviations so that the large constant w_a rho0
// never enters a rounding (the constant cancels exactly in every linear operation of the step).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dual.h"

namespace fvlbm {

enum : int32_t { kWall = 1, kMovingWall = 2, kInlet = 3, kOutlet = 4, kFarfield = 5 };

// Scalar constants for generic code: S is float, double or a dual number over one of them.
template <class S>
struct ScalarBase {
    using type = S;
};
template <class T, int K>
struct ScalarBase<Dual<T, K>> {
    using type = T;
};
template <class S>
__device__ __forceinline__ S cst(double x) { return S(typename ScalarBase<S>::type(x)); }

// 1 / x.  FP32: the hardware reciprocal (v_rcp_f32, within 1 ulp), one instruction instead of the
// correctly rounded division sequence; its error is below the FP32 rounding of the quantities it
// scales.  Dual numbers: the division.
template <class S>
__device__ __forceinline__ S recip(S x) { return cst<S>(1) / x; }
template <>
__device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64: the hardware reciprocal estimate (v_rcp_f64) refined by two steps of Newton's iteration for
// 1/x, r <- r + r (1 - x r), each of which squares the relative error, instead of the IEEE division
// sequence (measured on gfx950: the correctly rounded 1/x for 4.2M random x over 24 decades; the
// FP64 step 2 % faster).  x = 0 gives NaN where the division gives infinity: non-finite either way.
template <>
__device__ __forceinline__ double recip<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
    return r;
}

// Lattice velocities of Qian's D2Q9 model and their weights (a = 0 rest, 1-4 axes, 5-8 diagonals).
__host__ __device__ constexpr int ex(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0); }
__host__ __device__ constexpr int ey(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0); }
template <typename T>
__host__ __device__ constexpr T wt(int a) {
    return a == 0 ? T(4) / T(9) : (a < 5 ? T(1) / T(9) : T(1) / T(36));
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD b mod 8).  This maps
// them so that each XCD processes one contiguous range of blocks; with cells in space-filling-curve
// order its neighbour gathers then hit its own L2 instead of being fetched again by another XCD.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// The tile of a ring-tiled launch, the tiles in ascending order (FWD) or descending.  The stage
// sweeps alternate: stages 1 and 3 (and the explicit scheme's sweep) run descending (each XCD its
// own range), the SST and stage 2 ascending, so that each launch starts on the tiles whose data the launch before it wrote
// last, which the caches (each XCD's L2 and the 256 MB last-level cache) still hold (measured on the
// 4.0M-cell mesh: 0.662 -> 0.625 ms per FP32-deviation step).  The reverse alternates likewise.
template <bool FWD>
__device__ __forceinline__ int ring_tile() {
    if constexpr (FWD) return xcd_block(blockIdx.x, gridDim.x);
    // each XCD keeps its contiguous range of tiles (and its L2's data) and runs it backwards
    const int nb = gridDim.x, q = nb >> 3, r = nb & 7;
    const int x = blockIdx.x & 7, i = blockIdx.x >> 3;
    const int cnt = q + (x < r ? 1 : 0);
    return x * q + (x < r ? x : r) + (cnt - 1 - i);
}

__device__ __forceinline__ int cell_index() { return xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; }

// Geometry and boundary data on the device (pointers into the caller's workspace).  The per-edge
// arrays a sweep streams are held in the arithmetic type T of the state (FP64 masters of every
// quantity stay on the host and in the FP64 fields below): nl = outward normal x length,
// rf = x_f - x_c, q = x_f - x_N' (from the neighbour's centroid image), c = LSQ coefficients.
// FP64 copies of the geometry the ring sweeps stream, for FP32-deviation states that keep geometry
// and least-squares data in FP64 on the GPU (precision FVLBM_FP32_DEV_GEO64).  The members carry
// the names of Geo<double>'s, so one function forms the edge data from either.
struct GeoF64 {
    int32_t n;
    const double *nlx, *nly, *rfx, *rfy, *qx, *qy, *cx, *cy;         // [4][n]
    const double *inv_area;                                          // [n]
    const double *mi;                                                // [3][n]
    const double *tp;                                                // [6][n]
    const int32_t *bfirst;                                           // [n]
};

template <typename T>
struct Geo {
    int32_t n;    // cells
    int32_t nb;   // boundary edges
    const int32_t *nbr;                                              // [4][n]
    const T *nlx, *nly, *rfx, *rfy, *qx, *qy, *cx, *cy;              // [4][n]
    const T *inv_area;                                               // [n]
    const T *mi;                                                     // [3][n] inverse LSQ matrix: 00, 01, 11
    const T *tp;                                                     // [6][n] triangle vertices - centroid
    const int32_t *bfirst;                                           // [n] first boundary edge, -1 if none
    const double *area, *wdist;                                      // [n]
    const int32_t *perm;                                             // [n] internal -> user
    const int32_t *b_kind, *b_cell;                                  // [nb]
    const double *b_nx, *b_ny, *b_l, *b_dperp, *b_xfx;               // [nb]
    const double *b_ux, *b_uy, *b_rho, *b_drho, *b_k, *b_w;          // [nb] boundary values
    const int32_t *b_group;                                          // [nb]
    GeoF64 g64;                                                      // FP32_DEV_GEO64 only
};

// Equilibrium deviation f_eq,a(rho, u) - w_a rho0, with drho = rho - rho0 (second-order D2Q9
// equilibrium w_a rho (1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2)).
template <typename S>
__device__ __forceinline__ S dfeq(int a, S drho, S rho, S ux, S uy) {
    S eu = cst<S>(ex(a)) * ux + cst<S>(ey(a)) * uy;
    return cst<S>(a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0)) *
           (drho + rho * (cst<S>(3) * eu + cst<S>(4.5) * eu * eu - cst<S>(1.5) * (ux * ux + uy * uy)));
}

// Density deviation and velocity of a deviation vector (the collision invariants 1, e_x, e_y).
template <typename S>
__device__ __forceinline__ void moments(const S d[9], S rho0, S &drho, S &rho, S &ux, S &uy) {
    S s = cst<S>(0), jx = cst<S>(0), jy = cst<S>(0);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        s = s + d[a];
        jx = jx + cst<S>(ex(a)) * d[a];
        jy = jy + cst<S>(ey(a)) * d[a];
    }
    drho = s;
    rho = rho0 + s;
    const S r = recip(rho);
    ux = jx * r;
    uy = jy * r;
}

// Implicit stage of the IMEX scheme, solved explicitly: the stage moments equal those of rhs
// (the collision term has zero invariant moments), so f = (rhs + a f_eq) / (1 + a) with
// a = dt m_JJ / tau.  Also returns the equilibrium used.
template <typename T>
__device__ __forceinline__ void stage_collide(const T rhs[9], T a, T rho0, T out[9], T fe[9]) {
    T drho, rho, ux, uy;
    moments(rhs, rho0, drho, rho, ux, uy);
    const T inv = recip(T(1) + a);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        fe[q] = dfeq(q, drho, rho, ux, uy);
        out[q] = (rhs[q] + a * fe[q]) * inv;
    }
}

// The same stage solve with the stage moments given (Eq. (sumimeximplicitnew): they follow from f^n
// and the earlier convection terms alone, never from the collision terms, whose invariant moments
// vanish only up to rounding and would be amplified by dt / tau).
template <typename T>
__device__ __forceinline__ void stage_collide_m(const T rhs[9], T a, T drho, T rho, T ux, T uy, T out[9]) {
    const T inv = recip(T(1) + a);
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = (rhs[q] + a * dfeq(q, drho, rho, ux, uy)) * inv;
}

// Ghost deviation at the midpoint of boundary edge b of a cell whose state is gc (moments drho,
// rho, ux, uy), non-equilibrium extrapolation from the cell:
//   walls: f_eq(rho_c, u_w) + (g_c - f_eq(rho_c, u_c)) for every direction;
//   inlet / outlet / far field: replaced for incoming directions (e.n < 0) only.
// The ghost state for a boundary edge of the given kind, boundary velocity ub and density rb
// (drb = rb - rho0); generic in the scalar type S (the adjoint evaluates it on dual numbers).
template <typename S, typename T>
__device__ __forceinline__ void ghost_state(int kind, S ubx, S uby, S rb, S drb, T nlx, T nly, const S gc[9], S drho,
                                            S rho, S ux, S uy, S gb[9]) {
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const T en = T(ex(a)) * nlx + T(ey(a)) * nly;
        const S neq = gc[a] - dfeq(a, drho, rho, ux, uy);
        S v;
        if (kind == kWall || kind == kMovingWall) {
            v = dfeq(a, drho, rho, ubx, uby) + neq;
        } else if (en < T(0)) {
            if (kind == kInlet)
                v = dfeq(a, drho, rho, ubx, uby) + neq;
            else if (kind == kOutlet)
                v = dfeq(a, drb, rb, ux, uy) + neq;
            else
                v = dfeq(a, drb, rb, ubx, uby);
        } else {
            v = gc[a];
        }
        gb[a] = v;
    }
}

template <typename T>
__device__ __forceinline__ void ghost(const Geo<T> &g, int b, T nlx, T nly, const T gc[9], T drho, T rho, T ux,
                                      T uy, T gb[9]) {
    ghost_state<T, T>(g.b_kind[b], T(g.b_ux[b]), T(g.b_uy[b]), T(g.b_rho[b]), T(g.b_drho[b]), nlx, nly, gc, drho, rho,
                      ux, uy, gb);
}

}  // namespace fvlbm
