// HIP kernels of one IMEX step (gfx950).  Cells are renumbered along a space-filling curve so that
// neighbour gathers of a wavefront hit a few cache lines.  The ring-tiled kernels (k_sst_ring,
// k_stage_ring) are the main path; the one-thread-per-cell kernels below them are its fallbacks.
//
// Per step (Section 3.2 algorithm, SST once per step before the stages):
//   sst      LSQ gradients of u, v, k, omega; S, div u, CD, F1, F2, mu_t, blending, sources; k /
//            omega face fluxes (2nd-order upwind convection, central diffusion), point-implicit
//            update, nu_t from the updated k, omega, tau = 3 (nu + nu_t)        [Eq. (turbtau)]
//            (fallback: sst_a, sst_b)
//   sweep<J> convection term of stage J [Eq. (advection)] fused with the cell-local epilogue:
//            J=1: f^(1) = solve(f^n) on the fly [Eq. (fnewstage)], its convection term Ga1,
//                 f^(2) = solve(f^n + dt/2 Ga1)          (stores Ga1 unless stage 2 recovers it)
//            J=2: f^(3) = solve(f^n + dt/2 (Ga1+Ga2) + dt/3 (Gc1+Gc2));  Q = f^(3) - dt/6 (Ga1+Ga2)
//            J=3: f^{n+1} = Q + dt/3 Ga3                    (= Eq. (imextwo), see below)
//            (fallback: collide1 writes f^(1), grad writes the 16 gradient planes, sweep reads them)
// Eq. (imextwo) with n~ = n = 1/3: f^{n+1} = f^n + dt/3 sum Ga + dt/3 sum Gc.  Since the third
// stage satisfies f^(3) = rhs3 + dt/3 Gc3 and rhs3 = f^n + dt/2 (Ga1+Ga2) + dt/3 (Gc1+Gc2), this is
// f^{n+1} = f^(3) + dt/3 Ga3 - dt/6 (Ga1 + Ga2): no stored collision terms are needed.
#pragma once

#include "lattice.h"

namespace fvlbm {

template <typename T>
struct StepPar {
    T rho0, dt, nu;
    T a1, bstar, sk1, sk2, sw1, sw2, b1, b2, kappa;
    int limiter;   // 1: keep interior face values of f between the two cells' values (reading r32);
                   // 2: Barth and Jespersen's gradient limiter (reading r35)
    int recover;   // stage 2 recovers Ga1 from f^(2) instead of reading it (stage 1 does not store it)
};

// ----------------------------------------------------------------------------------------------
// Least-squares gradient of the eight moving directions of a stage field.
// G layout: plane 2(a-1) = d/dx, 2(a-1)+1 = d/dy of direction a, each [n].
// ----------------------------------------------------------------------------------------------
// LSQ gradient of the eight moving directions of one cell: gc receives the cell's own values,
// gx / gy the gradients (index 1..8).  Boundary edges contribute their ghost state.
template <typename T>
__device__ __forceinline__ void grad_cell(const Geo<T> &g, const T *__restrict__ f, int cell, T rho0, T gc[9], T gx[9],
                                          T gy[9]) {
    const int n = g.n;
#pragma unroll
    for (int a = 0; a < 9; ++a) gc[a] = f[(size_t)a * n + cell];
#pragma unroll
    for (int a = 0; a < 9; ++a) gx[a] = gy[a] = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + cell;
        const int nb = g.nbr[si];
        if (nb == -1) continue;
        const T cxs = g.cx[si], cys = g.cy[si];
        if (nb >= 0) {
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T d = f[(size_t)a * n + nb] - gc[a];
                gx[a] += cxs * d;
                gy[a] += cys * d;
            }
        } else {
            T drho, rho, ux, uy, gb[9];
            moments(gc, rho0, drho, rho, ux, uy);
            ghost(g, -2 - nb, g.nlx[si], g.nly[si], gc, drho, rho, ux, uy, gb);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T d = gb[a] - gc[a];
                gx[a] += cxs * d;
                gy[a] += cys * d;
            }
        }
    }
}

// Gradient planes of a stage field: plane 2(a-1) = d/dx, 2(a-1)+1 = d/dy of direction a, each [n].
template <typename T>
__global__ void __launch_bounds__(256) k_grad(Geo<T> g, const T *__restrict__ f, T *__restrict__ G, T rho0) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T gc[9], gx[9], gy[9];
    grad_cell(g, f, c, rho0, gc, gx, gy);
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        G[(size_t)(2 * (a - 1)) * n + c] = gx[a];
        G[(size_t)(2 * (a - 1) + 1) * n + c] = gy[a];
    }
}

// Neighbour access of the convection term: the upwind neighbour's value extrapolated to the edge
// midpoint, g_N + grad g_N . q.  From the global gradient planes, or from the tile's LDS copy.
template <typename T>
struct NbrGlobal {
    const T *f, *G;
    int n;
    __device__ __forceinline__ void slot(int, int) {}
    __device__ __forceinline__ T recon(int a, int nb, T qx, T qy) const {
        return f[(size_t)a * n + nb] + G[(size_t)(2 * (a - 1)) * n + nb] * qx + G[(size_t)(2 * (a - 1) + 1) * n + nb] * qy;
    }
    __device__ __forceinline__ T value(int a, int nb) const { return f[(size_t)a * n + nb]; }
};

template <typename T>
struct NbrTile {
    const T *f;
    const T *L;            // LDS gradient planes [16][W]
    const int16_t *lnb;    // tile-local neighbour index per slot
    int n, W, loc;
    __device__ __forceinline__ void slot(int s, int c) { loc = lnb[(size_t)s * n + c]; }
    __device__ __forceinline__ T recon(int a, int nb, T qx, T qy) const {
        return f[(size_t)a * n + nb] + L[(2 * (a - 1)) * W + loc] * qx + L[(2 * (a - 1) + 1) * W + loc] * qy;
    }
    __device__ __forceinline__ T value(int a, int nb) const { return f[(size_t)a * n + nb]; }
};

// Convection term of cell c (Eq. (advection)): -(1/A) sum over edges of (e.n) dl times the face
// value, the face value being the upwind cell's value extrapolated to the edge midpoint with its
// LSQ gradient; on walls the ghost state, on open boundaries the ghost state for incoming
// directions.  gc: the cell's own values; out[0] = 0 (the rest direction does not move).
// The limited face value: v kept between the values of the two cells sharing the edge.
template <typename T>
__device__ __forceinline__ T clip_between(T v, T a, T b) {
    const T lo = a <= b ? a : b, hi = a <= b ? b : a;
    return v < lo ? lo : (v > hi ? hi : v);
}
// FP32: the clip is the median of the three values (one v_med3_f32)
template <>
__device__ __forceinline__ float clip_between<float>(float v, float a, float b) { return __builtin_amdgcn_fmed3f(v, a, b); }

template <typename T, typename Nbr>
__device__ __forceinline__ void advect_cell(const Geo<T> &g, int c, T rho0, const T gc[9], const T gxc[9], const T gyc[9],
                                            Nbr nbr_acc, T out[9], int limiter = 0) {
    const int n = g.n;
    T acc[9];
#pragma unroll
    for (int a = 1; a < 9; ++a) acc[a] = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        if (nb == -1) continue;
        const T nlx = g.nlx[si], nly = g.nly[si];
        const T rx = g.rfx[si], ry = g.rfy[si];
        if (nb >= 0) {
            nbr_acc.slot(s, c);
            const T qx = g.qx[si], qy = g.qy[si];
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T end = T(ex(a)) * nlx + T(ey(a)) * nly;
                T val = end >= T(0) ? gc[a] + gxc[a] * rx + gyc[a] * ry : nbr_acc.recon(a, nb, qx, qy);
                if (limiter == 1) val = clip_between(val, gc[a], nbr_acc.value(a, nb));
                acc[a] += end * val;
            }
        } else {
            const int b = -2 - nb;
            T drho, rho, ux, uy, gb[9];
            moments(gc, rho0, drho, rho, ux, uy);
            ghost(g, b, nlx, nly, gc, drho, rho, ux, uy, gb);
            const int kind = g.b_kind[b];
            const bool wall = (kind == kWall || kind == kMovingWall);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T end = T(ex(a)) * nlx + T(ey(a)) * nly;
                const T val = (wall || end < T(0)) ? gb[a] : gc[a] + gxc[a] * rx + gyc[a] * ry;
                acc[a] += end * val;
            }
        }
    }
    const T ia = g.inv_area[c];
    out[0] = T(0);
#pragma unroll
    for (int a = 1; a < 9; ++a) out[a] = -acc[a] * ia;
}

// Convection term of cell c from the global gradient planes (gc = the cell's own values).
template <typename T>
__device__ __forceinline__ void advect_cell_global(const Geo<T> &g, const T *__restrict__ f, const T *__restrict__ G,
                                                   int c, T rho0, const T gc[9], T out[9], int limiter) {
    const int n = g.n;
    T gxc[9], gyc[9];
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        gxc[a] = G[(size_t)(2 * (a - 1)) * n + c];
        gyc[a] = G[(size_t)(2 * (a - 1) + 1) * n + c];
    }
    advect_cell(g, c, rho0, gc, gxc, gyc, NbrGlobal<T>{f, G, n}, out, limiter);
}

// f^(1) = stage solve of f^n with a = dt/(4 tau).
template <typename T>
__global__ void __launch_bounds__(256) k_collide1(int n, const T *__restrict__ F, const T *__restrict__ tau,
                                                  T *__restrict__ X, StepPar<T> p) {
    const int c = cell_index();
    if (c >= n) return;
    T fn[9], f1[9], fe[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fn[a] = F[(size_t)a * n + c];
    stage_collide(fn, p.dt * T(0.25) * recip(tau[c]), p.rho0, f1, fe);
#pragma unroll
    for (int a = 0; a < 9; ++a) X[(size_t)a * n + c] = f1[a];
}

// ---- stage epilogues (cell-local), shared by every sweep variant ----
// Operands an epilogue reads besides the stage field: f^n and tau (stages 1, 2), the stored
// convection term Ga1 (stage 2) or Q (stage 3).  Loaded by the caller so that a kernel can issue
// the loads early; members a stage does not use are dead code.
template <typename T>
struct EpiOps {
    T fn[9], a[9], tc, tc3;
};

// Buffers of one stage sweep: src = the stage field whose convection term is taken.  M: stage 3
// writes rho - rho0, u there; stage 1 writes the moments of f^(2) there when given (the per-stage
// SST reads them).  tau3: the third stage's relaxation time when it differs (per-stage SST).
template <typename T>
struct StageBufs {
    const T *src, *F_in, *tau;
    T *A, *out, *F_out, *M;
    const T *tau3;
    // with the face-value limiter of r32, while a step is recorded for the adjoint: per cell the
    // state of every interior edge's clip, 2 bits per edge slot s and direction a at bit
    // 2 (8 s + a - 1): clipped, and (if clipped) the bound is the cell's own value
    uint64_t *clip;
};

template <typename T, int J>
__device__ __forceinline__ void load_ops(const StageBufs<T> &b, int c, int n, EpiOps<T> &o, int recover) {
    if constexpr (J == 0) o.tc = b.tau[c];
    if constexpr (J == 1 || J == 2) {
#pragma unroll
        for (int a = 0; a < 9; ++a) o.fn[a] = b.F_in[(size_t)a * n + c];
        o.tc = b.tau[c];
    }
    if constexpr (J == 3) {
#pragma unroll
        for (int a = 0; a < 9; ++a) o.a[a] = b.A[(size_t)a * n + c];
    }
    if constexpr (J == 2) {
        if (!recover) {
#pragma unroll
            for (int a = 0; a < 9; ++a) o.a[a] = b.A[(size_t)a * n + c];
        }
        o.tc3 = b.tau3 ? b.tau3[c] : o.tc;
    }
}

// Stage 1 -> 2: f^(2) = solve(f^n + dt/2 Ga1, a = dt/(4 tau)); stores f^(2), and Ga1 unless stage 2
// recovers it.
template <typename T>
__device__ __forceinline__ void epilogue1(int c, int n, const T ga[9], const EpiOps<T> &o, T *__restrict__ Y,
                                          T *__restrict__ A, T *__restrict__ M2, const StepPar<T> &p) {
    T rhs[9], f2[9], fe[9];
    const T h = p.dt * T(0.5);
#pragma unroll
    for (int a = 0; a < 9; ++a) rhs[a] = o.fn[a] + h * ga[a];
    stage_collide(rhs, p.dt * T(0.25) * recip(o.tc), p.rho0, f2, fe);
#pragma unroll
    for (int a = 0; a < 9; ++a) Y[(size_t)a * n + c] = f2[a];
    if (!p.recover) {
#pragma unroll
        for (int a = 0; a < 9; ++a) A[(size_t)a * n + c] = ga[a];
    }
    if (M2) {
        // the stage-2 macro variables, for the third stage's SST
        T drho, rho, ux, uy;
        moments(f2, p.rho0, drho, rho, ux, uy);
        M2[c] = drho;
        M2[(size_t)n + c] = ux;
        M2[(size_t)2 * n + c] = uy;
    }
}

// Stage 2 -> 3: Gc1, Gc2 recomputed cell-locally; f^(3) = solve(rhs3, dt/(3 tau)) with the stage
// moments of Eq. (sumimeximplicitnew); stores f^(3) and Q = f^(3) - dt/6 (Ga1 + Ga2) (over Ga1).
// Ga1 is read, or recovered from the stage-2 solve: f^(2) = (rhs2 + a f_eq(f^(2))) / (1 + a) with
// rhs2 = f^n + dt/2 Ga1 and a = dt/(4 tau), so Ga1 = (2/dt) (f^(2) + a (f^(2) - f_eq(f^(2))) - f^n).
// The recovery amplifies the rounding of f^(2) by 1 + a; the host enables it for a <= 4 only.
template <typename T>
__device__ __forceinline__ void epilogue2(int c, int n, const T f2[9], const T ga2[9], const EpiOps<T> &o,
                                          T *__restrict__ X, T *__restrict__ A, const StepPar<T> &p) {
    T f1[9], fe1[9], rhs[9], f3[9], gsum[9];
    const T tc = o.tc;
    const T itau = recip(tc);
    const T a12 = p.dt * T(0.25) * itau;                         // a of stages 1 and 2
    stage_collide(o.fn, a12, p.rho0, f1, fe1);                   // f^(1), f_eq^(1)
    T drho2, rho2, ux2, uy2;
    moments(f2, p.rho0, drho2, rho2, ux2, uy2);                  // stage-2 moments
    const T h2 = p.dt * T(0.5), h3 = p.dt * T(1.0 / 3.0);
    const T i_h2 = T(2) * recip(p.dt);
    // stage-3 moments from f^n and the convection terms (Eq. (sumimeximplicitnew))
    T m0 = 0, mx = 0, my = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const T fe2 = dfeq(a, drho2, rho2, ux2, uy2);
        const T gc1 = (fe1[a] - f1[a]) * itau;
        const T gc2 = (fe2 - f2[a]) * itau;
        const T ga1 = p.recover ? (f2[a] + a12 * (f2[a] - fe2) - o.fn[a]) * i_h2 : o.a[a];
        gsum[a] = ga1 + ga2[a];                                    // Ga1 + Ga2
        rhs[a] = o.fn[a] + h2 * gsum[a] + h3 * (gc1 + gc2);
        const T mv = o.fn[a] + h2 * gsum[a];
        m0 += mv;
        mx += T(ex(a)) * mv;
        my += T(ey(a)) * mv;
    }
    const T rho3 = p.rho0 + m0;
    const T ir3 = recip(rho3);
    stage_collide_m(rhs, h3 * recip(o.tc3), m0, rho3, mx * ir3, my * ir3, f3);
    const T h6 = p.dt * T(1.0 / 6.0);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        X[(size_t)a * n + c] = f3[a];
        A[(size_t)a * n + c] = f3[a] - h6 * gsum[a];
    }
}

// Stage 3 -> n+1: f^{n+1} = Q + dt/3 Ga3; macro variables (Step 7): rho - rho0, u.
template <typename T>
__device__ __forceinline__ void epilogue3(int c, int n, const T ga3[9], const EpiOps<T> &o, T *__restrict__ F,
                                          T *__restrict__ M, const StepPar<T> &p) {
    T fnew[9];
    const T h3 = p.dt * T(1.0 / 3.0);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        fnew[a] = o.a[a] + h3 * ga3[a];
        F[(size_t)a * n + c] = fnew[a];
    }
    T drho, rho, ux, uy;
    moments(fnew, p.rho0, drho, rho, ux, uy);
    M[c] = drho;
    M[(size_t)n + c] = ux;
    M[(size_t)2 * n + c] = uy;
}

// The explicit scheme (forward Euler of Eq. (semibgk)): f^{n+1} = f^n + dt (Ga + (f_eq - f^n) / tau)
// from the convection term Ga of f^n = gc; stores f^{n+1} and its macro variables.
template <typename T>
__device__ __forceinline__ void epilogue_explicit(int c, int n, const T gc[9], const T ga[9], const EpiOps<T> &o,
                                                  T *__restrict__ F, T *__restrict__ M, const StepPar<T> &p) {
    T drho, rho, ux, uy, fnew[9];
    moments(gc, p.rho0, drho, rho, ux, uy);
    const T itau = recip(o.tc);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        fnew[a] = gc[a] + p.dt * (ga[a] + (dfeq(a, drho, rho, ux, uy) - gc[a]) * itau);
        F[(size_t)a * n + c] = fnew[a];
    }
    moments(fnew, p.rho0, drho, rho, ux, uy);
    M[c] = drho;
    M[(size_t)n + c] = ux;
    M[(size_t)2 * n + c] = uy;
}

template <typename T, int J>
__device__ __forceinline__ void stage_epilogue_ops(int c, int n, const T gc[9], const T ga[9], const EpiOps<T> &o,
                                                   const StageBufs<T> &b, const StepPar<T> &p) {
    if constexpr (J == 0)
        epilogue_explicit(c, n, gc, ga, o, b.F_out, b.M, p);
    else if constexpr (J == 1)
        epilogue1(c, n, ga, o, b.out, b.A, b.M, p);
    else if constexpr (J == 2)
        epilogue2(c, n, gc, ga, o, b.out, b.A, p);
    else
        epilogue3(c, n, ga, o, b.F_out, b.M, p);
}

template <typename T, int J>
__device__ __forceinline__ void stage_epilogue(int c, int n, const T gc[9], const T ga[9], const StageBufs<T> &b,
                                               const StepPar<T> &p) {
    EpiOps<T> o;
    load_ops<T, J>(b, c, n, o, p.recover);
    stage_epilogue_ops<T, J>(c, n, gc, ga, o, b, p);
}

// Two-kernel sweep (after k_grad): the convection term of stage J from the global gradient planes.
//   J=1: src = f^(1), out = f^(2), A = Ga1
//   J=2: src = f^(2), out = f^(3), A: Ga1 -> Q
//   J=3: src = f^(3), A = Q, F_out = f^{n+1}, M = macro variables
template <typename T, int J>
__global__ void __launch_bounds__(256) k_sweep(Geo<T> g, const T *__restrict__ G, StageBufs<T> b, StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T gc[9], ga[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) gc[a] = b.src[(size_t)a * n + c];
    advect_cell_global(g, b.src, G, c, p.rho0, gc, ga, p.limiter);
    stage_epilogue<T, J>(c, n, gc, ga, b, p);
}

// ---- edge loop with atomics: the alternative to the cell loop, kept for the measured choice ----
// One thread per interior edge, each edge once (face code 4 c + s: slot s of cell c, the lower
// index of the two cells): the upwind face value of every moving direction from the gradient
// planes of k_grad (clipped between the two cells' values with the limiter of reading r32), and
// its flux (e.n) dl times the face value added to the outflow sum of c and subtracted from that of
// the neighbour with global atomics.  Consecutive edges belong to nearby cells; workgroups are
// mapped so that each XCD takes one contiguous range of edges.  acc ([8][n], directions 1..8)
// starts at zero.  The order in which the atomics add up differs from run to run, so results vary
// at rounding level, where the cell loop is deterministic.
template <typename T, bool LIM>
__global__ void __launch_bounds__(256) k_face_flux(Geo<T> g, const int32_t *__restrict__ faces, int nf,
                                                   const T *__restrict__ f, const T *__restrict__ G,
                                                   T *__restrict__ acc) {
    const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int code = faces[i];
    const int c = code >> 2, s = code & 3, n = g.n;
    const size_t si = (size_t)s * n + c;
    const int nb = g.nbr[si];
    const T nlx = g.nlx[si], nly = g.nly[si], rx = g.rfx[si], ry = g.rfy[si], qx = g.qx[si], qy = g.qy[si];
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const T end = T(ex(a)) * nlx + T(ey(a)) * nly;
        const size_t pa = (size_t)a * n, px = (size_t)(2 * (a - 1)) * n, py = px + n;
        const T vc = f[pa + c], vn = f[pa + nb];
        T val = end >= T(0) ? vc + G[px + c] * rx + G[py + c] * ry : vn + G[px + nb] * qx + G[py + nb] * qy;
        if constexpr (LIM) val = clip_between(val, vc, vn);
        const T flux = end * val;
        atomicAdd(&acc[(size_t)(a - 1) * n + c], flux);
        atomicAdd(&acc[(size_t)(a - 1) * n + nb], -flux);
    }
}

// After k_face_flux: the boundary edges of the cell (ghost states at walls and for incoming
// directions, the cell's own reconstruction for outgoing ones, as the cell loop), the convection
// term -(1/A) times the outflow sum, and the stage-J epilogue.
template <typename T, int J>
__global__ void __launch_bounds__(256) k_face_epilogue(Geo<T> g, const T *__restrict__ G, const T *__restrict__ acc,
                                                       StageBufs<T> b, StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T gc[9], sum[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) gc[a] = b.src[(size_t)a * n + c];
    sum[0] = T(0);
#pragma unroll
    for (int a = 1; a < 9; ++a) sum[a] = acc[(size_t)(a - 1) * n + c];
    if (g.bfirst[c] >= 0) {
        T drho, rho, ux, uy;
        moments(gc, p.rho0, drho, rho, ux, uy);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const size_t si = (size_t)s * n + c;
            const int nb = g.nbr[si];
            if (nb > -2) continue;
            const int bi = -2 - nb;
            const T nlx = g.nlx[si], nly = g.nly[si], rx = g.rfx[si], ry = g.rfy[si];
            T gb[9];
            ghost(g, bi, nlx, nly, gc, drho, rho, ux, uy, gb);
            const int kind = g.b_kind[bi];
            const bool wall = (kind == kWall || kind == kMovingWall);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T end = T(ex(a)) * nlx + T(ey(a)) * nly;
                const T own = gc[a] + G[(size_t)(2 * (a - 1)) * n + c] * rx + G[(size_t)(2 * (a - 1) + 1) * n + c] * ry;
                sum[a] += end * ((wall || end < T(0)) ? gb[a] : own);
            }
        }
    }
    const T ia = g.inv_area[c];
    T ga[9];
    ga[0] = T(0);
#pragma unroll
    for (int a = 1; a < 9; ++a) ga[a] = -sum[a] * ia;
    stage_epilogue<T, J>(c, n, gc, ga, b, p);
}

// Tiled sweep: one workgroup per tile of kTileCells consecutive cells plus kHaloThreads extra
// threads for the tile's halo (the interior neighbours outside the tile).
//   VALS = true : phase 0 stages the stage field of the tile and its halo in LDS (directions 1..8);
//                 phase 1 computes the LSQ gradients of the tile cells from LDS and those of the
//                 halo cells from global memory (their own neighbours lie further out);
//   VALS = false: phase 1 reads every neighbour value from global memory.
// Phase 2 takes the convection term with each upwind neighbour's value and gradient from LDS and
// runs the stage epilogue.  LDS planes (W = kTileCells + halo_max columns): 16 gradient planes
// (d/dx, d/dy of directions 1..8) then, with VALS, 8 value planes.  Tile cell t is column t, halo
// cell j column kTileCells + j; lnb gives the column of each slot's neighbour.
constexpr int kTileCells = 256;
constexpr int kHaloThreads = 64;

template <typename T>
struct NbrTileVals {
    const T *L;            // LDS planes [24][W]
    const int16_t *lnb;
    int n, W, loc;
    __device__ __forceinline__ void slot(int s, int c) { loc = lnb[(size_t)s * n + c]; }
    __device__ __forceinline__ T recon(int a, int, T qx, T qy) const {
        return L[(15 + a) * W + loc] + L[(2 * (a - 1)) * W + loc] * qx + L[(2 * (a - 1) + 1) * W + loc] * qy;
    }
    __device__ __forceinline__ T value(int a, int) const { return L[(15 + a) * W + loc]; }
};

// LSQ gradient of a tile cell whose neighbours' values are all in LDS (value plane of direction a
// is 15 + a); boundary edges use the ghost state of the cell's own values gc.
template <typename T>
__device__ __forceinline__ void grad_cell_lds(const Geo<T> &g, int cell, const int16_t *__restrict__ lnb,
                                              const T *L, int W, T rho0, const T gc[9], T gx[9], T gy[9]) {
    const int n = g.n;
#pragma unroll
    for (int a = 0; a < 9; ++a) gx[a] = gy[a] = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + cell;
        const int nb = g.nbr[si];
        if (nb == -1) continue;
        const T cxs = g.cx[si], cys = g.cy[si];
        if (nb >= 0) {
            const int loc = lnb[si];
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T d = L[(15 + a) * W + loc] - gc[a];
                gx[a] += cxs * d;
                gy[a] += cys * d;
            }
        } else {
            T drho, rho, ux, uy, gb[9];
            moments(gc, rho0, drho, rho, ux, uy);
            ghost(g, -2 - nb, g.nlx[si], g.nly[si], gc, drho, rho, ux, uy, gb);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T d = gb[a] - gc[a];
                gx[a] += cxs * d;
                gy[a] += cys * d;
            }
        }
    }
}

template <typename T, int J, bool VALS>
__global__ void __launch_bounds__(kTileCells + kHaloThreads)
    k_stage_tiled(Geo<T> g, const int32_t *__restrict__ hptr, const int32_t *__restrict__ hcell,
                  const int16_t *__restrict__ lnb, int W, StageBufs<T> b, StepPar<T> p) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *L = reinterpret_cast<T *>(smem);
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const int start = tile * kTileCells;
    const int ncell = min(kTileCells, g.n - start);
    const int h0 = hptr[tile], hcnt = hptr[tile + 1] - h0;
    const int t = threadIdx.x;
    const int n = g.n;
    T gc[9], gx[9], gy[9];
    if constexpr (VALS) {
        // phase 0: stage values of the tile (coalesced) and of its halo (gathered)
        if (t < ncell) {
#pragma unroll
            for (int a = 0; a < 9; ++a) gc[a] = b.src[(size_t)a * n + start + t];
#pragma unroll
            for (int a = 1; a < 9; ++a) L[(15 + a) * W + t] = gc[a];
        }
        for (int j = t; j < hcnt; j += kTileCells + kHaloThreads) {
            const int hc = hcell[h0 + j];
#pragma unroll
            for (int a = 1; a < 9; ++a) L[(15 + a) * W + kTileCells + j] = b.src[(size_t)a * n + hc];
        }
        __syncthreads();
    }
    // phase 1: gradients of the tile cells (threads < kTileCells) and of the halo (the rest first)
    if (t < ncell) {
        if constexpr (VALS)
            grad_cell_lds(g, start + t, lnb, L, W, p.rho0, gc, gx, gy);
        else
            grad_cell(g, b.src, start + t, p.rho0, gc, gx, gy);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            L[(2 * (a - 1)) * W + t] = gx[a];
            L[(2 * (a - 1) + 1) * W + t] = gy[a];
        }
    }
    {
        // halo cell j is taken by thread kTileCells + j, then (beyond kHaloThreads) by thread j - kHaloThreads
        const int first = t >= kTileCells ? t - kTileCells : t + kHaloThreads;
        for (int j = first; j < hcnt; j += kTileCells + kHaloThreads) {
            T hc[9], hx[9], hy[9];
            grad_cell(g, b.src, hcell[h0 + j], p.rho0, hc, hx, hy);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                L[(2 * (a - 1)) * W + kTileCells + j] = hx[a];
                L[(2 * (a - 1) + 1) * W + kTileCells + j] = hy[a];
            }
        }
    }
    __syncthreads();
    if (t >= ncell) return;
    const int c = start + t;
    T ga[9];
    if constexpr (VALS)
        advect_cell(g, c, p.rho0, gc, gx, gy, NbrTileVals<T>{L, lnb, n, W, 0}, ga, p.limiter);
    else
        advect_cell(g, c, p.rho0, gc, gx, gy, NbrTile<T>{b.src, L, lnb, n, W, 0}, ga, p.limiter);
    stage_epilogue<T, J>(c, n, gc, ga, b, p);
}

// ---- ring-tiled sweep ----
// One workgroup of kTileCells threads per tile of kTileCells consecutive cells.  The tile's
// extended halo (ring 1: the interior neighbours of its cells outside it; ring 2: the interior
// neighbours of ring-1 cells outside tile and ring 1) is listed per tile, so every global load a
// workgroup needs is issued early, at most one dependent step behind the tile's own loads:
//   phase 0: thread t loads tile cell t (stage values, its edge geometry; stage 1 also f^n and
//            tau) and ext cell t (stage values; for a ring-1 cell also its neighbour columns and
//            the edge data its LSQ coefficients are formed from, as in its own tile); the stage
//            values of directions 1..8 go to LDS;
//   phase 1: LSQ gradients of ring-1 cell t and tile cell t from the LDS values, into LDS; the
//            epilogue operands of stages 2, 3 (and of the explicit scheme) are loaded between the
//            two, so that they are not live during phase 0 and the ring-1 gradient;
//   phase 2: the convection term of tile cell t (Eq. (advection)) with each upwind neighbour's
//            value and gradient from LDS, then the stage epilogue.
// Stage 1 takes f^(1) = stage solve of f^n (a = dt/(4 tau)) on the fly, for tile and ext cells.
// J = 0 is the explicit scheme: src = f^n, forward-Euler epilogue.
// LDS, cell-major so that a neighbour's data is a few 16-byte reads: V [Wv][8] values of
// directions 1..8 (Wv = kTileCells + largest extended halo), Gl [Wg][16] their x / y gradients
// interleaved (Wg = kTileCells + largest ring 1), both with chunks permuted by row (vrow, grow);
// tile cell t is row t, ext entry j row kTileCells + j.
// S = edges per cell of the mesh (3: triangles only; 4 otherwise).
struct RingTiles {
    const int32_t *ptr;    // [n_tiles + 1] offsets into cell
    const int32_t *n1;     // [n_tiles] ring-1 count
    const int32_t *cell;   // [n_ext] internal cell ids: ring 1 then ring 2 of each tile
    const int16_t *lnb;    // [4][n_ext] columns of the neighbours of ring-1 entries
    int32_t n_ext;
};

// Cell-major LDS rows with their 16-byte chunks permuted by row: chunk j of row r is stored at
// chunk position j ^ (bits of r), so that the rows a wave reads (random within the tile) spread
// over all LDS banks instead of the few that the row stride alone would reach.
// vrow: 8 values per row (2 chunks); grow: 16 values per row (4 chunks).
// The permutation pays off for 8-byte values; FP32 rows keep the plain order (the index arithmetic
// costs more issue slots than the bank conflicts it removes there).
template <typename T>
__device__ __forceinline__ int vrow(int r, int k) {
    if constexpr (sizeof(T) == 4) return r * 8 + k;
    return r * 8 + ((((k >> 2) ^ (r >> 3)) & 1) << 2) + (k & 3);
}
template <typename T>
__device__ __forceinline__ int grow(int r, int k) {
    if constexpr (sizeof(T) == 4) return r * 16 + k;
    return r * 16 + ((((k >> 2) ^ (r >> 2)) & 3) << 2) + (k & 3);
}

// LSQ gradient from LDS values of a cell with edge data held in registers (nb, col, cx, cy per
// slot; the normal of a boundary edge is read when needed).  The interior edges are summed in
// straight-line code (an edge without an interior neighbour reads row 0 with weight 0), the
// boundary edges' ghost states after them, in a branch that only boundary cells take.
// BOUNDS: also the least and greatest difference between a stencil value (neighbour or ghost) and
// the cell's own value, each bounded by 0 (dlo <= 0 <= dhi), for the gradient limiter of r35.
template <typename T, int S, bool BOUNDS = false>
__device__ __forceinline__ void grad_ring(const Geo<T> &g, int cell, const int nb[S], const int col[S], const T cxs[S],
                                          const T cys[S], const T *V, T rho0, const T gc[9], T gx[9], T gy[9],
                                          T *dlo = nullptr, T *dhi = nullptr) {
    const int n = g.n;
#pragma unroll
    for (int a = 0; a < 9; ++a) gx[a] = gy[a] = T(0);
    if constexpr (BOUNDS) {
#pragma unroll
        for (int a = 0; a < 9; ++a) dlo[a] = dhi[a] = T(0);
    }
    bool bnd = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool in = nb[s] >= 0;
        bnd = bnd || nb[s] <= -2;
        const int r = in ? col[s] : 0;
        const T wx = in ? cxs[s] : T(0), wy = in ? cys[s] : T(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const T d = V[vrow<T>(r, a - 1)] - gc[a];
            gx[a] += wx * d;
            gy[a] += wy * d;
            if constexpr (BOUNDS) {
                dlo[a] = in && d < dlo[a] ? d : dlo[a];
                dhi[a] = in && d > dhi[a] ? d : dhi[a];
            }
        }
    }
    if (bnd) {
        T drho, rho, ux, uy;
        moments(gc, rho0, drho, rho, ux, uy);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] > -2) continue;
            const size_t si = (size_t)s * n + cell;
            T gb[9];
            ghost(g, -2 - nb[s], g.nlx[si], g.nly[si], gc, drho, rho, ux, uy, gb);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T d = gb[a] - gc[a];
                gx[a] += cxs[s] * d;
                gy[a] += cys[s] * d;
                if constexpr (BOUNDS) {
                    dlo[a] = d < dlo[a] ? d : dlo[a];
                    dhi[a] = d > dhi[a] ? d : dhi[a];
                }
            }
        }
    }
}

// Reading r35 (Barth and Jespersen): scales the gradient of each direction by the largest psi in
// [0, 1] that keeps the reconstructed values at all the cell's edge midpoints (offsets rx, ry from
// the centroid) within the cell's value plus [dlo, dhi], the stencil's bounds from grad_ring:
// psi = min over the edges of dhi / increment (positive increments), dlo / increment (negative).
template <typename T, int S>
__device__ __forceinline__ void bj_scale(const int nb[S], const T rx[S], const T ry[S], const T dlo[9], const T dhi[9],
                                         T gx[9], T gy[9]) {
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        T psi = T(1);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] == -1) continue;
            const T inc = gx[a] * rx[s] + gy[a] * ry[s];
            const T r = inc > T(0) ? dhi[a] / inc : (inc < T(0) ? dlo[a] / inc : T(1));
            psi = r < psi ? r : psi;
        }
        gx[a] *= psi;
        gy[a] *= psi;
    }
}

// Reading r35 on the gradient planes of k_grad (the two-kernel, edge-loop and diagnostic paths):
// each cell's stencil bounds from its neighbours' values and boundary ghost states, then the scaling
// of bj_scale, in place.
template <typename T>
__global__ void __launch_bounds__(256) k_bj(Geo<T> g, const T *__restrict__ f, T *__restrict__ G, T rho0) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T gc[9], lo[9], hi[9], gx[9], gy[9], rx[4], ry[4];
    int nbs[4];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        gc[a] = f[(size_t)a * n + c];
        lo[a] = hi[a] = T(0);
    }
    T drho, rho, ux, uy;
    moments(gc, rho0, drho, rho, ux, uy);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        nbs[s] = nb;
        rx[s] = g.rfx[si];
        ry[s] = g.rfy[si];
        if (nb == -1) continue;
        T v[9];
        if (nb >= 0) {
#pragma unroll
            for (int a = 1; a < 9; ++a) v[a] = f[(size_t)a * n + nb];
        } else {
            ghost(g, -2 - nb, g.nlx[si], g.nly[si], gc, drho, rho, ux, uy, v);
        }
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const T d = v[a] - gc[a];
            lo[a] = d < lo[a] ? d : lo[a];
            hi[a] = d > hi[a] ? d : hi[a];
        }
    }
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        gx[a] = G[(size_t)(2 * (a - 1)) * n + c];
        gy[a] = G[(size_t)(2 * (a - 1) + 1) * n + c];
    }
    bj_scale<T, 4>(nbs, rx, ry, lo, hi, gx, gy);
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        G[(size_t)(2 * (a - 1)) * n + c] = gx[a];
        G[(size_t)(2 * (a - 1) + 1) * n + c] = gy[a];
    }
}

// Slot codes of a cell (tile-local int16 columns: >= 0 an interior neighbour's LDS column, -1 an
// unused slot, -2 - k the cell's k-th boundary edge) decoded into the classification the sweeps
// use: nb >= 0 interior, -1 unused, -2 - b boundary edge b = bfirst[cell] + k.  Only cells with a
// boundary edge read bfirst.
template <int S>
__device__ __forceinline__ void decode_slots(const int32_t *__restrict__ bfirst, int cell, const int col[S], int nb[S]) {
    bool bnd = false;
#pragma unroll
    for (int s = 0; s < S; ++s) bnd = bnd || col[s] <= -2;
    const int bf = bnd ? bfirst[cell] : 0;
#pragma unroll
    for (int s = 0; s < S; ++s) nb[s] = col[s] >= -1 ? col[s] : col[s] - bf;
}

// Edge geometry of a triangle cell from its vertex offsets p_k (vertex k minus the centroid; edge k
// runs from vertex k to vertex k+1, counter-clockwise): outward normal x length, midpoint minus
// centroid, and the inverse area.  FP32 reads p0, p1 and takes p2 = -p0 - p1 (the centroid of a
// triangle is its vertex mean; the difference is far below FP32 resolution); FP64 reads all three.
template <typename T, typename GG>
__device__ __forceinline__ void tri_edges(const GG &g, int c, T nlx[3], T nly[3], T rx[3], T ry[3], T &ia) {
    const size_t n = g.n;
    T px[3], py[3];
    px[0] = g.tp[c];
    py[0] = g.tp[n + c];
    px[1] = g.tp[2 * n + c];
    py[1] = g.tp[3 * n + c];
    if constexpr (sizeof(T) == 4) {
        px[2] = -px[0] - px[1];
        py[2] = -py[0] - py[1];
    } else {
        px[2] = g.tp[4 * n + c];
        py[2] = g.tp[5 * n + c];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = k, b = (k + 1) % 3;
        nlx[k] = py[b] - py[a];
        nly[k] = px[a] - px[b];
        rx[k] = T(0.5) * (px[a] + px[b]);
        ry[k] = T(0.5) * (py[a] + py[b]);
    }
    ia = T(2) * recip((px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]));
}

// LSQ coefficients of all slots of a cell from its centroid offsets d = r_f - q (Section 3 LSQ
// gradient with weights 1 / |d|^2): M = sum w d d^T, (cx, cy) = w M^-1 d; zero on unused slots.
template <typename T, int S>
__device__ __forceinline__ void lsq_cell(const T rx[S], const T ry[S], const T qx[S], const T qy[S], const int nb[S],
                                         T cx[S], T cy[S], T mi[3]) {
    T dx[S], dy[S], w[S], m00 = T(0), m01 = T(0), m11 = T(0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        dx[s] = rx[s] - qx[s];
        dy[s] = ry[s] - qy[s];
        w[s] = nb[s] != -1 ? recip(dx[s] * dx[s] + dy[s] * dy[s]) : T(0);
        m00 += w[s] * dx[s] * dx[s];
        m01 += w[s] * dx[s] * dy[s];
        m11 += w[s] * dy[s] * dy[s];
    }
    const T idet = recip(m00 * m11 - m01 * m01);
    const T i00 = m11 * idet, i01 = -m01 * idet, i11 = m00 * idet;
    mi[0] = i00;
    mi[1] = i01;
    mi[2] = i11;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        cx[s] = w[s] * (i00 * dx[s] + i01 * dy[s]);
        cy[s] = w[s] * (i01 * dx[s] + i11 * dy[s]);
    }
}

// LSQ coefficients of one slot, (cx, cy) = w M^-1 d with d = r_f - q the centroid offset to the
// neighbour (to the edge midpoint on a boundary edge, where q = 0), w = 1 / |d|^2 and M^-1 the
// cell's inverse least-squares matrix (m00, m01, m11).  Zero on an unused slot.
template <typename T>
__device__ __forceinline__ void lsq_coef(T m00, T m01, T m11, T rx, T ry, T qx, T qy, bool used, T &cx, T &cy) {
    const T dx = rx - qx, dy = ry - qy;
    const T w = used ? recip(dx * dx + dy * dy) : T(0);
    cx = w * (m00 * dx + m01 * dy);
    cy = w * (m01 * dx + m11 * dy);
}

// Edge data of cell c in registers: slot codes (from lnb, row stride ls), classification, normal
// x length, midpoint and neighbour-centroid offsets, LSQ coefficients, inverse LSQ matrix, inverse
// area.  Triangle meshes (S = 3) form normals, midpoints, area and LSQ data from the vertex
// offsets and q; other meshes read them, with the LSQ coefficients from the stored inverse matrix.
// FP32 takes the LSQ coefficients themselves from the host's FP64 values, rounded once: formed in
// FP32 on skewed, stretched cells they lose up to 2e-5 relative (cancellation in w M^-1 d), which
// the FP32-deviation error gates resolve.  Tile cells and halo cells of other tiles go through this
// one function, so a cell's coefficients never depend on the tile that evaluates them.
template <typename T, int S, typename GG>
__device__ __forceinline__ void cell_edges(const GG &g, const int16_t *__restrict__ lnb, size_t ls, size_t li,
                                           int c, int col[S], int nb[S], T nlx[S], T nly[S], T rx[S], T ry[S],
                                           T qx[S], T qy[S], T cxs[S], T cys[S], T mi[3], T &ia) {
    const int n = g.n;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const size_t si = (size_t)s * n + c;
        col[s] = lnb[(size_t)s * ls + li];
        qx[s] = g.qx[si];
        qy[s] = g.qy[si];
        if constexpr (S != 3) {
            nlx[s] = g.nlx[si];
            nly[s] = g.nly[si];
            rx[s] = g.rfx[si];
            ry[s] = g.rfy[si];
        }
    }
    decode_slots<S>(g.bfirst, c, col, nb);
    if constexpr (S == 3) {
        tri_edges<T>(g, c, nlx, nly, rx, ry, ia);
        lsq_cell<T, S>(rx, ry, qx, qy, nb, cxs, cys, mi);
    } else {
        mi[0] = g.mi[c];
        mi[1] = g.mi[(size_t)n + c];
        mi[2] = g.mi[(size_t)2 * n + c];
#pragma unroll
        for (int s = 0; s < S; ++s) lsq_coef(mi[0], mi[1], mi[2], rx[s], ry[s], qx[s], qy[s], nb[s] != -1, cxs[s], cys[s]);
        ia = g.inv_area[c];
    }
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            cxs[s] = g.cx[(size_t)s * n + c];
            cys[s] = g.cy[(size_t)s * n + c];
        }
    }
}

// FP32 edge data of an FP32_DEV_GEO64 state: formed in FP64 from the FP64 geometry copies exactly as
// an FP64 state forms it (LSQ coefficients from the FP64 centroid offsets), then each value rounded
// once to FP32 for the FP32 flux arithmetic.
template <int S>
__device__ __forceinline__ void cell_edges_g64(const Geo<float> &g, const int16_t *__restrict__ lnb, size_t ls,
                                               size_t li, int c, int col[S], int nb[S], float nlx[S], float nly[S],
                                               float rx[S], float ry[S], float qx[S], float qy[S], float cxs[S],
                                               float cys[S], float mi[3], float &ia) {
    double dnx[S], dny[S], drx[S], dry[S], dqx[S], dqy[S], dcx[S], dcy[S], dmi[3], dia;
    cell_edges<double, S>(g.g64, lnb, ls, li, c, col, nb, dnx, dny, drx, dry, dqx, dqy, dcx, dcy, dmi, dia);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        nlx[s] = (float)dnx[s];
        nly[s] = (float)dny[s];
        rx[s] = (float)drx[s];
        ry[s] = (float)dry[s];
        qx[s] = (float)dqx[s];
        qy[s] = (float)dqy[s];
        cxs[s] = (float)dcx[s];
        cys[s] = (float)dcy[s];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) mi[k] = (float)dmi[k];
    ia = (float)dia;
}

// The edge data of a cell from the state's geometry (G64: from the FP64 copies, FP32 states only).
template <typename T, int S, bool G64>
__device__ __forceinline__ void edges_of(const Geo<T> &g, const int16_t *__restrict__ lnb, size_t ls, size_t li,
                                         int c, int col[S], int nb[S], T nlx[S], T nly[S], T rx[S], T ry[S], T qx[S],
                                         T qy[S], T cxs[S], T cys[S], T mi[3], T &ia) {
    if constexpr (G64)
        cell_edges_g64<S>(g, lnb, ls, li, c, col, nb, nlx, nly, rx, ry, qx, qy, cxs, cys, mi, ia);
    else
        cell_edges<T, S>(g, lnb, ls, li, c, col, nb, nlx, nly, rx, ry, qx, qy, cxs, cys, mi, ia);
}

template <typename T, int J, int S, int LIM, bool G64 = false>
__global__ void __launch_bounds__(kTileCells, sizeof(T) == 4 ? 4 : 2)
    k_stage_ring(Geo<T> g, RingTiles rt, const int16_t *__restrict__ lnb, int Wv, int Wg, StageBufs<T> b,
                 StepPar<T> p) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *V = reinterpret_cast<T *>(smem);
    T *Gl = V + 8 * Wv;
    const int tile = ring_tile<J == 2>();
    const int start = tile * kTileCells;
    const int ncell = min(kTileCells, g.n - start);
    const int x0 = rt.ptr[tile], nx = rt.ptr[tile + 1] - x0, n1 = rt.n1[tile];
    const int t = threadIdx.x;
    const int n = g.n;
    const bool own = t < ncell, ext = t < nx, ring1 = t < n1;
    const int c = start + t;

    // ---- phase 0 ----
    T gc[9];
    EpiOps<T> ops;
    int nb[S], col[S];
    T cxs[S], cys[S], nlx[S], nly[S], rx[S], ry[S], qx[S], qy[S], ia = T(0);
    if (own) {
        if constexpr (J == 1) {
            load_ops<T, 1>(b, c, n, ops, p.recover);
            T fe[9];
            stage_collide(ops.fn, p.dt * T(0.25) * recip(ops.tc), p.rho0, gc, fe);
        } else {
#pragma unroll
            for (int a = 0; a < 9; ++a) gc[a] = b.src[(size_t)a * n + c];
        }
        T mi[3];
        edges_of<T, S, G64>(g, lnb, n, c, c, col, nb, nlx, nly, rx, ry, qx, qy, cxs, cys, mi, ia);
#pragma unroll
        for (int a = 1; a < 9; ++a) V[vrow<T>(t, a - 1)] = gc[a];
    }
    T hv[9];
    int hc = 0, hnb[S], hcol[S];
    T hcx[S], hcy[S], hrx[S], hry[S];   // hrx, hry: used by the gradient limiter of r35 only
    if (ext) {
        hc = rt.cell[x0 + t];
        if constexpr (J == 1) {
            T hf[9], fe[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) hf[a] = b.F_in[(size_t)a * n + hc];
            stage_collide(hf, p.dt * T(0.25) * recip(b.tau[hc]), p.rho0, hv, fe);
        } else {
            // the rest direction only where a ring-1 cell's ghost states need the moments
            hv[0] = ring1 ? b.src[hc] : T(0);
#pragma unroll
            for (int a = 1; a < 9; ++a) hv[a] = b.src[(size_t)a * n + hc];
        }
#pragma unroll
        for (int a = 1; a < 9; ++a) V[vrow<T>(kTileCells + t, a - 1)] = hv[a];
        if (ring1) {
            // the ring-1 cell's LSQ coefficients formed exactly as in its own tile (same data, same
            // code), so that its gradient, and the face values built from it, do not depend on
            // which tile evaluates them
            T hnlx[S], hnly[S], hqx[S], hqy[S], hmi[3], hia;
            edges_of<T, S, G64>(g, rt.lnb, rt.n_ext, x0 + t, hc, hcol, hnb, hnlx, hnly, hrx, hry, hqx, hqy, hcx, hcy,
                             hmi, hia);
        }
    }
    // ring-2 cells beyond one per thread (tiles of stretched cells): their values only
    for (int e = t + kTileCells; e < nx; e += kTileCells) {
        const int ec = rt.cell[x0 + e];
        T ev[9];
        if constexpr (J == 1) {
            T ef[9], fe[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) ef[a] = b.F_in[(size_t)a * n + ec];
            stage_collide(ef, p.dt * T(0.25) * recip(b.tau[ec]), p.rho0, ev, fe);
        } else {
#pragma unroll
            for (int a = 1; a < 9; ++a) ev[a] = b.src[(size_t)a * n + ec];
        }
#pragma unroll
        for (int a = 1; a < 9; ++a) V[vrow<T>(kTileCells + e, a - 1)] = ev[a];
    }
    __syncthreads();

    // ---- phase 1 ----
    if (ring1) {
        T hx[9], hy[9];
        if constexpr (LIM == 2) {
            T lo[9], hi[9];
            grad_ring<T, S, true>(g, hc, hnb, hcol, hcx, hcy, V, p.rho0, hv, hx, hy, lo, hi);
            bj_scale<T, S>(hnb, hrx, hry, lo, hi, hx, hy);
        } else {
            grad_ring<T, S>(g, hc, hnb, hcol, hcx, hcy, V, p.rho0, hv, hx, hy);
        }
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            Gl[grow<T>(kTileCells + t, 2 * (a - 1))] = hx[a];
            Gl[grow<T>(kTileCells + t, 2 * (a - 1) + 1)] = hy[a];
        }
    }
    T gx[9], gy[9];
    if (own) {
        // the epilogue operands of stages other than 1 are loaded here, after the ring-1 work:
        // they are in flight during the gradient and the barrier without being live in phase 0
        if constexpr (J != 1) load_ops<T, J>(b, c, n, ops, p.recover);
        if constexpr (LIM == 2) {
            T lo[9], hi[9];
            grad_ring<T, S, true>(g, c, nb, col, cxs, cys, V, p.rho0, gc, gx, gy, lo, hi);
            bj_scale<T, S>(nb, rx, ry, lo, hi, gx, gy);
        } else {
            grad_ring<T, S>(g, c, nb, col, cxs, cys, V, p.rho0, gc, gx, gy);
        }
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            Gl[grow<T>(t, 2 * (a - 1))] = gx[a];
            Gl[grow<T>(t, 2 * (a - 1) + 1)] = gy[a];
        }
    }
    __syncthreads();
    if (!own) return;

    // ---- phase 2: convection term; interior edges in straight-line code (an edge without an
    // interior neighbour reads row 0 with a zero normal), boundary edges after them ----
    T acc[9];
#pragma unroll
    for (int a = 1; a < 9; ++a) acc[a] = T(0);
    bool bnd = false;
    uint64_t cm = 0;   // clip states (LIM == 3: the r32 clip of a recorded step)
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool in = nb[s] >= 0;
        bnd = bnd || nb[s] <= -2;
        const int loc = in ? col[s] : 0;
        const T mx = in ? nlx[s] : T(0), my = in ? nly[s] : T(0);
        // both reconstructions, then a select: the upwind side differs from lane to lane
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const T end = T(ex(a)) * mx + T(ey(a)) * my;
            const T vn = V[vrow<T>(loc, a - 1)];
            const T up_n = vn + Gl[grow<T>(loc, 2 * (a - 1))] * qx[s] + Gl[grow<T>(loc, 2 * (a - 1) + 1)] * qy[s];
            const T up_c = gc[a] + gx[a] * rx[s] + gy[a] * ry[s];
            T val = end >= T(0) ? up_c : up_n;
            if constexpr (LIM == 1 || LIM == 3) {
                const T lim = clip_between(val, gc[a], vn);
                if constexpr (LIM == 3) {
                    const bool clipped = in && lim != val;
                    cm |= (uint64_t)clipped << (2 * (8 * s + a - 1));
                    cm |= (uint64_t)(clipped && lim == gc[a]) << (2 * (8 * s + a - 1) + 1);
                }
                val = lim;
            }
            acc[a] += end * val;
        }
        // one edge's LDS reads in flight at a time (bounds the registers they occupy)
        __builtin_amdgcn_sched_barrier(0);
    }
    if (bnd) {
        // rare: the edge data is read again and the cell's gradient taken from LDS, so that
        // neither stays live in registers through the interior loop
        T drho, rho, ux, uy;
        moments(gc, p.rho0, drho, rho, ux, uy);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] > -2) continue;
            const int bi = -2 - nb[s];
            const size_t si = (size_t)s * n + c;
            const T bnx = g.nlx[si], bny = g.nly[si], brx = g.rfx[si], bry = g.rfy[si];
            T gb[9];
            ghost(g, bi, bnx, bny, gc, drho, rho, ux, uy, gb);
            const int kind = g.b_kind[bi];
            const bool wall = (kind == kWall || kind == kMovingWall);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T end = T(ex(a)) * bnx + T(ey(a)) * bny;
                const T own_f = gc[a] + Gl[grow<T>(t, 2 * (a - 1))] * brx + Gl[grow<T>(t, 2 * (a - 1) + 1)] * bry;
                const T val = (wall || end < T(0)) ? gb[a] : own_f;
                acc[a] += end * val;
            }
        }
    }
    if constexpr (LIM == 3) b.clip[c] = cm;
    T ga[9];
    ga[0] = T(0);
#pragma unroll
    for (int a = 1; a < 9; ++a) ga[a] = -acc[a] * ia;
    stage_epilogue_ops<T, J>(c, n, gc, ga, ops, b, p);
}

// Convection term alone (diagnostic entry point).
template <typename T>
__global__ void __launch_bounds__(256) k_advect(Geo<T> g, const T *__restrict__ X, const T *__restrict__ G,
                                                T *__restrict__ out, T rho0, int limiter) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T gc[9], ga[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) gc[a] = X[(size_t)a * n + c];
    advect_cell_global(g, X, G, c, rho0, gc, ga, limiter);
#pragma unroll
    for (int a = 0; a < 9; ++a) out[(size_t)a * n + c] = ga[a];
}

// ----------------------------------------------------------------------------------------------
// k-omega SST (Section 2 model; finite-volume form Eq. (SSTequint)).
// aux planes: 0,1 grad k; 2,3 grad omega; 4 Gamma_k; 5 Gamma_omega; 6 dt P / rho;
//             7 dt (P_omega + cross diffusion) / rho; 8 blended beta; 9 strain rate S;
//             10, 11 net inflows of k, omega (written by the flux / update stage);
//             12..14 the input macro variables rho - rho0, u, v (kept for the adjoint).
// Boundary data per edge (set at init): b_ux, b_uy velocity (0 on resting walls), b_k (0 on walls),
// b_w (60 nu / (beta1 d_perp^2) on walls), and b_zg = 1 where k, omega, u are zero-gradient
// (outlets, far-field outflow edges).
// ----------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T tmax(T a, T b) { return a >= b ? a : b; }
template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return a <= b ? a : b; }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> tmax(const Dual<T, K> &a, const Dual<T, K> &b) { return dmax(a, b); }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> tmin(const Dual<T, K> &a, const Dual<T, K> &b) { return dmin(a, b); }
template <typename T>
__device__ __forceinline__ T ssqrt(T a) { return sqrt(a); }
// FP32: the hardware square root (v_sqrt_f32, within 1 ulp)
template <>
__device__ __forceinline__ float ssqrt<float>(float a) { return __builtin_amdgcn_sqrtf(a); }
template <typename T>
__device__ __forceinline__ T stanh(T a) { return tanh(a); }
// FP32: tanh x = 1 - 2 / (exp(2x) + 1) with the hardware exponential and reciprocal (the SST
// evaluates it at squares, x >= 0; large x gives exp = inf and the result 1; near 0 the absolute
// error is a few FP32 ulps of 1, far below what the blending functions resolve)
template <>
__device__ __forceinline__ float stanh<float>(float a) {
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * a) + 1.0f);
}
// exp: FP32 with the hardware exponential
template <typename T>
__device__ __forceinline__ T sexp(T a) { return exp(a); }
template <>
__device__ __forceinline__ float sexp<float>(float a) { return __expf(a); }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> ssqrt(const Dual<T, K> &a) { return dsqrt(a); }
template <typename T, int K>
__device__ __forceinline__ Dual<T, K> stanh(const Dual<T, K> &a) { return dtanh(a); }
template <typename S>
__device__ __forceinline__ S sval(const S &a) { return a; }
template <typename T, int K>
__device__ __forceinline__ T sval(const Dual<T, K> &a) { return a.v; }

// The four SST constants the adjoint differentiates (a1, beta*, sigma_k1, sigma_omega1), in the
// scalar type S; the others come from StepPar.
template <typename S>
struct SstParams {
    S a1, bstar, sk1, sw1;
};

// Cell-local closure of the SST model (Section 2): from rho, k, omega, the wall distance d and the
// gradients of u, v, k, omega, the diffusion coefficients Gamma_k, Gamma_omega, the explicit
// sources dt P / rho and dt (P_omega + cross diffusion) / rho, the blended beta and the strain S.
template <typename S>
struct SstLocal {
    S Gk, Gw, sk, sw, beta, Sr;
};

template <typename S, typename T>
__device__ __forceinline__ SstLocal<S> sst_local(S rho, S k, S w, S dux, S duy, S dvx, S dvy, S dkx, S dky, S dwx,
                                                 S dwy, T d, const StepPar<T> &p, const SstParams<S> &q) {
    // C_omega_i = beta_i / beta* - sigma_omega_i kappa^2 / sqrt(beta*)
    const S ib = recip(q.bstar), isb = recip(ssqrt(q.bstar));
    const S cw1 = cst<S>(p.b1) * ib - q.sw1 * cst<S>(p.kappa * p.kappa) * isb;
    const S cw2 = cst<S>(p.b2) * ib - cst<S>(p.sw2 * p.kappa * p.kappa) * isb;
    const S s11 = dux, s22 = dvy, s12 = cst<S>(0.5) * (duy + dvx);
    const S S2 = cst<S>(2) * (s11 * s11 + s22 * s22 + cst<S>(2) * s12 * s12);
    const S Sr = ssqrt(S2);
    const S div = dux + dvy;
    const S gkgw = dkx * dwx + dky * dwy;
    const S iw = recip(w);
    const S CD = tmax(cst<S>(2) * rho * cst<S>(p.sw2) * iw * gkgw, cst<S>(1e-20));
    const S sk = ssqrt(k);
    const S idd = cst<S>(recip(d)), idd2 = idd * idd;
    const S visc = cst<S>(500) * cst<S>(p.nu) * iw * idd2;
    const S t1 = sk * iw * idd * cst<S>(1.0 / 0.09);   // sqrt(k) / (0.09 omega d)
    const S arg1 = tmin(tmax(t1, visc), cst<S>(4) * rho * cst<S>(p.sw2) * k * recip(CD) * idd2);
    const S a2 = arg1 * arg1;
    const S F1 = stanh(a2 * a2);
    const S arg2 = tmax(cst<S>(2) * t1, visc);
    const S F2 = stanh(arg2 * arg2);
    const S den = tmax(q.a1 * w, Sr * F2);
    const S mu = rho * cst<S>(p.nu);
    const S mut = q.a1 * rho * k * recip(den);
    const S one = cst<S>(1);
    const S sig_k = F1 * q.sk1 + (one - F1) * cst<S>(p.sk2);
    const S sig_w = F1 * q.sw1 + (one - F1) * cst<S>(p.sw2);
    const S beta = F1 * cst<S>(p.b1) + (one - F1) * cst<S>(p.b2);
    const S gam = F1 * cw1 + (one - F1) * cw2;
    const S tt = cst<S>(2.0 / 3.0);
    const S P = mut * (S2 - tt * div * div) - tt * rho * k * div;
    // gamma rho P / mu_t without the 0/0 at k = 0: rho k / mu_t = den / a1
    const S Pw = gam * rho * (S2 - tt * div * div) - tt * gam * rho * (den * recip(q.a1)) * div;
    const S cross = cst<S>(2) * (one - F1) * rho * cst<S>(p.sw2) * gkgw * iw;
    const S dtr = cst<S>(p.dt) * recip(rho);
    SstLocal<S> o;
    o.Gk = mu + sig_k * mut;
    o.Gw = mu + sig_w * mut;
    o.sk = dtr * P;
    o.sw = dtr * (Pw + cross);
    o.beta = beta;
    o.Sr = Sr;
    return o;
}

// Upwind k / omega face value, kept in [0, 2 phi_up] so the explicit outflow cannot drive k or
// omega negative (inactive where |grad phi . r| <= phi_up).
template <typename S>
__device__ __forceinline__ S bound_face(S v, S up) { return tmin(tmax(v, cst<S>(0)), cst<S>(2) * up); }

// Convective and diffusive flux of k and omega through an interior edge, seen from cell c (the
// contribution to c's net inflow): -mdot phi_f + Gamma_f (phi_N - phi_c) (d^ . n l) / |d|, with
// mdot = ((rho u)_c + (rho u)_N) / 2 . n l and phi_f the bounded upwind extrapolation.
// Cell data x = (rho, u, v, k, omega, dk/dx, dk/dy, domega/dx, domega/dy, Gamma_k, Gamma_omega).
template <typename S, typename T>
__device__ __forceinline__ void sst_face(const S xc[11], const S xn[11], T nlx, T nly, T rx, T ry, T qx, T qy, S &Tk,
                                         S &Tw) {
    const S mdot = cst<S>(0.5) * ((xc[0] * xc[1] + xn[0] * xn[1]) * cst<S>(nlx) + (xc[0] * xc[2] + xn[0] * xn[2]) * cst<S>(nly));
    // both upwind candidates, then a select (the upwind side differs from lane to lane)
    const S kc = bound_face(xc[3] + xc[5] * cst<S>(rx) + xc[6] * cst<S>(ry), xc[3]);
    const S wc = bound_face(xc[4] + xc[7] * cst<S>(rx) + xc[8] * cst<S>(ry), xc[4]);
    const S kn = bound_face(xn[3] + xn[5] * cst<S>(qx) + xn[6] * cst<S>(qy), xn[3]);
    const S wn = bound_face(xn[4] + xn[7] * cst<S>(qx) + xn[8] * cst<S>(qy), xn[4]);
    const bool up_c = sval(mdot) >= 0;
    const S kf = up_c ? kc : kn, wf = up_c ? wc : wn;
    // central two-point face gradient along the centroid line: (phi_N - phi_c) / |d| d^
    const T ddx = rx - qx, ddy = ry - qy;
    const T hn = (ddx * nlx + ddy * nly) * recip(ddx * ddx + ddy * ddy);
    Tk = -(mdot * kf) + cst<S>(0.5) * (xc[9] + xn[9]) * (xn[3] - xc[3]) * cst<S>(hn);
    Tw = -(mdot * wf) + cst<S>(0.5) * (xc[10] + xn[10]) * (xn[4] - xc[4]) * cst<S>(hn);
}

// The same through a boundary edge: ghost values are the cell's own where zero-gradient (zg),
// else the boundary data (ub velocity, kb, wb); Dirichlet diffusion (phi_b - phi_c) l / d_perp.
template <typename S, typename T>
__device__ __forceinline__ void sst_bface(const S xc[11], bool zg, S ubx, S uby, T kb, T wb, T nlx, T nly, T rx, T ry,
                                          T l_over_dp, S &Tk, S &Tw) {
    const S bux = zg ? xc[1] : ubx, buy = zg ? xc[2] : uby;
    const S bk = zg ? xc[3] : cst<S>(kb), bw = zg ? xc[4] : cst<S>(wb);
    const S mdot = xc[0] * (bux * cst<S>(nlx) + buy * cst<S>(nly));
    S kf, wf;
    if (sval(mdot) >= 0) {
        kf = bound_face(xc[3] + xc[5] * cst<S>(rx) + xc[6] * cst<S>(ry), xc[3]);
        wf = bound_face(xc[4] + xc[7] * cst<S>(rx) + xc[8] * cst<S>(ry), xc[4]);
    } else {
        kf = bk;
        wf = bw;
    }
    Tk = -(mdot * kf);
    Tw = -(mdot * wf);
    if (!zg) {
        Tk = Tk + xc[9] * (bk - xc[3]) * cst<S>(l_over_dp);
        Tw = Tw + xc[10] * (bw - xc[4]) * cst<S>(l_over_dp);
    }
}

// Eddy viscosity a1 k / max(a1 omega, S F2) from the updated k, omega (F2 evaluated again) and the
// level-n strain rate S.
template <typename S, typename T>
__device__ __forceinline__ S sst_nut(S k1, S w1, S Sr, T d, const StepPar<T> &p, const SstParams<S> &q) {
    const S iw1 = recip(w1), idd = cst<S>(recip(d));
    const S arg2 = tmax(cst<S>(2.0 / 0.09) * ssqrt(k1) * iw1 * idd, cst<S>(500) * cst<S>(p.nu) * iw1 * idd * idd);
    const S F2 = stanh(arg2 * arg2);
    return q.a1 * k1 * recip(tmax(q.a1 * w1, Sr * F2));
}

// Point-implicit update (negative parts of the explicit sources join the denominator), floor,
// and the eddy viscosity from the updated k, omega with the level-n strain rate.
template <typename S, typename T>
__device__ __forceinline__ void sst_update(S rho, S k, S w, S net_k, S net_w, S sk, S sw, S beta, S Sr, T d,
                                           T inv_area, const StepPar<T> &p, const SstParams<S> &q, S &k1, S &w1,
                                           S &nut) {
    const S fac = cst<S>(p.dt * inv_area) * recip(rho);
    const S zero = cst<S>(0), one = cst<S>(1), dt = cst<S>(p.dt);
    k1 = (k + fac * net_k + tmax(sk, zero)) * recip(one + dt * q.bstar * w + tmax(-sk, zero) * recip(k));
    w1 = (w + fac * net_w + tmax(sw, zero)) * recip(one + dt * beta * w + tmax(-sw, zero) * recip(w));
    k1 = tmax(k1, cst<S>(1e-20));
    w1 = tmax(w1, cst<S>(1e-20));
    nut = sst_nut<S, T>(k1, w1, Sr, d, p, q);
}

template <typename T>
__device__ __forceinline__ SstParams<T> sst_params(const StepPar<T> &p) {
    return SstParams<T>{p.a1, p.bstar, p.sk1, p.sw1};
}

// ---- implicit variant (params.sst_sweeps = m > 0) ----
// Per cell and variable phi in {k, omega} the increment delta = phi^{n+1} - phi^n solves
//   (sigma - dt / (rho A) L) delta = R,
// L the net inflow with first-order upwind convection and the two-point diffusion (level-n mass
// fluxes, diffusion coefficients and upwind sides), sigma the point-implicit denominator of
// sst_update, R the explicit increment before the sinks act (the second-order flux stays at level n).
// Each row is stored divided by its diagonal, for the Jacobi sweeps delta <- R' + sum_s c_s delta_N
// from delta = 0 (the first sweep gives R').  System planes J [kSysPlanes][n]: 0-3 c_s of k per
// edge slot (0 without an interior neighbour), 4-7 c_s of omega, 8, 9 R' of k, omega, 10, 11 and
// 12, 13 the two increment buffers (k, omega), 14 the strain rate S for nu_t.
constexpr int kSysPlanes = 15;

template <typename S>
struct SstRow {
    S dk, dw;   // flux parts of the two diagonals (outflow and diffusion conductances)
};

// Interior edge: its parts of the diagonals, and the (unscaled) couplings of the neighbour's
// increments: mdot^- + D for the upwind inflow and the diffusion.
template <typename S, typename T>
__device__ __forceinline__ void sst_row_edge(const S xc[11], const S xn[11], T nlx, T nly, T rx, T ry, T qx, T qy,
                                             SstRow<S> &r, S &ck, S &cw) {
    const S mdot = cst<S>(0.5) * ((xc[0] * xc[1] + xn[0] * xn[1]) * cst<S>(nlx) + (xc[0] * xc[2] + xn[0] * xn[2]) * cst<S>(nly));
    const T ddx = rx - qx, ddy = ry - qy;
    const T hn = (ddx * nlx + ddy * nly) * recip(ddx * ddx + ddy * ddy);
    const S Dk = cst<S>(0.5) * (xc[9] + xn[9]) * cst<S>(hn);
    const S Dw = cst<S>(0.5) * (xc[10] + xn[10]) * cst<S>(hn);
    const S out = tmax(mdot, cst<S>(0)), in = tmax(-mdot, cst<S>(0));
    r.dk = r.dk + out + Dk;
    r.dw = r.dw + out + Dw;
    ck = in + Dk;
    cw = in + Dw;
}

// Boundary edge: the cell's own value leaves through an outflow edge or stands for the ghost of a
// zero-gradient edge; Dirichlet diffusion Gamma_c l / d_perp.  Fixed ghost values enter R only.
template <typename S, typename T>
__device__ __forceinline__ void sst_row_bedge(const S xc[11], bool zg, S ubx, S uby, T nlx, T nly, T l_over_dp,
                                              SstRow<S> &r) {
    const S bux = zg ? xc[1] : ubx, buy = zg ? xc[2] : uby;
    const S mdot = xc[0] * (bux * cst<S>(nlx) + buy * cst<S>(nly));
    const S own = (zg || sval(mdot) >= 0) ? mdot : cst<S>(0);
    r.dk = r.dk + own;
    r.dw = r.dw + own;
    if (!zg) {
        r.dk = r.dk + xc[9] * cst<S>(l_over_dp);
        r.dw = r.dw + xc[10] * cst<S>(l_over_dp);
    }
}

// sigma, R and the diagonals; returns R' and the factors fac / diag that scale the couplings.
template <typename S, typename T>
__device__ __forceinline__ void sst_row_finish(S rho, S k, S w, S net_k, S net_w, S sk, S sw, S beta, T inv_area,
                                               const StepPar<T> &p, const SstParams<S> &q, const SstRow<S> &r,
                                               S &Rk, S &Rw, S &gk, S &gw) {
    const S fac = cst<S>(p.dt * inv_area) * recip(rho);
    const S zero = cst<S>(0), one = cst<S>(1), dt = cst<S>(p.dt);
    const S dstk = dt * q.bstar * w, dstw = dt * beta * w;
    const S sig_k = one + dstk + tmax(-sk, zero) * recip(k);
    const S sig_w = one + dstw + tmax(-sw, zero) * recip(w);
    const S ik = recip(sig_k + fac * r.dk), iw = recip(sig_w + fac * r.dw);
    Rk = (fac * net_k + sk - dstk * k) * ik;
    Rw = (fac * net_w + sw - dstw * w) * iw;
    gk = fac * ik;
    gw = fac * iw;
}

// One Jacobi sweep of both increments, cell per thread: delta <- R' + sum_s c_s delta_N (ITER), or
// delta taken as it is (the single-sweep case).  FIN: k^{n+1} = max(k^n + delta, floor), omega
// likewise, then nu_t and tau; else the new increments go to dout.  FWD: the blocks' cell ranges in
// ascending order, else descending within each XCD's range (consecutive sweeps alternate, as the ring
// sweeps do).
template <typename T, int S, bool ITER, bool FIN, bool FWD = true>
__global__ void __launch_bounds__(256) k_sst_jacobi(Geo<T> g, const T *__restrict__ J, const T *__restrict__ din,
                                                    T *__restrict__ dout, const T *__restrict__ K0,
                                                    const T *__restrict__ W0, T *__restrict__ K1,
                                                    T *__restrict__ W1, T *__restrict__ tau, T *__restrict__ nut,
                                                    StepPar<T> p) {
    const int c = ring_tile<FWD>() * (int)blockDim.x + (int)threadIdx.x;
    if (c >= g.n) return;
    const size_t n = (size_t)g.n;
    T dk, dw;
    if constexpr (ITER) {
        dk = J[8 * n + c];
        dw = J[9 * n + c];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int nb = g.nbr[s * n + c];
            if (nb >= 0) {
                dk += J[s * n + c] * din[nb];
                dw += J[(4 + s) * n + c] * din[n + nb];
            }
        }
    } else {
        dk = din[c];
        dw = din[n + c];
    }
    if constexpr (FIN) {
        const T k1 = tmax(K0[c] + dk, T(1e-20)), w1 = tmax(W0[c] + dw, T(1e-20));
        const T nt = sst_nut<T, T>(k1, w1, J[14 * n + c], T(g.wdist[c]), p, sst_params(p));
        K1[c] = k1;
        W1[c] = w1;
        nut[c] = nt;
        tau[c] = T(3) * (p.nu + nt);
    } else {
        dout[c] = dk;
        dout[n + c] = dw;
    }
}

// ----------------------------------------------------------------------------------------------
// k-omega SST kernels (Section 2 model; finite-volume form Eq. (SSTequint)).
// aux planes: 0,1 grad k; 2,3 grad omega; 4 Gamma_k; 5 Gamma_omega; 6 dt P / rho;
//             7 dt (P_omega + cross diffusion) / rho; 8 blended beta; 9 strain rate S;
//             10, 11 net inflows of k, omega (written by the flux / update stage);
//             12..14 the input macro variables rho - rho0, u, v (kept for the adjoint).
// Boundary data per edge (set at init): b_ux, b_uy velocity (0 on resting walls), b_k (0 on walls),
// b_w (60 nu / (beta1 d_perp^2) on walls), and b_zg = 1 where k, omega, u are zero-gradient
// (outlets, far-field outflow edges).
// ----------------------------------------------------------------------------------------------
// LSQ gradients of u, v, k, omega of cell c (ghost values at boundary edges as above).
template <typename T>
__device__ __forceinline__ void sst_gradients(const Geo<T> &g, const int32_t *__restrict__ bzg, const T *__restrict__ M,
                                              const T *__restrict__ K, const T *__restrict__ W, int c, T gu[2], T gv[2],
                                              T gk[2], T gw[2]) {
    const int n = g.n;
    const T ux = M[(size_t)n + c], uy = M[(size_t)2 * n + c], kc = K[c], wc = W[c];
    gu[0] = gu[1] = gv[0] = gv[1] = gk[0] = gk[1] = gw[0] = gw[1] = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        if (nb == -1) continue;
        const T cxs = g.cx[si], cys = g.cy[si];
        T du, dv, dk, dw;
        if (nb >= 0) {
            du = M[(size_t)n + nb] - ux;
            dv = M[(size_t)2 * n + nb] - uy;
            dk = K[nb] - kc;
            dw = W[nb] - wc;
        } else {
            const int b = -2 - nb;
            if (bzg[b]) {
                du = dv = dk = dw = T(0);
            } else {
                du = T(g.b_ux[b]) - ux;
                dv = T(g.b_uy[b]) - uy;
                dk = T(g.b_k[b]) - kc;
                dw = T(g.b_w[b]) - wc;
            }
        }
        gu[0] += cxs * du; gu[1] += cys * du;
        gv[0] += cxs * dv; gv[1] += cys * dv;
        gk[0] += cxs * dk; gk[1] += cys * dk;
        gw[0] += cxs * dw; gw[1] += cys * dw;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_sst_a(Geo<T> g, const int32_t *__restrict__ bzg, const T *__restrict__ M,
                                               const T *__restrict__ K, const T *__restrict__ W,
                                               T *__restrict__ aux, StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T gu[2], gv[2], gk[2], gw[2];
    sst_gradients(g, bzg, M, K, W, c, gu, gv, gk, gw);
    const T rho = p.rho0 + M[c];
    const SstLocal<T> o = sst_local<T, T>(rho, K[c], W[c], gu[0], gu[1], gv[0], gv[1], gk[0], gk[1], gw[0], gw[1],
                                          T(g.wdist[c]), p, sst_params(p));
    aux[c] = gk[0];
    aux[(size_t)1 * n + c] = gk[1];
    aux[(size_t)2 * n + c] = gw[0];
    aux[(size_t)3 * n + c] = gw[1];
    aux[(size_t)4 * n + c] = o.Gk;
    aux[(size_t)5 * n + c] = o.Gw;
    aux[(size_t)6 * n + c] = o.sk;
    aux[(size_t)7 * n + c] = o.sw;
    aux[(size_t)8 * n + c] = o.beta;
    aux[(size_t)9 * n + c] = o.Sr;
}

// The 11 cell values the SST face flux uses (see sst_face).
template <typename T>
__device__ __forceinline__ void sst_cell_x(int n, int c, T rho0, const T *__restrict__ M, const T *__restrict__ K,
                                           const T *__restrict__ W, const T *__restrict__ aux, T x[11]) {
    x[0] = rho0 + M[c];
    x[1] = M[(size_t)n + c];
    x[2] = M[(size_t)2 * n + c];
    x[3] = K[c];
    x[4] = W[c];
#pragma unroll
    for (int i = 0; i < 6; ++i) x[5 + i] = aux[(size_t)i * n + c];
}

// IMPL: the implicit variant's system rows into J (see kSysPlanes) instead of the update.
template <typename T, bool IMPL>
__global__ void __launch_bounds__(256) k_sst_b(Geo<T> g, const int32_t *__restrict__ bzg, const T *__restrict__ M,
                                               const T *__restrict__ K, const T *__restrict__ W,
                                               T *__restrict__ aux, T *__restrict__ K1, T *__restrict__ W1,
                                               T *__restrict__ tau, T *__restrict__ nut, T *__restrict__ J,
                                               StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T xc[11];
    sst_cell_x(n, c, p.rho0, M, K, W, aux, xc);
    T net_k = 0, net_w = 0;
    SstRow<T> row{T(0), T(0)};
    T ck[4] = {T(0), T(0), T(0), T(0)}, cw[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        if (nb == -1) continue;
        T tk, tw;
        if (nb >= 0) {
            T xn[11];
            sst_cell_x(n, nb, p.rho0, M, K, W, aux, xn);
            sst_face<T, T>(xc, xn, g.nlx[si], g.nly[si], g.rfx[si], g.rfy[si], g.qx[si], g.qy[si], tk, tw);
            if constexpr (IMPL)
                sst_row_edge<T, T>(xc, xn, g.nlx[si], g.nly[si], g.rfx[si], g.rfy[si], g.qx[si], g.qy[si], row, ck[s], cw[s]);
        } else {
            const int b = -2 - nb;
            sst_bface<T, T>(xc, bzg[b] != 0, T(g.b_ux[b]), T(g.b_uy[b]), T(g.b_k[b]), T(g.b_w[b]), g.nlx[si], g.nly[si],
                            g.rfx[si], g.rfy[si], T(g.b_l[b] / g.b_dperp[b]), tk, tw);
            if constexpr (IMPL)
                sst_row_bedge<T, T>(xc, bzg[b] != 0, T(g.b_ux[b]), T(g.b_uy[b]), g.nlx[si], g.nly[si],
                                    T(g.b_l[b] / g.b_dperp[b]), row);
        }
        net_k += tk;
        net_w += tw;
    }
    aux[(size_t)10 * n + c] = net_k;
    aux[(size_t)11 * n + c] = net_w;
    aux[(size_t)12 * n + c] = M[c];
    aux[(size_t)13 * n + c] = M[(size_t)n + c];
    aux[(size_t)14 * n + c] = M[(size_t)2 * n + c];
    if constexpr (IMPL) {
        // a periodic cell that is its own neighbour across an edge: that coupling is on the diagonal
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (g.nbr[(size_t)s * n + c] == c) {
                row.dk = row.dk - ck[s];
                row.dw = row.dw - cw[s];
                ck[s] = cw[s] = T(0);
            }
        T Rk, Rw, gk, gw;
        sst_row_finish<T, T>(xc[0], xc[3], xc[4], net_k, net_w, aux[(size_t)6 * n + c], aux[(size_t)7 * n + c],
                             aux[(size_t)8 * n + c], g.inv_area[c], p, sst_params(p), row, Rk, Rw, gk, gw);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            J[(size_t)s * n + c] = ck[s] * gk;
            J[(size_t)(4 + s) * n + c] = cw[s] * gw;
        }
        J[(size_t)8 * n + c] = Rk;
        J[(size_t)9 * n + c] = Rw;
        J[(size_t)14 * n + c] = aux[(size_t)9 * n + c];
        return;
    }
    T k1, w1, nt;
    sst_update<T, T>(xc[0], xc[3], xc[4], net_k, net_w, aux[(size_t)6 * n + c], aux[(size_t)7 * n + c],
                     aux[(size_t)8 * n + c], aux[(size_t)9 * n + c], T(g.wdist[c]), g.inv_area[c], p, sst_params(p),
                     k1, w1, nt);
    K1[c] = k1;
    W1[c] = w1;
    nut[c] = nt;
    tau[c] = T(3) * (p.nu + nt);
}

// ---- ring-tiled SST: gradients, closure, face fluxes and update in one launch ----
// The layout of the ring-tiled stage sweeps (one workgroup per tile, extended halo lists):
//   phase 0: rho, u, v, k, omega of tile cell t and ext cell t into LDS; the edge data of tile
//            cell t and of ring-1 cell t into registers;
//   phase 1: LSQ gradients of u, v, k, omega and the cell-local closure (sst_local) of tile cell t
//            and ring-1 cell t; grad k, grad omega, Gamma_k, Gamma_omega into LDS;
//   phase 2: face fluxes of tile cell t with its neighbours' data from LDS, point-implicit update,
//            nu_t and tau.  AUX: also store the aux planes (the adjoint reads them).
// LDS, cell-major: Vv [Wv][8] (u, v, k, omega, rho, 3 unused), Vx [Wg][6] (dk/dx, dk/dy, dw/dx,
// dw/dy, Gamma_k, Gamma_w).  Interior edges are summed in straight-line code (an edge without an
// interior neighbour reads row 0 with weight 0), boundary edges after them in a branch.
// Row position of the SST cell data x = (rho, u, v, k, omega, dk/dx, dk/dy, dw/dx, dw/dy, Gamma_k,
// Gamma_w) in a cell-major LDS row: u, v, k, omega first (one 16-byte read for the gradients).
__host__ __device__ constexpr int xpos(int i) { return i == 0 ? 4 : (i <= 4 ? i - 1 : i); }

// RS: LDS row stride; u, v, k, omega at row offsets 0..3.
template <typename T, int S, int RS = 8>
__device__ __forceinline__ void sst_grad_ring(const Geo<T> &g, const int32_t *__restrict__ bzg, const int nb[S],
                                              const int col[S], const T cxs[S], const T cys[S], const T *Vv,
                                              T ux, T uy, T kc, T wc, T gu[2], T gv[2], T gk[2], T gw[2]) {
    gu[0] = gu[1] = gv[0] = gv[1] = gk[0] = gk[1] = gw[0] = gw[1] = T(0);
    bool bnd = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool in = nb[s] >= 0;
        bnd = bnd || nb[s] <= -2;
        const int r = in ? col[s] : 0;
        const T wx = in ? cxs[s] : T(0), wy = in ? cys[s] : T(0);
        const T du = Vv[r * RS + 0] - ux, dv = Vv[r * RS + 1] - uy, dk = Vv[r * RS + 2] - kc, dw = Vv[r * RS + 3] - wc;
        gu[0] += wx * du; gu[1] += wy * du;
        gv[0] += wx * dv; gv[1] += wy * dv;
        gk[0] += wx * dk; gk[1] += wy * dk;
        gw[0] += wx * dw; gw[1] += wy * dw;
    }
    if (bnd) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] > -2) continue;
            const int b = -2 - nb[s];
            if (bzg[b]) continue;   // zero-gradient edge: the ghost equals the cell
            const T du = T(g.b_ux[b]) - ux, dv = T(g.b_uy[b]) - uy, dk = T(g.b_k[b]) - kc, dw = T(g.b_w[b]) - wc;
            gu[0] += cxs[s] * du; gu[1] += cys[s] * du;
            gv[0] += cxs[s] * dv; gv[1] += cys[s] * dv;
            gk[0] += cxs[s] * dk; gk[1] += cys[s] * dk;
            gw[0] += cxs[s] * dw; gw[1] += cys[s] * dw;
        }
    }
}

// IMPL: the implicit variant's system rows into J (see kSysPlanes) instead of the update.
template <typename T, int S, bool AUX, bool IMPL, bool G64 = false>
__global__ void __launch_bounds__(kTileCells, sizeof(T) == 4 ? 4 : 2)
    k_sst_ring(Geo<T> g, RingTiles rt, const int16_t *__restrict__ lnb, int Wv, int Wg,
               const int32_t *__restrict__ bzg, const T *__restrict__ M, const T *__restrict__ K,
               const T *__restrict__ W, T *__restrict__ aux, T *__restrict__ K1, T *__restrict__ W1,
               T *__restrict__ tau, T *__restrict__ nut, T *__restrict__ J, StepPar<T> p) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *Vv = reinterpret_cast<T *>(smem);
    T *Vx = Vv + 8 * Wv;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const int start = tile * kTileCells;
    const int ncell = min(kTileCells, g.n - start);
    const int x0 = rt.ptr[tile], nx = rt.ptr[tile + 1] - x0, n1 = rt.n1[tile];
    const int t = threadIdx.x;
    const int n = g.n;
    const bool own = t < ncell, ext = t < nx, ring1 = t < n1;
    const int c = start + t;
    const SstParams<T> q = sst_params(p);

    // ---- phase 0 ----
    T rho = T(0), ux = T(0), uy = T(0), kc = T(0), wc = T(0), dc = T(0), ia = T(0);
    int nb[S], col[S];
    T cxs[S], cys[S], nlx[S], nly[S], rx[S], ry[S], qx[S], qy[S];
    if (own) {
        const T drho = M[c];
        rho = p.rho0 + drho;
        ux = M[(size_t)n + c];
        uy = M[(size_t)2 * n + c];
        kc = K[c];
        wc = W[c];
        if constexpr (AUX) {
            aux[(size_t)12 * n + c] = drho;
            aux[(size_t)13 * n + c] = ux;
            aux[(size_t)14 * n + c] = uy;
        }
        T mi[3];
        edges_of<T, S, G64>(g, lnb, n, c, c, col, nb, nlx, nly, rx, ry, qx, qy, cxs, cys, mi, ia);
        dc = T(g.wdist[c]);
        Vv[t * 8 + 0] = ux;
        Vv[t * 8 + 1] = uy;
        Vv[t * 8 + 2] = kc;
        Vv[t * 8 + 3] = wc;
        Vv[t * 8 + 4] = rho;
    }
    T hr = T(0), hu = T(0), hvv = T(0), hk = T(0), hw = T(0), hd = T(0);
    int hnb[S], hcol[S];
    T hcx[S], hcy[S];
    if (ext) {
        const int hc = rt.cell[x0 + t];
        hr = p.rho0 + M[hc];
        hu = M[(size_t)n + hc];
        hvv = M[(size_t)2 * n + hc];
        hk = K[hc];
        hw = W[hc];
        const int j = kTileCells + t;
        Vv[j * 8 + 0] = hu;
        Vv[j * 8 + 1] = hvv;
        Vv[j * 8 + 2] = hk;
        Vv[j * 8 + 3] = hw;
        Vv[j * 8 + 4] = hr;
        if (ring1) {
            // LSQ coefficients formed as in the cell's own tile (see k_stage_ring)
            T hnlx[S], hnly[S], hrx[S], hry[S], hqx[S], hqy[S], hmi[3], hia;
            edges_of<T, S, G64>(g, rt.lnb, rt.n_ext, x0 + t, hc, hcol, hnb, hnlx, hnly, hrx, hry, hqx, hqy, hcx, hcy,
                             hmi, hia);
            hd = T(g.wdist[hc]);
        }
    }
    // ring-2 cells beyond one per thread (tiles of stretched cells): their values only
    for (int e = t + kTileCells; e < nx; e += kTileCells) {
        const int ec = rt.cell[x0 + e];
        const int j = kTileCells + e;
        Vv[j * 8 + 0] = M[(size_t)n + ec];
        Vv[j * 8 + 1] = M[(size_t)2 * n + ec];
        Vv[j * 8 + 2] = K[ec];
        Vv[j * 8 + 3] = W[ec];
        Vv[j * 8 + 4] = p.rho0 + M[ec];
    }
    __syncthreads();

    // ---- phase 1 ----
    if (ring1) {
        T gu[2], gv[2], gk[2], gw[2];
        sst_grad_ring<T, S>(g, bzg, hnb, hcol, hcx, hcy, Vv, hu, hvv, hk, hw, gu, gv, gk, gw);
        const SstLocal<T> o = sst_local<T, T>(hr, hk, hw, gu[0], gu[1], gv[0], gv[1], gk[0], gk[1], gw[0], gw[1], hd, p, q);
        const int j = kTileCells + t;
        Vx[j * 6 + 0] = gk[0];
        Vx[j * 6 + 1] = gk[1];
        Vx[j * 6 + 2] = gw[0];
        Vx[j * 6 + 3] = gw[1];
        Vx[j * 6 + 4] = o.Gk;
        Vx[j * 6 + 5] = o.Gw;
    }
    SstLocal<T> oc{};
    T xc[11];
    if (own) {
        T gu[2], gv[2], gk[2], gw[2];
        sst_grad_ring<T, S>(g, bzg, nb, col, cxs, cys, Vv, ux, uy, kc, wc, gu, gv, gk, gw);
        oc = sst_local<T, T>(rho, kc, wc, gu[0], gu[1], gv[0], gv[1], gk[0], gk[1], gw[0], gw[1], dc, p, q);
        Vx[t * 6 + 0] = gk[0];
        Vx[t * 6 + 1] = gk[1];
        Vx[t * 6 + 2] = gw[0];
        Vx[t * 6 + 3] = gw[1];
        Vx[t * 6 + 4] = oc.Gk;
        Vx[t * 6 + 5] = oc.Gw;
        xc[0] = rho; xc[1] = ux; xc[2] = uy; xc[3] = kc; xc[4] = wc;
        xc[5] = gk[0]; xc[6] = gk[1]; xc[7] = gw[0]; xc[8] = gw[1]; xc[9] = oc.Gk; xc[10] = oc.Gw;
        if constexpr (AUX) {
#pragma unroll
            for (int i = 0; i < 6; ++i) aux[(size_t)i * n + c] = xc[5 + i];
            aux[(size_t)6 * n + c] = oc.sk;
            aux[(size_t)7 * n + c] = oc.sw;
            aux[(size_t)8 * n + c] = oc.beta;
            aux[(size_t)9 * n + c] = oc.Sr;
        }
    }
    __syncthreads();
    if (!own) return;

    // ---- phase 2: fluxes (interior edges straight-line, boundary edges after) and the update ----
    T net_k = 0, net_w = 0;
    bool bnd = false;
    SstRow<T> row{T(0), T(0)};
    T ck[S], cw[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool in = nb[s] >= 0;
        bnd = bnd || nb[s] <= -2;
        const int l = in ? col[s] : 0;
        T xn[11];
        xn[0] = Vv[l * 8 + 4];
#pragma unroll
        for (int i = 0; i < 4; ++i) xn[1 + i] = Vv[l * 8 + i];
#pragma unroll
        for (int i = 0; i < 6; ++i) xn[5 + i] = Vx[l * 6 + i];
        T tk, tw;
        sst_face<T, T>(xc, xn, nlx[s], nly[s], rx[s], ry[s], qx[s], qy[s], tk, tw);
        net_k += in ? tk : T(0);
        net_w += in ? tw : T(0);
        if constexpr (IMPL) {
            SstRow<T> re{T(0), T(0)};
            T a, b;
            sst_row_edge<T, T>(xc, xn, nlx[s], nly[s], rx[s], ry[s], qx[s], qy[s], re, a, b);
            row.dk += in ? re.dk : T(0);
            row.dw += in ? re.dw : T(0);
            ck[s] = in ? a : T(0);
            cw[s] = in ? b : T(0);
        }
    }
    if (bnd) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] > -2) continue;
            const int b = -2 - nb[s];
            const size_t si = (size_t)s * n + c;
            T tk, tw;
            sst_bface<T, T>(xc, bzg[b] != 0, T(g.b_ux[b]), T(g.b_uy[b]), T(g.b_k[b]), T(g.b_w[b]), g.nlx[si], g.nly[si],
                            g.rfx[si], g.rfy[si], T(g.b_l[b] / g.b_dperp[b]), tk, tw);
            net_k += tk;
            net_w += tw;
            if constexpr (IMPL)
                sst_row_bedge<T, T>(xc, bzg[b] != 0, T(g.b_ux[b]), T(g.b_uy[b]), g.nlx[si], g.nly[si],
                                    T(g.b_l[b] / g.b_dperp[b]), row);
        }
    }
    if constexpr (AUX) {
        aux[(size_t)10 * n + c] = net_k;
        aux[(size_t)11 * n + c] = net_w;
    }
    if constexpr (IMPL) {
        // a periodic cell that is its own neighbour across an edge: that coupling is on the diagonal
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (g.nbr[(size_t)s * n + c] == c) {   // nb[] holds tile-local codes here
                row.dk -= ck[s];
                row.dw -= cw[s];
                ck[s] = cw[s] = T(0);
            }
        T Rk, Rw, gk, gw;
        sst_row_finish<T, T>(rho, kc, wc, net_k, net_w, oc.sk, oc.sw, oc.beta, ia, p, q, row, Rk, Rw, gk, gw);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            J[(size_t)s * n + c] = ck[s] * gk;
            J[(size_t)(4 + s) * n + c] = cw[s] * gw;
        }
        J[(size_t)8 * n + c] = Rk;
        J[(size_t)9 * n + c] = Rw;
        J[(size_t)14 * n + c] = oc.Sr;
        return;
    }
    T k1, w1, nt;
    sst_update<T, T>(rho, kc, wc, net_k, net_w, oc.sk, oc.sw, oc.beta, oc.Sr, dc, ia, p, q, k1, w1, nt);
    K1[c] = k1;
    W1[c] = w1;
    nut[c] = nt;
    tau[c] = T(3) * (p.nu + nt);
}

// ----------------------------------------------------------------------------------------------
// Reductions (FP64, deterministic two-pass: per-block partials in a fixed grid, then one block).
// ----------------------------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_store(double v[NV], double *partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_down(v[k], off, 64);
    __shared__ double sh[NV][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) partial[(size_t)blockIdx.x * NV + k] = sh[k][0] + sh[k][1] + sh[k][2] + sh[k][3];
}

template <int NV>
__global__ void __launch_bounds__(256) k_finish(const double *__restrict__ partial, int nblocks, double *__restrict__ out) {
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += partial[(size_t)b * NV + k];
    block_store<NV>(v, out);
}

// sum of an n-array
template <typename T>
__global__ void __launch_bounds__(256) k_sum(int n, const T *__restrict__ x, double *__restrict__ partial) {
    double v[1] = {0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) v[0] += (double)x[c];
    block_store<1>(v, partial);
}

// sum |u_new - u_old|^2, sum |u_new|^2
template <typename T>
__global__ void __launch_bounds__(256) k_residual(int n, const T *__restrict__ Mn, const T *__restrict__ Mo,
                                                  double *__restrict__ partial) {
    double v[2] = {0, 0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double ux = Mn[(size_t)n + c], uy = Mn[(size_t)2 * n + c];
        const double dx = ux - (double)Mo[(size_t)n + c], dy = uy - (double)Mo[(size_t)2 * n + c];
        v[0] += dx * dx + dy * dy;
        v[1] += ux * ux + uy * uy;
    }
    block_store<2>(v, partial);
}

// sum A rho, sum A rho u
template <typename T>
__global__ void __launch_bounds__(256) k_totals(Geo<T> g, const T *__restrict__ M, double rho0, double *__restrict__ partial) {
    double v[3] = {0, 0, 0};
    const int n = g.n;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double rho = rho0 + (double)M[c];
        const double A = g.area[c];
        v[0] += A * rho;
        v[1] += A * rho * (double)M[(size_t)n + c];
        v[2] += A * rho * (double)M[(size_t)2 * n + c];
    }
    block_store<3>(v, partial);
}

// force on selected wall edges and the smooth reversed-flow length
template <typename T>
__global__ void __launch_bounds__(256) k_forces(Geo<T> g, const T *__restrict__ M, double rho0, double nu,
                                                unsigned long long mask, int jr_group, double jr_xmin, double eps,
                                                double *__restrict__ partial) {
    double v[3] = {0, 0, 0};
    const int n = g.n;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < g.nb; b += gridDim.x * blockDim.x) {
        const int kind = g.b_kind[b];
        if (kind != kWall && kind != kMovingWall) continue;
        const int grp = g.b_group[b];
        const int c = g.b_cell[b];
        const double rho = rho0 + (double)M[c];
        const double rux = (double)M[(size_t)n + c] - g.b_ux[b], ruy = (double)M[(size_t)2 * n + c] - g.b_uy[b];
        const double nx = g.b_nx[b], ny = g.b_ny[b], l = g.b_l[b], dp = g.b_dperp[b];
        const double un = rux * nx + ruy * ny;
        const double mu = rho * nu;
        const double tx = mu * (rux - un * nx) / dp, ty = mu * (ruy - un * ny) / dp;
        const double dpres = (rho - rho0) / 3.0;
        if ((mask >> grp) & 1ull) {
            v[0] += l * (dpres * nx + tx);
            v[1] += l * (dpres * ny + ty);
        }
        if (grp == jr_group && g.b_xfx[b] > jr_xmin) v[2] += l * 0.5 * (1.0 - tanh(tx / eps));
    }
    block_store<3>(v, partial);
}

// ----------------------------------------------------------------------------------------------
// Import / export between the caller's FP64 user-order arrays and the internal state.
// ----------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_import_f(Geo<T> g, const double *__restrict__ fu, T *__restrict__ F, double rho0) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int u = g.perm[c];
#pragma unroll
    for (int a = 0; a < 9; ++a) F[(size_t)a * g.n + c] = T(fu[(size_t)a * g.n + u] - wt<double>(a) * rho0);
}

template <typename T>
__global__ void k_export_f(Geo<T> g, const T *__restrict__ F, double *__restrict__ fu, double rho0) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int u = g.perm[c];
#pragma unroll
    for (int a = 0; a < 9; ++a) fu[(size_t)a * g.n + u] = (double)F[(size_t)a * g.n + c] + wt<double>(a) * rho0;
}

// f = f_eq(rho, u) (Step 0), from user-order rho [n], u [n][2]
template <typename T>
__global__ void k_init_feq(Geo<T> g, const double *__restrict__ rho_u, const double *__restrict__ vel_u,
                           T *__restrict__ F, double rho0) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int u = g.perm[c];
    const double rho = rho_u[u], ux = vel_u[2 * (size_t)u], uy = vel_u[2 * (size_t)u + 1];
#pragma unroll
    for (int a = 0; a < 9; ++a) F[(size_t)a * g.n + c] = T(dfeq<double>(a, rho - rho0, rho, ux, uy));
}

template <typename T>
__global__ void k_import_scalar(Geo<T> g, const double *__restrict__ su, T *__restrict__ S) {
    const int c = cell_index();
    if (c >= g.n) return;
    S[c] = T(su[g.perm[c]]);
}

template <typename T>
__global__ void k_export_scalar(Geo<T> g, const T *__restrict__ S, double add, double *__restrict__ su) {
    const int c = cell_index();
    if (c >= g.n) return;
    su[g.perm[c]] = (double)S[c] + add;
}

template <typename T>
__global__ void k_export_vel(Geo<T> g, const T *__restrict__ M, double *__restrict__ vu) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int u = g.perm[c];
    vu[2 * (size_t)u] = (double)M[(size_t)g.n + c];
    vu[2 * (size_t)u + 1] = (double)M[(size_t)2 * g.n + c];
}

// macro variables of the current f (after import / init)
template <typename T>
__global__ void k_macro(int n, const T *__restrict__ F, T *__restrict__ M, T rho0) {
    const int c = cell_index();
    if (c >= n) return;
    T d[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = F[(size_t)a * n + c];
    T drho, rho, ux, uy;
    moments(d, rho0, drho, rho, ux, uy);
    M[c] = drho;
    M[(size_t)n + c] = ux;
    M[(size_t)2 * n + c] = uy;
}

template <typename T>
__global__ void k_fill(int n, T *__restrict__ x, T v) {
    const int c = cell_index();
    if (c < n) x[c] = v;
}

}  // namespace fvlbm
