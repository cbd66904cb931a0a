// The ring-tiled stage sweep with two threads per cell (k_stage_pair).
//
// The same computation as k_stage_ring (Section 3.1: the LSQ gradient, the convection term of
// Eq. (advection), the stage solve of Eq. (fnewstage), the combination of Eq. (imextwo)), with the
// nine directions of a cell split over a pair of adjacent lanes: thread 2p + h of a workgroup works
// on tile cell p (and on ext cell p), h = 0 on the rest direction and the axis directions 1-4,
// h = 1 on the diagonal directions 5-8.  Each thread then holds half the per-direction state of
// k_stage_ring (stage values, gradients, convection sums, epilogue operands), so twice as many waves
// fit in the registers.  The moments that couple the directions (density and momentum, for the
// equilibria, the ghost states and the stage solves) are summed per lane and exchanged between the
// two lanes of a pair with one DPP move; a + b = b + a in IEEE arithmetic, so both lanes hold
// identical moments.  LDS holds the same rows as in k_stage_ring; each lane reads and writes its
// half of a row.
#pragma once

#include "kernels.h"

namespace fvlbm {

// The directions of one lane of a pair.  The diagonals are the axes turned by 45 degrees
// (e_{5+k} = e_{1+k} + e_{1+(k+1) mod 4}), so direction k = 0..3 of either half has
// e = (1, h), (-h, 1), (-1, -h), (h, -1).
template <typename T>
struct Half {
    int h;    // 0: rest and axes 1-4; 1: diagonals 5-8
    T hv;     // h as a value
    T w;      // weight of the half's moving directions, 1/9 or 1/36
    __device__ __forceinline__ T ex(int k) const { return k == 0 ? T(1) : (k == 1 ? -hv : (k == 2 ? T(-1) : hv)); }
    __device__ __forceinline__ T ey(int k) const { return k == 0 ? hv : (k == 1 ? T(1) : (k == 2 ? -hv : T(-1))); }
};

// The partner lane's value (quad_perm [1, 0, 3, 2]: lanes 2p and 2p + 1 swap).
__device__ __forceinline__ int pair_swap_i(int x) { return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ float pair_swap(float x) { return __int_as_float(pair_swap_i(__float_as_int(x))); }
__device__ __forceinline__ double pair_swap(double x) {
    const unsigned long long v = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)pair_swap_i((int)(unsigned)v), hi = (unsigned)pair_swap_i((int)(unsigned)(v >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ uint64_t pair_swap(uint64_t x) {
    const unsigned lo = (unsigned)pair_swap_i((int)(unsigned)x), hi = (unsigned)pair_swap_i((int)(unsigned)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <typename T>
__device__ __forceinline__ T pair_sum(T x) { return x + pair_swap(x); }

// Density deviation and velocity of a cell from its values on the pair: v[k] the lane's moving
// directions, v0 the rest direction (counted by half 0).
template <typename T>
__device__ __forceinline__ void pair_moments(const Half<T> &hf, T v0, const T v[4], T rho0, T &drho, T &rho, T &ux,
                                             T &uy) {
    T s = hf.h == 0 ? v0 : T(0), jx = T(0), jy = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        s += v[k];
        jx += hf.ex(k) * v[k];
        jy += hf.ey(k) * v[k];
    }
    s = pair_sum(s);
    jx = pair_sum(jx);
    jy = pair_sum(jy);
    drho = s;
    rho = rho0 + s;
    const T r = recip(rho);
    ux = jx * r;
    uy = jy * r;
}

// Equilibrium deviations (the second-order D2Q9 equilibrium, as dfeq) of the lane's direction k
// and of the rest direction.
template <typename T>
__device__ __forceinline__ T pair_feq(const Half<T> &hf, int k, T drho, T rho, T ux, T uy) {
    const T eu = hf.ex(k) * ux + hf.ey(k) * uy;
    return hf.w * (drho + rho * (T(3) * eu + T(4.5) * eu * eu - T(1.5) * (ux * ux + uy * uy)));
}
template <typename T>
__device__ __forceinline__ T pair_feq0(T drho, T rho, T ux, T uy) {
    return T(4.0 / 9.0) * (drho + rho * (-T(1.5) * (ux * ux + uy * uy)));
}

// The stage solve f = (rhs + a f_eq(rhs)) / (1 + a) (as stage_collide) on the pair.
template <typename T>
__device__ __forceinline__ void pair_collide(const Half<T> &hf, T r0, const T r[4], T a, T rho0, T &o0, T o[4]) {
    T drho, rho, ux, uy;
    pair_moments(hf, r0, r, rho0, drho, rho, ux, uy);
    const T inv = recip(T(1) + a);
    o0 = (r0 + a * pair_feq0(drho, rho, ux, uy)) * inv;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = (r[k] + a * pair_feq(hf, k, drho, rho, ux, uy)) * inv;
}

// Ghost deviations of the lane's directions at boundary edge b (as ghost_state: non-equilibrium
// extrapolation; walls replace every direction, open boundaries the incoming ones).
template <typename T>
__device__ __forceinline__ void pair_ghost(const Geo<T> &g, const Half<T> &hf, int b, T nlx, T nly, const T gc[4],
                                           T drho, T rho, T ux, T uy, T gb[4]) {
    const int kind = g.b_kind[b];
    const T ubx = T(g.b_ux[b]), uby = T(g.b_uy[b]), rb = T(g.b_rho[b]), drb = T(g.b_drho[b]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T en = hf.ex(k) * nlx + hf.ey(k) * nly;
        const T neq = gc[k] - pair_feq(hf, k, drho, rho, ux, uy);
        T v;
        if (kind == kWall || kind == kMovingWall) {
            v = pair_feq(hf, k, drho, rho, ubx, uby) + neq;
        } else if (en < T(0)) {
            if (kind == kInlet)
                v = pair_feq(hf, k, drho, rho, ubx, uby) + neq;
            else if (kind == kOutlet)
                v = pair_feq(hf, k, drb, rb, ux, uy) + neq;
            else
                v = pair_feq(hf, k, drb, rb, ubx, uby);
        } else {
            v = gc[k];
        }
        gb[k] = v;
    }
}

// LSQ gradient of the lane's directions (as grad_ring), from the LDS rows of the neighbours;
// BOUNDS: also the stencil bounds of reading r35.
template <typename T, int S, bool BOUNDS = false>
__device__ __forceinline__ void grad_pair(const Geo<T> &g, const Half<T> &hf, int cell, const int nb[S],
                                          const int col[S], const T cxs[S], const T cys[S], const T *V, T rho0, T g0,
                                          const T gc[4], T gx[4], T gy[4], T *dlo = nullptr, T *dhi = nullptr) {
    const int n = g.n;
#pragma unroll
    for (int k = 0; k < 4; ++k) gx[k] = gy[k] = T(0);
    if constexpr (BOUNDS) {
#pragma unroll
        for (int k = 0; k < 4; ++k) dlo[k] = dhi[k] = T(0);
    }
    bool bnd = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool in = nb[s] >= 0;
        bnd = bnd || nb[s] <= -2;
        const int r = in ? col[s] : 0;
        const T wx = in ? cxs[s] : T(0), wy = in ? cys[s] : T(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T d = V[vrow<T>(r, 4 * hf.h + k)] - gc[k];
            gx[k] += wx * d;
            gy[k] += wy * d;
            if constexpr (BOUNDS) {
                dlo[k] = in && d < dlo[k] ? d : dlo[k];
                dhi[k] = in && d > dhi[k] ? d : dhi[k];
            }
        }
    }
    if (bnd) {
        T drho, rho, ux, uy;
        pair_moments(hf, g0, gc, rho0, drho, rho, ux, uy);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] > -2) continue;
            const size_t si = (size_t)s * n + cell;
            T gb[4];
            pair_ghost(g, hf, -2 - nb[s], g.nlx[si], g.nly[si], gc, drho, rho, ux, uy, gb);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T d = gb[k] - gc[k];
                gx[k] += cxs[s] * d;
                gy[k] += cys[s] * d;
                if constexpr (BOUNDS) {
                    dlo[k] = d < dlo[k] ? d : dlo[k];
                    dhi[k] = d > dhi[k] ? d : dhi[k];
                }
            }
        }
    }
}

// Reading r35's scaling of the lane's gradients (as bj_scale).
template <typename T, int S>
__device__ __forceinline__ void bj_pair(const int nb[S], const T rx[S], const T ry[S], const T dlo[4], const T dhi[4],
                                        T gx[4], T gy[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T psi = T(1);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] == -1) continue;
            const T inc = gx[k] * rx[s] + gy[k] * ry[s];
            const T r = inc > T(0) ? dhi[k] / inc : (inc < T(0) ? dlo[k] / inc : T(1));
            psi = r < psi ? r : psi;
        }
        gx[k] *= psi;
        gy[k] *= psi;
    }
}

// Epilogue operands of the lane (as EpiOps): f^n and tau (stages 1, 2), the stored Ga1 (stage 2
// without its recovery) or Q (stage 3); index 0 the rest direction, loaded by both lanes.
template <typename T>
struct PairOps {
    T f0, fn[4], a0, a[4], tc, tc3;
};

template <typename T, int J>
__device__ __forceinline__ void load_pair_ops(const StageBufs<T> &b, int c, int n, size_t hn, PairOps<T> &o,
                                              int recover) {
    if constexpr (J == 0) o.tc = b.tau[c];
    if constexpr (J == 1 || J == 2) {
        o.f0 = b.F_in[c];
#pragma unroll
        for (int k = 0; k < 4; ++k) o.fn[k] = b.F_in[hn + (size_t)k * n + c];
        o.tc = b.tau[c];
    }
    if constexpr (J == 3) {
        o.a0 = b.A[c];
#pragma unroll
        for (int k = 0; k < 4; ++k) o.a[k] = b.A[hn + (size_t)k * n + c];
    }
    if constexpr (J == 2) {
        if (!recover) {
            o.a0 = b.A[c];
#pragma unroll
            for (int k = 0; k < 4; ++k) o.a[k] = b.A[hn + (size_t)k * n + c];
        }
        o.tc3 = b.tau3 ? b.tau3[c] : o.tc;
    }
}

// Stores of the lane's directions of a cell into nine planes: the rest direction by half 0.
template <typename T>
__device__ __forceinline__ void pair_store(const Half<T> &hf, T *__restrict__ P, int c, int n, size_t hn, T v0,
                                           const T v[4]) {
    if (hf.h == 0) P[c] = v0;
#pragma unroll
    for (int k = 0; k < 4; ++k) P[hn + (size_t)k * n + c] = v[k];
}

// Macro variables (rho - rho0, u) of a cell from its values on the pair, written by half 0.
template <typename T>
__device__ __forceinline__ void pair_macro(const Half<T> &hf, T *__restrict__ M, int c, int n, T v0, const T v[4],
                                           T rho0) {
    T drho, rho, ux, uy;
    pair_moments(hf, v0, v, rho0, drho, rho, ux, uy);
    if (hf.h == 0) {
        M[c] = drho;
        M[(size_t)n + c] = ux;
        M[(size_t)2 * n + c] = uy;
    }
}

// The stage epilogues (epilogue1, 2, 3, explicit) on the pair: g0, gc the stage field, ga its
// convection term (zero in the rest direction).
template <typename T, int J>
__device__ __forceinline__ void pair_epilogue(const Half<T> &hf, int c, int n, size_t hn, T g0, const T gc[4],
                                              const T ga[4], const PairOps<T> &o, const StageBufs<T> &b,
                                              const StepPar<T> &p) {
    if constexpr (J == 0) {
        // forward Euler of Eq. (semibgk)
        T drho, rho, ux, uy;
        pair_moments(hf, g0, gc, p.rho0, drho, rho, ux, uy);
        const T itau = recip(o.tc);
        T f0 = g0 + p.dt * ((pair_feq0(drho, rho, ux, uy) - g0) * itau), f[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) f[k] = gc[k] + p.dt * (ga[k] + (pair_feq(hf, k, drho, rho, ux, uy) - gc[k]) * itau);
        pair_store(hf, b.F_out, c, n, hn, f0, f);
        pair_macro(hf, b.M, c, n, f0, f, p.rho0);
    } else if constexpr (J == 1) {
        // f^(2) = solve(f^n + dt/2 Ga1, a = dt/(4 tau)); Ga1 stored unless stage 2 recovers it
        const T h = p.dt * T(0.5);
        T r[4], f20, f2[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = o.fn[k] + h * ga[k];
        pair_collide(hf, o.f0, r, p.dt * T(0.25) * recip(o.tc), p.rho0, f20, f2);
        pair_store(hf, b.out, c, n, hn, f20, f2);
        if (!p.recover) pair_store(hf, b.A, c, n, hn, T(0), ga);
        if (b.M) pair_macro(hf, b.M, c, n, f20, f2, p.rho0);
    } else if constexpr (J == 2) {
        // f^(3) with the stage moments of Eq. (sumimeximplicitnew); Q = f^(3) - dt/6 (Ga1 + Ga2)
        const T itau = recip(o.tc);
        const T a12 = p.dt * T(0.25) * itau;
        T f10, f1[4], fe10, fe1[4];
        {
            T drho, rho, ux, uy;
            pair_moments(hf, o.f0, o.fn, p.rho0, drho, rho, ux, uy);
            const T inv = recip(T(1) + a12);
            fe10 = pair_feq0(drho, rho, ux, uy);
            f10 = (o.f0 + a12 * fe10) * inv;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                fe1[k] = pair_feq(hf, k, drho, rho, ux, uy);
                f1[k] = (o.fn[k] + a12 * fe1[k]) * inv;
            }
        }
        T d2, r2, ux2, uy2;
        pair_moments(hf, g0, gc, p.rho0, d2, r2, ux2, uy2);
        const T h2 = p.dt * T(0.5), h3 = p.dt * T(1.0 / 3.0);
        const T i_h2 = T(2) * recip(p.dt);
        T gs0, rh0, gs[4], rh[4];
        {
            const T fe2 = pair_feq0(d2, r2, ux2, uy2);
            const T ga1 = p.recover ? (g0 + a12 * (g0 - fe2) - o.f0) * i_h2 : o.a0;
            gs0 = ga1;
            rh0 = o.f0 + h2 * gs0 + h3 * ((fe10 - f10) * itau + (fe2 - g0) * itau);
        }
        T m0 = hf.h == 0 ? o.f0 + h2 * gs0 : T(0), mx = T(0), my = T(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T fe2 = pair_feq(hf, k, d2, r2, ux2, uy2);
            const T ga1 = p.recover ? (gc[k] + a12 * (gc[k] - fe2) - o.fn[k]) * i_h2 : o.a[k];
            gs[k] = ga1 + ga[k];
            rh[k] = o.fn[k] + h2 * gs[k] + h3 * ((fe1[k] - f1[k]) * itau + (fe2 - gc[k]) * itau);
            const T mv = o.fn[k] + h2 * gs[k];
            m0 += mv;
            mx += hf.ex(k) * mv;
            my += hf.ey(k) * mv;
        }
        m0 = pair_sum(m0);
        mx = pair_sum(mx);
        my = pair_sum(my);
        const T rho3 = p.rho0 + m0;
        const T ir3 = recip(rho3);
        const T ux3 = mx * ir3, uy3 = my * ir3;
        const T a3 = h3 * recip(o.tc3);
        const T inv3 = recip(T(1) + a3);
        const T h6 = p.dt * T(1.0 / 6.0);
        const T f30 = (rh0 + a3 * pair_feq0(m0, rho3, ux3, uy3)) * inv3;
        T f3[4], q[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            f3[k] = (rh[k] + a3 * pair_feq(hf, k, m0, rho3, ux3, uy3)) * inv3;
            q[k] = f3[k] - h6 * gs[k];
        }
        pair_store(hf, b.out, c, n, hn, f30, f3);
        pair_store(hf, b.A, c, n, hn, f30 - h6 * gs0, q);
    } else {
        // f^{n+1} = Q + dt/3 Ga3 and its macro variables (Step 7)
        const T h3 = p.dt * T(1.0 / 3.0);
        T f[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) f[k] = o.a[k] + h3 * ga[k];
        pair_store(hf, b.F_out, c, n, hn, o.a0, f);
        pair_macro(hf, b.M, c, n, o.a0, f, p.rho0);
    }
}

// One tile per workgroup of 2 x 256 threads; phases as k_stage_ring.
template <typename T, int J, int S, int LIM>
__global__ void __launch_bounds__(2 * kTileCells, 4)
    k_stage_pair(Geo<T> g, RingTiles rt, const int16_t *__restrict__ lnb, int Wv, int Wg, StageBufs<T> b,
                 StepPar<T> p) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *V = reinterpret_cast<T *>(smem);
    T *Gl = V + 8 * Wv;
    const int tile = ring_tile<J == 2>();
    const int start = tile * kTileCells;
    const int ncell = min(kTileCells, g.n - start);
    const int x0 = rt.ptr[tile], nx = rt.ptr[tile + 1] - x0, n1 = rt.n1[tile];
    const int t = threadIdx.x >> 1;
    Half<T> hf;
    hf.h = threadIdx.x & 1;
    hf.hv = T(hf.h);
    hf.w = hf.h ? T(1.0 / 36.0) : T(1.0 / 9.0);
    const int n = g.n;
    const size_t hn = (size_t)(1 + 4 * hf.h) * n;   // the lane's first moving-direction plane
    const bool own = t < ncell, ext = t < nx, ring1 = t < n1;
    const int c = start + t;

    // ---- phase 0 ----
    T g0 = T(0), gc[4];
    PairOps<T> ops;
    int nb[S], col[S];
    T cxs[S], cys[S], nlx[S], nly[S], rx[S], ry[S], qx[S], qy[S], ia = T(0);
    if (own) {
        if constexpr (J == 1) {
            T f0 = b.F_in[c], f[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) f[k] = b.F_in[hn + (size_t)k * n + c];
            pair_collide(hf, f0, f, p.dt * T(0.25) * recip(b.tau[c]), p.rho0, g0, gc);
        } else {
            g0 = b.src[c];
#pragma unroll
            for (int k = 0; k < 4; ++k) gc[k] = b.src[hn + (size_t)k * n + c];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) V[vrow<T>(t, 4 * hf.h + k)] = gc[k];
    }
    T h0 = T(0), hv[4];
    int hc = 0, hnb[S], hcol[S];
    T hcx[S], hcy[S], hrx[S], hry[S];   // hrx, hry: used by the gradient limiter of r35 only
    if (ext) {
        hc = rt.cell[x0 + t];
        if constexpr (J == 1) {
            T f0 = b.F_in[hc], f[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) f[k] = b.F_in[hn + (size_t)k * n + hc];
            pair_collide(hf, f0, f, p.dt * T(0.25) * recip(b.tau[hc]), p.rho0, h0, hv);
        } else {
            // the rest direction only where a ring-1 cell's ghost states need the moments
            h0 = ring1 ? b.src[hc] : T(0);
#pragma unroll
            for (int k = 0; k < 4; ++k) hv[k] = b.src[hn + (size_t)k * n + hc];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) V[vrow<T>(kTileCells + t, 4 * hf.h + k)] = hv[k];
        if (ring1) {
            T hnlx[S], hnly[S], hqx[S], hqy[S], hmi[3], hia;
            cell_edges<T, S>(g, rt.lnb, rt.n_ext, x0 + t, hc, hcol, hnb, hnlx, hnly, hrx, hry, hqx, hqy, hcx, hcy,
                             hmi, hia);
        }
    }
    // ring-2 cells beyond one per pair (tiles of stretched cells): their values only
    for (int e = t + kTileCells; e < nx; e += kTileCells) {
        const int ec = rt.cell[x0 + e];
        T ev[4];
        if constexpr (J == 1) {
            T f0 = b.F_in[ec], f[4], e0;
#pragma unroll
            for (int k = 0; k < 4; ++k) f[k] = b.F_in[hn + (size_t)k * n + ec];
            pair_collide(hf, f0, f, p.dt * T(0.25) * recip(b.tau[ec]), p.rho0, e0, ev);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) ev[k] = b.src[hn + (size_t)k * n + ec];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) V[vrow<T>(kTileCells + e, 4 * hf.h + k)] = ev[k];
    }
    __syncthreads();

    // ---- phase 1 ----
    if (ring1) {
        T hx[4], hy[4];
        if constexpr (LIM == 2) {
            T lo[4], hi[4];
            grad_pair<T, S, true>(g, hf, hc, hnb, hcol, hcx, hcy, V, p.rho0, h0, hv, hx, hy, lo, hi);
            bj_pair<T, S>(hnb, hrx, hry, lo, hi, hx, hy);
        } else {
            grad_pair<T, S>(g, hf, hc, hnb, hcol, hcx, hcy, V, p.rho0, h0, hv, hx, hy);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            Gl[grow<T>(kTileCells + t, 8 * hf.h + 2 * k)] = hx[k];
            Gl[grow<T>(kTileCells + t, 8 * hf.h + 2 * k + 1)] = hy[k];
        }
    }
    T gx[4], gy[4];
    if (own) {
        // the cell's edge data after the ring-1 gradients, so that the two are never live together
        T mi[3];
        cell_edges<T, S>(g, lnb, n, c, c, col, nb, nlx, nly, rx, ry, qx, qy, cxs, cys, mi, ia);
        if constexpr (LIM == 2) {
            T lo[4], hi[4];
            grad_pair<T, S, true>(g, hf, c, nb, col, cxs, cys, V, p.rho0, g0, gc, gx, gy, lo, hi);
            bj_pair<T, S>(nb, rx, ry, lo, hi, gx, gy);
        } else {
            grad_pair<T, S>(g, hf, c, nb, col, cxs, cys, V, p.rho0, g0, gc, gx, gy);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            Gl[grow<T>(t, 8 * hf.h + 2 * k)] = gx[k];
            Gl[grow<T>(t, 8 * hf.h + 2 * k + 1)] = gy[k];
        }
    }
    __syncthreads();
    if (!own) return;

    // ---- phase 2: convection term (interior edges straight-line, boundary edges after) ----
    T acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = T(0);
    bool bnd = false;
    uint64_t cm = 0;   // clip states (LIM == 3, recorded steps): bit 2 (8 s + a - 1) per slot and direction
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool in = nb[s] >= 0;
        bnd = bnd || nb[s] <= -2;
        const int loc = in ? col[s] : 0;
        const T mx = in ? nlx[s] : T(0), my = in ? nly[s] : T(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T end = hf.ex(k) * mx + hf.ey(k) * my;
            const T vn = V[vrow<T>(loc, 4 * hf.h + k)];
            const T up_n = vn + Gl[grow<T>(loc, 8 * hf.h + 2 * k)] * qx[s] + Gl[grow<T>(loc, 8 * hf.h + 2 * k + 1)] * qy[s];
            const T up_c = gc[k] + gx[k] * rx[s] + gy[k] * ry[s];
            T val = end >= T(0) ? up_c : up_n;
            if constexpr (LIM == 1 || LIM == 3) {
                const T lim = clip_between(val, gc[k], vn);
                if constexpr (LIM == 3) {
                    const bool clipped = in && lim != val;
                    const int bit = 16 * s + 8 * hf.h + 2 * k;
                    cm |= (uint64_t)clipped << bit;
                    cm |= (uint64_t)(clipped && lim == gc[k]) << (bit + 1);
                }
                val = lim;
            }
            acc[k] += end * val;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (bnd) {
        T drho, rho, ux, uy;
        pair_moments(hf, g0, gc, p.rho0, drho, rho, ux, uy);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] > -2) continue;
            const int bi = -2 - nb[s];
            const size_t si = (size_t)s * n + c;
            const T bnx = g.nlx[si], bny = g.nly[si], brx = g.rfx[si], bry = g.rfy[si];
            T gb[4];
            pair_ghost(g, hf, bi, bnx, bny, gc, drho, rho, ux, uy, gb);
            const int kind = g.b_kind[bi];
            const bool wall = (kind == kWall || kind == kMovingWall);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T end = hf.ex(k) * bnx + hf.ey(k) * bny;
                const T own_f = gc[k] + Gl[grow<T>(t, 8 * hf.h + 2 * k)] * brx + Gl[grow<T>(t, 8 * hf.h + 2 * k + 1)] * bry;
                const T val = (wall || end < T(0)) ? gb[k] : own_f;
                acc[k] += end * val;
            }
        }
    }
    if constexpr (LIM == 3) {
        cm |= pair_swap(cm);
        if (hf.h == 0) b.clip[c] = cm;
    }
    // the epilogue operands after the convection term (stage 1 reads f^n and tau a second time):
    // they are not live through the gradients and the edge loop
    load_pair_ops<T, J>(b, c, n, hn, ops, p.recover);
    T ga[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ga[k] = -acc[k] * ia;
    pair_epilogue<T, J>(hf, c, n, hn, g0, gc, ga, ops, b, p);
}

}  // namespace fvlbm
