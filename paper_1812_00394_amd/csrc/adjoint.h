// Discrete adjoint of the IMEX step: transposed operators.
//
// The convection term Gamma^a of Eq. (advection) is linear in the stage field g except through the
// boundary ghost states (which depend on the moments of the boundary cell).  Its transpose applied
// to an adjoint field L (one value per cell and direction) is taken in two gathers:
//   adv_T1 (per cell j): with mu_c = -L_c / A_c, every edge whose face value j reconstructs
//           (outgoing directions, e.n > 0) carries weight en (mu_j - mu_N) to g_j and, through the
//           extrapolation g_j + grad g_j . r_f, en (mu_j - mu_N) r_f to the adjoint of grad g_j
//           (Gbar_j).
//   adv_T1b (per cell with boundary edges): boundary edges route their weight through the ghost
//           state's Jacobian (dual numbers), together with the ghost's use in j's own LSQ gradient
//           (c_b . Gbar_j); the inflow angle theta enters through the rotated inlet / far-field
//           velocities.
//   adv_T2 (per cell s): the transposed LSQ gradient, gbar_s += sum_j c_(j->s) . Gbar_j over the
//           neighbours j of s, minus (sum_k c_sk) . Gbar_s.
// The same slot data serves both sides of an edge: seen from the neighbour N, e.n changes sign and
// its reconstruction vector x_f - x_N is the slot's q.
#pragma once

#include "kernels.h"
#include "sst_reverse.h"

namespace fvlbm {

// Value and partial derivatives of the equilibrium deviation dfeq(a, drho, rho0 + drho, ux, uy)
// with respect to drho (through rho as well), ux and uy.
template <typename T>
struct FeqPartials {
    T dr, dux, duy;
};

template <typename T>
__device__ __forceinline__ FeqPartials<T> dfeq_partials(int a, T rho, T ux, T uy) {
    const T w = wt<T>(a);
    const T eu = T(ex(a)) * ux + T(ey(a)) * uy;
    const T poly = T(3) * eu + T(4.5) * eu * eu - T(1.5) * (ux * ux + uy * uy);
    return FeqPartials<T>{w * (T(1) + poly), w * rho * (T(3) * T(ex(a)) + T(9) * eu * T(ex(a)) - T(3) * ux),
                          w * rho * (T(3) * T(ey(a)) + T(9) * eu * T(ey(a)) - T(3) * uy)};
}

// d(ghost state)/d(cell state, theta) contracted with gbar (directions 1..8), in reverse mode:
// adds to gout[0..8] and returns the theta part.  The ghost state (ghost_state in lattice.h) of
// direction a replaced by the boundary is f_eq(rho_g, u_g) + c (g_a - f_eq(rho, u)), with (rho, u)
// the cell's moments and (rho_g, u_g, c) set by the edge kind; theta rotates the velocity of inlet
// and far-field edges (d u_b / d theta = (-u_b,y, u_b,x)).
template <typename T>
__device__ __forceinline__ T ghost_vjp(const Geo<T> &g, int b, T nlx, T nly, const T gc[9], T rho0, const T gbar[9],
                                       T gout[9]) {
    const int kind = g.b_kind[b];
    const T ubx = T(g.b_ux[b]), uby = T(g.b_uy[b]), rb = T(g.b_rho[b]);
    const bool wall = kind == kWall || kind == kMovingWall;
    const bool rot = kind == kInlet || kind == kFarfield;
    T drho, rho, ux, uy;
    moments(gc, rho0, drho, rho, ux, uy);
    T r_b = 0, ux_b = 0, uy_b = 0, ubx_b = 0, uby_b = 0;   // adjoints of drho, ux, uy, u_b
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const T en = T(ex(a)) * nlx + T(ey(a)) * nly;
        const T gb = gbar[a];
        if (!(wall || en < T(0))) {
            gout[a] += gb;           // the cell's own value
            continue;
        }
        if (kind != kFarfield) {
            // + (g_a - f_eq(rho, u)): the non-equilibrium part of the cell
            gout[a] += gb;
            const FeqPartials<T> d = dfeq_partials<T>(a, rho, ux, uy);
            r_b -= gb * d.dr;
            ux_b -= gb * d.dux;
            uy_b -= gb * d.duy;
        }
        if (wall || kind == kInlet) {
            // f_eq(rho, u_b)
            const FeqPartials<T> d = dfeq_partials<T>(a, rho, ubx, uby);
            r_b += gb * d.dr;
            ubx_b += gb * d.dux;
            uby_b += gb * d.duy;
        } else if (kind == kOutlet) {
            // f_eq(rho_b, u)
            const FeqPartials<T> d = dfeq_partials<T>(a, rb, ux, uy);
            ux_b += gb * d.dux;
            uy_b += gb * d.duy;
        } else {
            // far field: f_eq(rho_b, u_b)
            const FeqPartials<T> d = dfeq_partials<T>(a, rb, ubx, uby);
            ubx_b += gb * d.dux;
            uby_b += gb * d.duy;
        }
    }
    // moments: drho = sum g, u = (sum e g) / rho
    const T ir = recip(rho);
#pragma unroll
    for (int i = 0; i < 9; ++i) gout[i] += r_b + (T(ex(i)) - ux) * ir * ux_b + (T(ey(i)) - uy) * ir * uy_b;
    return rot ? ubx_b * (-uby) + uby_b * ubx : T(0);
}

// L, gbar: [9][n] (direction 0 of L unused); Gbar: [16][n].  Every edge except the ghost-state
// parts, which k_adv_T1b adds.
// OWN = false leaves out the own part of the transposed LSQ gradient (the gradient limiter's reverse,
// k_adv_T_bj, adds it from the adjoint of the unlimited gradient).  CLIP: the face-value limiter of
// reading r32 with the clip states of k_clip_states (as the ring-tiled transpose takes them: a
// clipped edge's weight goes to the cell whose value bounded it, from that cell's own edge loop).
template <typename T, bool OWN = true, bool CLIP = false>
__global__ void __launch_bounds__(256) k_adv_T1(Geo<T> g, const T *__restrict__ L, T lscale, T *__restrict__ gbar,
                                                T *__restrict__ Gbar, const uint64_t *__restrict__ clip = nullptr) {
    const int j = cell_index();
    if (j >= g.n) return;
    const int n = g.n;
    T mu[9], gd[9], Gx[9], Gy[9];
    const T ia = g.inv_area[j];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        mu[a] = -(lscale * L[(size_t)a * n + j]) * ia;
        gd[a] = Gx[a] = Gy[a] = T(0);
    }
    // interior edges: interior edges and open-boundary outgoing directions
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + j;
        const int nb = g.nbr[si];
        if (nb == -1) continue;
        const T nlx = g.nlx[si], nly = g.nly[si], rx = g.rfx[si], ry = g.rfy[si];
        if (nb >= 0) {
            const T ian = g.inv_area[nb];
            if constexpr (CLIP) {
                const uint64_t cm = clip[j];
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    const T en = T(ex(a)) * nlx + T(ey(a)) * nly;
                    const int bit = 2 * (8 * s + a - 1);
                    const bool clipped = (cm >> bit) & 1, self = (cm >> (bit + 1)) & 1;
                    const T wa = en * (mu[a] + (lscale * L[(size_t)a * n + nb]) * ian);
                    const T wr = (!clipped && en > T(0)) ? wa : T(0);
                    gd[a] += clipped ? (self ? wa : T(0)) : wr;
                    Gx[a] += wr * rx;
                    Gy[a] += wr * ry;
                }
            } else {
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    const T en = T(ex(a)) * nlx + T(ey(a)) * nly;
                    if (en > T(0)) {
                        const T w = en * (mu[a] + (lscale * L[(size_t)a * n + nb]) * ian);
                        gd[a] += w;
                        Gx[a] += w * rx;
                        Gy[a] += w * ry;
                    }
                }
            }
        } else {
            const int kind = g.b_kind[-2 - nb];
            if (kind == kWall || kind == kMovingWall) continue;
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T en = T(ex(a)) * nlx + T(ey(a)) * nly;
                if (en >= T(0)) {
                    const T w = en * mu[a];
                    gd[a] += w;
                    Gx[a] += w * rx;
                    Gy[a] += w * ry;
                }
            }
        }
    }
    // own part of the transposed LSQ gradient: grad g_j = sum_k c_jk (v_k - g_j)
    if constexpr (OWN) {
        T sx = 0, sy = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const size_t si = (size_t)s * n + j;
            if (g.nbr[si] == -1) continue;
            sx += g.cx[si];
            sy += g.cy[si];
        }
#pragma unroll
        for (int a = 1; a < 9; ++a) gd[a] -= sx * Gx[a] + sy * Gy[a];
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) gbar[(size_t)a * n + j] += gd[a];
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        Gbar[(size_t)(2 * (a - 1)) * n + j] = Gx[a];
        Gbar[(size_t)(2 * (a - 1) + 1) * n + j] = Gy[a];
    }
}

// Interior neighbours' part of the transposed LSQ gradient.  rev[k][s]: the slot of neighbour
// nbr[k][s] that points back to s.
// BJ: also the gradient limiter's bound parts (k_adv_T_bj): a neighbour whose limiting bound was
// this cell's value (its code, the slot it reached this cell through) passes lD on.
template <typename T, bool BJ = false>
__global__ void __launch_bounds__(256) k_adv_T2(Geo<T> g, const int8_t *__restrict__ rev, const T *__restrict__ Gbar,
                                                T *__restrict__ gbar, const T *__restrict__ lD = nullptr,
                                                const int8_t *__restrict__ code = nullptr) {
    const int s0 = cell_index();
    if (s0 >= g.n) return;
    const int n = g.n;
    T acc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) acc[a] = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t si = (size_t)k * n + s0;
        const int j = g.nbr[si];
        if (j < 0) continue;
        const size_t sj = (size_t)rev[si] * n + j;
        const T cx = g.cx[sj], cy = g.cy[sj];
#pragma unroll
        for (int a = 1; a < 9; ++a)
            acc[a] += cx * Gbar[(size_t)(2 * (a - 1)) * n + j] + cy * Gbar[(size_t)(2 * (a - 1) + 1) * n + j];
        if constexpr (BJ) {
            const int8_t back = rev[si];
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const size_t aj = (size_t)(a - 1) * n + j;
                if (code[aj] == back) acc[a] += lD[aj];
            }
        }
    }
#pragma unroll
    for (int a = 1; a < 9; ++a) gbar[(size_t)a * n + s0] += acc[a];
}

// The clip states of the face-value limiter of reading r32 found again from a stage field f and its
// LSQ gradient planes G (k_grad), for the two-kernel transposes: per cell and interior edge slot s
// and direction a, bit 2 (8 s + a - 1) = the edge's upwind value was clipped, the next bit = to the
// cell's own value (the layout the ring-tiled sweeps record).  The upwind value and the clip are
// formed as the two-kernel sweeps form them.
template <typename T>
__global__ void __launch_bounds__(256) k_clip_states(Geo<T> g, const T *__restrict__ f, const T *__restrict__ G,
                                                     uint64_t *__restrict__ clip) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    uint64_t cm = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        if (nb < 0) continue;
        const T nlx = g.nlx[si], nly = g.nly[si], rx = g.rfx[si], ry = g.rfy[si], qx = g.qx[si], qy = g.qy[si];
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const T end = T(ex(a)) * nlx + T(ey(a)) * nly;
            const size_t pa = (size_t)a * n, px = (size_t)(2 * (a - 1)) * n, py = px + n;
            const T vc = f[pa + c], vn = f[pa + nb];
            const T val = end >= T(0) ? vc + G[px + c] * rx + G[py + c] * ry : vn + G[px + nb] * qx + G[py + nb] * qy;
            const T lim = clip_between(val, vc, vn);
            const bool clipped = lim != val;
            const int bit = 2 * (8 * s + a - 1);
            cm |= (uint64_t)clipped << bit;
            cm |= (uint64_t)(clipped && lim == vc) << (bit + 1);
        }
    }
    clip[c] = cm;
}

// Reverse of the gradient limiter of reading r35 on the two-kernel paths (after k_adv_T1 without
// its own part, before k_adv_T1b and k_adv_T2), cell c per thread.  The forward, per direction a of
// the stage field v (f, or its stage solve with a = a_dt / tau1): g the LSQ gradient, lo <= 0 <= hi
// the least and greatest difference v_s - v_c over the stencil (neighbours and ghost states, in slot
// order, the first extreme kept), psi = min(1, min over the edges of hi / (g . r_s) for increments
// g . r_s > 0 and lo / (g . r_s) for negative ones), and the limited gradient psi g.  Where the
// minimum is an edge s*, psi = D / (g . r_s*) with D = hi or lo, so with lambda the adjoint of
// psi g (Gbar on entry):
//   adjoint of g = psi lambda - (lambda . g) (psi / (g . r_s*)) r_s*,
//   adjoint of D = (lambda . g) / (g . r_s*), which goes to the value that set the bound (minus to
// the cell's own): to a ghost state through its Jacobian here, to an interior neighbour through
// lD / code [8][n] (the slot of that neighbour, -1 for none), gathered by k_adv_T2<T, true>.  Gbar
// leaves as the adjoint of g, and the own part of the transposed LSQ gradient is added to gbar.
template <typename T>
__global__ void __launch_bounds__(256) k_adv_T_bj(Geo<T> g, const T *__restrict__ f, const T *__restrict__ tau1,
                                                  T a_dt, T rho0, T *__restrict__ Gbar, T *__restrict__ gbar,
                                                  T *__restrict__ lD, int8_t *__restrict__ code,
                                                  double *__restrict__ dth) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    // the stage field at the cell
    T vc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) vc[a] = f[(size_t)a * n + c];
    if (tau1) {
        T f1[9], fe[9];
        stage_collide(vc, a_dt * recip(tau1[c]), rho0, f1, fe);
#pragma unroll
        for (int a = 0; a < 9; ++a) vc[a] = f1[a];
    }
    T drho, rho, ux, uy;
    moments(vc, rho0, drho, rho, ux, uy);
    // the forward: unlimited gradient and stencil bounds with the slots that set them
    T gx[9], gy[9], lo[9], hi[9];
    int8_t slo[9], shi[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        gx[a] = gy[a] = lo[a] = hi[a] = T(0);
        slo[a] = shi[a] = -1;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        if (nb == -1) continue;
        T v[9];
        if (nb >= 0) {
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = f[(size_t)a * n + nb];
            if (tau1) {
                T f1[9], fe[9];
                stage_collide(v, a_dt * recip(tau1[nb]), rho0, f1, fe);
#pragma unroll
                for (int a = 0; a < 9; ++a) v[a] = f1[a];
            }
        } else {
            ghost(g, -2 - nb, g.nlx[si], g.nly[si], vc, drho, rho, ux, uy, v);
        }
        const T cxs = g.cx[si], cys = g.cy[si];
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const T d = v[a] - vc[a];
            gx[a] += cxs * d;
            gy[a] += cys * d;
            if (d < lo[a]) {
                lo[a] = d;
                slo[a] = (int8_t)s;
            }
            if (d > hi[a]) {
                hi[a] = d;
                shi[a] = (int8_t)s;
            }
        }
    }
    // psi and the edge that sets it; the reverse
    T gbx[4][9];   // adjoints of the ghost states, per boundary slot
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 9; ++a) gbx[s][a] = T(0);
    T own[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) own[a] = T(0);
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        T psi = T(1), inc_s = T(0), rsx = T(0), rsy = T(0);
        int ss = -1;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const size_t si = (size_t)s * n + c;
            if (g.nbr[si] == -1) continue;
            const T rx = g.rfx[si], ry = g.rfy[si];
            const T inc = gx[a] * rx + gy[a] * ry;
            const T r = inc > T(0) ? hi[a] / inc : (inc < T(0) ? lo[a] / inc : T(1));
            if (r < psi) {
                psi = r;
                ss = s;
                inc_s = inc;
                rsx = rx;
                rsy = ry;
            }
        }
        const size_t ga = (size_t)(2 * (a - 1)) * n + c, gb = (size_t)(2 * (a - 1) + 1) * n + c;
        const T lx = Gbar[ga], ly = Gbar[gb];
        T ogx = lx, ogy = ly, dD = T(0);
        int js = -1;
        if (ss >= 0) {
            const T lpsi = lx * gx[a] + ly * gy[a];
            const T q = psi / inc_s;
            ogx = psi * lx - lpsi * q * rsx;
            ogy = psi * ly - lpsi * q * rsy;
            js = inc_s > T(0) ? shi[a] : slo[a];
            dD = lpsi / inc_s;
        }
        Gbar[ga] = ogx;
        Gbar[gb] = ogy;
        const size_t aj = (size_t)(a - 1) * n + c;
        lD[aj] = T(0);
        code[aj] = -1;
        if (js >= 0) {
            own[a] -= dD;
            const int nbj = g.nbr[(size_t)js * n + c];
            if (nbj >= 0) {
                lD[aj] = dD;
                code[aj] = (int8_t)js;
            } else {
                gbx[js][a] += dD;
            }
        }
        // own part of the transposed LSQ gradient, with the unlimited gradient's adjoint
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const size_t si = (size_t)s * n + c;
            if (g.nbr[si] == -1) continue;
            own[a] -= g.cx[si] * ogx + g.cy[si] * ogy;
        }
    }
    // ghost states that set a bound
    T th = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        if (nb > -2) continue;
        bool any = false;
#pragma unroll
        for (int a = 1; a < 9; ++a) any = any || gbx[s][a] != T(0);
        if (any) th += ghost_vjp(g, -2 - nb, g.nlx[si], g.nly[si], vc, rho0, gbx[s], own);
    }
    if (th != T(0)) dth[c] += (double)th;
#pragma unroll
    for (int a = 0; a < 9; ++a) gbar[(size_t)a * n + c] += own[a];
}

}  // namespace fvlbm

namespace fvlbm {

// ----------------------------------------------------------------------------------------------
// Stage collisions, reversed.  With m = (rho - rho0, j_x, j_y), the equilibrium f_eq(m) and
// M^T lam = lam_0 + e_x lam_x + e_y lam_y:
//   f = (rhs + a f_eq(m)) / (1 + a)  gives  rhs_bar = f_bar / (1 + a),
//   m_bar = (d f_eq / d m)^T (a / (1 + a) f_bar),  a_bar = sum f_bar (f_eq - f) / (1 + a),
// and a = dt m_JJ / tau gives tau_bar = -a_bar a / tau.
// ----------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void feq_vjp(T drho, T jx, T jy, T rho0, const T lam[9], T mbar[3]) {
    using D = Dual<T, 3>;
    const D dr = D::var(drho, 0), dx = D::var(jx, 1), dy = D::var(jy, 2);
    const D rho = D(rho0) + dr;
    const D ux = dx / rho, uy = dy / rho;
    mbar[0] = mbar[1] = mbar[2] = T(0);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const D fe = dfeq(a, dr, rho, ux, uy);
        mbar[0] += lam[a] * fe.d[0];
        mbar[1] += lam[a] * fe.d[1];
        mbar[2] += lam[a] * fe.d[2];
    }
}

template <typename T>
__device__ __forceinline__ void raw_moments(const T d[9], T &m0, T &mx, T &my) {
    m0 = mx = my = T(0);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        m0 += d[a];
        mx += T(ex(a)) * d[a];
        my += T(ey(a)) * d[a];
    }
}

// Reverse of the stage solve with the moments taken from rhs itself; adds rhs_bar to out and
// returns a_bar.  f: the stage result, mom: the moments of rhs (= those of f).
template <typename T>
__device__ __forceinline__ T collide_vjp(const T f[9], T m0, T mx, T my, T a, T rho0, const T fbar[9], T out[9]) {
    const T inv = recip(T(1) + a);
    const T rho = rho0 + m0, irho = recip(rho), ux = mx * irho, uy = my * irho;
    T lam[9], mb[3], abar = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        lam[q] = a * inv * fbar[q];
        abar += fbar[q] * (dfeq(q, m0, rho, ux, uy) - f[q]) * inv;
    }
    feq_vjp(m0, mx, my, rho0, lam, mb);
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] += fbar[q] * inv + mb[0] + T(ex(q)) * mb[1] + T(ey(q)) * mb[2];
    return abar;
}

// Buffers of the step reverse.
// y += x over n values (the per-stage SST's two parts of the k^n, omega^n adjoints).
template <typename T>
__global__ void k_add(int n, const T *__restrict__ x, T *__restrict__ y) {
    const int c = cell_index();
    if (c < n) y[c] += x[c];
}

template <typename T>
struct AdjBufs {
    const T *fn, *f2, *f3, *Q, *tau;        // forward data of the step (f^(1) is formed from f^n)
    const T *lnext;   // adjoint of f^{n+1} (the step's output)
    T *lfn;    // adjoint of f^n (written by the third stage's reverse, then accumulated)
    T *lf1, *lf2, *lf3;                     // adjoints of the stage fields
    T *lam;    // input of the transposed convection (adjoint of a convection term)
    T *lg1;    // adjoint of Ga1
    T *ltau;   // adjoint of tau
    // per-stage SST coupling (reading r33): the third stage's relaxation time and the adjoint of it
    // (nullptr: the third stage uses tau, whose adjoint takes its part)
    const T *tau3 = nullptr;
    T *ltau3 = nullptr;
    // gradient limiter of reading r35: the bound parts k_adv_T_bj passes to the neighbours [8][n]
    T *lD = nullptr;
    int8_t *bjc = nullptr;
    // the gradient-plane adjoints of the two-kernel transposes [16][n] (nullptr: the state's own
    // gradient planes, which a recompute on the side stream of a ring-tiled state may be using)
    T *Gb = nullptr;
    // the face-value limiter of r32 on the two-kernel transposes: the stage field [9][n] and the
    // clip states [n] formed again there
    T *sf = nullptr;
    uint64_t *clipr = nullptr;
};

// Reverse of the third stage and of the combination f^{n+1} = Q + dt/3 Ga3, given lf3 (the
// transpose of Ga3 applied to dt/3 lam_{n+1}) and lam_{n+1} = lnext (the adjoint of f^{n+1}).
// Writes lfn (the adjoint of f^n so far), lf2 (Gc2 part), lf1 (Gc1 part), lam (the Ga2 adjoint and
// the Ga1 adjoint so far), ltau.
// lnext_c: the cell's lam_{n+1} when the caller holds it already (nullptr: read here).
// Written in three sections that the scheduler keeps apart (f^(2) and f^(1) are needed only by the
// later ones), which bounds the values live at once.
template <typename T>
__device__ __forceinline__ void adj_stage3_cell(int c, int n, const T lf3[9], const AdjBufs<T> &b, const StepPar<T> &p,
                                                const T *lnext_c = nullptr) {
    const T tc = b.tau[c];
    const T dt = p.dt;
    const T itau = recip(tc);
    // ---- the combination and the third stage: needs f^n, f3, Q ----
    T fn[9], lq[9], l3[9];
    T m0 = 0, mx = 0, my = 0, f3d[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const size_t i = (size_t)a * n + c;
        fn[a] = b.fn[i];
        const T f3a = b.f3[i];
        lq[a] = lnext_c ? lnext_c[a] : b.lnext[i];   // lam_{n+1} = adjoint of Q
        l3[a] = lf3[a] + lq[a];                      // f3 enters Q with weight 1
        // f3 = (rhs3 + a3 f_eq(m3)) / (1 + a3), m3 = m(f^n) + dt/2 m(Ga1 + Ga2), Ga1 + Ga2 = 6 (f3 - Q) / dt
        const T mv = fn[a] + T(3) * (f3a - b.Q[i]);
        m0 += mv;
        mx += T(ex(a)) * mv;
        my += T(ey(a)) * mv;
        f3d[a] = f3a;
    }
    // Q = f3 - dt/6 (Ga1 + Ga2)
    T lg12[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) lg12[a] = -dt * T(1.0 / 6.0) * lq[a];
    const T itau3 = b.tau3 ? recip(b.tau3[c]) : itau;
    const T a3 = dt * T(1.0 / 3.0) * itau3;
    const T inv3 = recip(T(1) + a3);
    const T rho3 = p.rho0 + m0, ir3 = recip(rho3), ux3 = mx * ir3, uy3 = my * ir3;
    T lrhs[9], lfe[9], mb[3], abar = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        lrhs[a] = l3[a] * inv3;
        lfe[a] = a3 * inv3 * l3[a];
        abar += l3[a] * (dfeq(a, m0, rho3, ux3, uy3) - f3d[a]) * inv3;
    }
    T ltau = T(0);
    if (b.tau3)
        b.ltau3[c] = -abar * a3 * itau3;
    else
        ltau = -abar * a3 * itau;
    feq_vjp(m0, mx, my, p.rho0, lfe, mb);
    T lfn[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const T mt = mb[0] + T(ex(a)) * mb[1] + T(ey(a)) * mb[2];   // M^T m3_bar
        lfn[a] = mt + lrhs[a];                                      // through m3 and rhs3
        lg12[a] += dt * T(0.5) * (mt + lrhs[a]);
    }
    // rhs3 = f^n + dt/2 (Ga1 + Ga2) + dt/3 (Gc1 + Gc2)
    T lgc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) lgc[a] = dt * T(1.0 / 3.0) * lrhs[a];
#pragma unroll
    for (int a = 0; a < 9; ++a) b.lam[(size_t)a * n + c] = lg12[a];   // Ga2 adjoint, and the Ga1 adjoint so far
    __builtin_amdgcn_sched_barrier(0);
    // ---- Gc2 = (f_eq(m(f2)) - f2) / tau: needs f2 ----
    {
        T f2[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) f2[a] = b.f2[(size_t)a * n + c];
        T q0, qx, qy;
        raw_moments(f2, q0, qx, qy);
        const T r = p.rho0 + q0, ir = recip(r), vx = qx * ir, vy = qy * ir;
        T l[9], mb2[3];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            l[a] = lgc[a] * itau;
            ltau -= lgc[a] * (dfeq(a, q0, r, vx, vy) - f2[a]) * itau * itau;
        }
        feq_vjp(q0, qx, qy, p.rho0, l, mb2);
#pragma unroll
        for (int a = 0; a < 9; ++a)
            b.lf2[(size_t)a * n + c] = mb2[0] + T(ex(a)) * mb2[1] + T(ey(a)) * mb2[2] - l[a];
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- Gc1 = (f_eq(m(f^n)) - f1) / tau, f1 = the first stage's solve of f^n ----
    {
        T f1[9];
        {
            T fe[9];
            stage_collide(fn, dt * T(0.25) * itau, p.rho0, f1, fe);   // f^(1)
        }
        T q0, qx, qy;
        raw_moments(fn, q0, qx, qy);
        const T r = p.rho0 + q0, ir = recip(r), vx = qx * ir, vy = qy * ir;
        T l[9], mb1[3];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            l[a] = lgc[a] * itau;
            ltau -= lgc[a] * (dfeq(a, q0, r, vx, vy) - f1[a]) * itau * itau;
        }
        feq_vjp(q0, qx, qy, p.rho0, l, mb1);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            lfn[a] += mb1[0] + T(ex(a)) * mb1[1] + T(ey(a)) * mb1[2];
            b.lf1[(size_t)a * n + c] = -l[a];
        }
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) b.lfn[(size_t)a * n + c] = lfn[a];
    b.ltau[c] = ltau;
}

// Reverse of the second stage f2 = solve(f^n + dt/2 Ga1, a2 = dt/(4 tau)) given the complete f2
// adjoint lf2 of cell c: lfn += rhs2_bar; lam_out <- Ga1 adjoint = (its part from the third stage,
// in lam) + dt/2 rhs2_bar; ltau += ...
template <typename T>
// lam_c: the cell's values of lam when the caller holds them already (nullptr: read here).
__device__ __forceinline__ void adj_stage2_cell(int c, int n, const T lf2[9], const AdjBufs<T> &b, T *lam_out,
                                                const StepPar<T> &p, const T *lam_c = nullptr) {
    T f2[9], lr[9];
    const T tc = b.tau[c];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        f2[a] = b.f2[(size_t)a * n + c];
        lr[a] = T(0);
    }
    T m0, mx, my;
    raw_moments(f2, m0, mx, my);
    const T a2 = p.dt * T(0.25) * recip(tc);
    const T abar = collide_vjp(f2, m0, mx, my, a2, p.rho0, lf2, lr);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const size_t i = (size_t)a * n + c;
        b.lfn[i] += lr[a];
        lam_out[i] = (lam_c ? lam_c[a] : b.lam[i]) + p.dt * T(0.5) * lr[a];
    }
    b.ltau[c] += -abar * a2 * recip(tc);
}

// Reverse of the first stage f1 = solve(f^n, a1 = dt/(4 tau)) given the complete f1 adjoint lf1.
template <typename T>
__device__ __forceinline__ void adj_stage1_cell(int c, int n, const T lf1[9], const AdjBufs<T> &b, const StepPar<T> &p) {
    T f1[9], fe[9], fn[9], lr[9];
    const T tc = b.tau[c];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        fn[a] = b.fn[(size_t)a * n + c];
        lr[a] = T(0);
    }
    stage_collide(fn, p.dt * T(0.25) * recip(tc), p.rho0, f1, fe);   // f^(1)
    T m0, mx, my;
    raw_moments(fn, m0, mx, my);
    const T a1 = p.dt * T(0.25) * recip(tc);
    const T abar = collide_vjp(f1, m0, mx, my, a1, p.rho0, lf1, lr);
#pragma unroll
    for (int a = 0; a < 9; ++a) b.lfn[(size_t)a * n + c] += lr[a];
    b.ltau[c] += -abar * a1 * recip(tc);
}

// The stage reverse that follows the transposed convection of stage J (EPI = J, 0: none), for cell
// c with the complete adjoint lf of its stage field: stage 3 (with the combination) leaves the Ga2
// adjoint in lam, stage 2 the Ga1 adjoint in lg1.
// lin_c: the cell's values of the transposed convection's input (lam_{n+1} for stage 3, lam for
// stage 2) when the caller holds them already (nullptr: read here).
template <typename T, int EPI>
__device__ __forceinline__ void adj_stage_epilogue(int c, int n, const T lf[9], const AdjBufs<T> &b, const StepPar<T> &p,
                                                   const T *lin_c = nullptr) {
    if constexpr (EPI == 3)
        adj_stage3_cell(c, n, lf, b, p, lin_c);
    else if constexpr (EPI == 2)
        adj_stage2_cell(c, n, lf, b, b.lg1, p, lin_c);
    else if constexpr (EPI == 1)
        adj_stage1_cell(c, n, lf, b, p);
}

template <typename T, int EPI>
__global__ void __launch_bounds__(256) k_adj_stage(int n, AdjBufs<T> b, StepPar<T> p, const T *__restrict__ lf_in) {
    const int c = cell_index();
    if (c >= n) return;
    T lf[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) lf[a] = lf_in[(size_t)a * n + c];
    adj_stage_epilogue<T, EPI>(c, n, lf, b, p);
}

// Ghost-state part of adv_T1 for cells with boundary edges (after k_adv_T1): the face values on
// walls and incoming directions, and the ghosts' use in the cell's own LSQ gradient, through the
// ghost state's Jacobian.  One thread per cell: boundary edges are ordered by owner cell, and the
// thread of a cell's first boundary edge takes all of them in slot order.  Kept out of k_adv_T1 so
// that its dual-number registers do not limit the occupancy of the all-cell kernel.  With tau1
// given, the field is the stage solve of f with a = a_dt / tau1 (f^(1) from f^n).  EPI = J: the
// cell's stage-J reverse follows (k_adv_T_ring left the cell's adjoint in gbar without it).
template <typename T, int EPI>
__global__ void __launch_bounds__(256) k_adv_T1b(Geo<T> g, const T *__restrict__ f, const T *__restrict__ tau1, T a_dt,
                                                 const T *__restrict__ L, T lscale, T *__restrict__ gbar,
                                                 const T *__restrict__ Gbar, double *__restrict__ dth, T rho0,
                                                 AdjBufs<T> ab, StepPar<T> p) {
    const int b0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (b0 >= g.nb) return;
    const int j = g.b_cell[b0];
    if (b0 > 0 && g.b_cell[b0 - 1] == j) return;
    const int n = g.n;
    T mu[9], gj[9], gd[9], Gx[9], Gy[9];
    const T ia = g.inv_area[j];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        mu[a] = -(lscale * L[(size_t)a * n + j]) * ia;
        gj[a] = f[(size_t)a * n + j];
        gd[a] = T(0);
    }
    if (tau1) {
        T f1[9], fe[9];
        stage_collide(gj, a_dt * recip(tau1[j]), rho0, f1, fe);
#pragma unroll
        for (int a = 0; a < 9; ++a) gj[a] = f1[a];
    }
    Gx[0] = Gy[0] = T(0);
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        Gx[a] = Gbar[(size_t)(2 * (a - 1)) * n + j];
        Gy[a] = Gbar[(size_t)(2 * (a - 1) + 1) * n + j];
    }
    T th = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + j;
        const int nb = g.nbr[si];
        if (nb >= -1) continue;
        const int b = -2 - nb;
        const int kind = g.b_kind[b];
        const bool wall = (kind == kWall || kind == kMovingWall);
        const T nlx = g.nlx[si], nly = g.nly[si], cxs = g.cx[si], cys = g.cy[si];
        T gb_bar[9];
        gb_bar[0] = T(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const T en = T(ex(a)) * nlx + T(ey(a)) * nly;
            gb_bar[a] = cxs * Gx[a] + cys * Gy[a] + ((wall || en < T(0)) ? en * mu[a] : T(0));
        }
        th += ghost_vjp(g, b, nlx, nly, gj, rho0, gb_bar, gd);
    }
    dth[j] += (double)th;
    if constexpr (EPI == 0) {
#pragma unroll
        for (int a = 0; a < 9; ++a) gbar[(size_t)a * n + j] += gd[a];
    } else {
        T lf[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) lf[a] = gbar[(size_t)a * n + j] + gd[a];
        adj_stage_epilogue<T, EPI>(j, n, lf, ab, p);
    }
}

// Ring-tiled transposed convection (adv_T1 and adv_T2 in one launch, ghost parts excepted), in the
// layout of the ring-tiled forward sweeps:
//   phase 0: mu = -L / A of tile cell t and ext cell t into LDS; the edge data of tile cell t and
//            of ring-1 cell t into registers (triangle meshes: their inverse LSQ matrices into
//            LDS; other meshes: the LSQ coefficient of each interior neighbour's slot that points
//            back, c_(j->t), gathered);
//   phase 1: adv_T1 of ring-1 cell t and tile cell t: Gbar (the adjoint of the LSQ gradient) into
//            LDS, and the own part of tile cell t;
//   phase 2: adv_T2 of tile cell t from its neighbours' Gbar in LDS (triangle meshes: c_(j->t) =
//            w M_j^-1 (-d) from neighbour j's inverse LSQ matrix); a cell with boundary edges adds
//            the ghost part (as k_adv_T1b does for the other paths); out += (ACC) or = the sum, or
//            with EPI = J the cell's stage-J reverse follows at once (nothing stored in out).
// LDS, cell-major: V [Wv][8] mu, Gl [Wg][16] Gbar (x, y interleaved), Mi [Wg][3] (S = 3).
// Interior edges are summed in straight-line code (an edge without an interior neighbour reads
// row 0 with weight 0), open-boundary edges after them.
// CLIP: the convection was limited by the face-value clip of reading r32, whose per-edge states the
// forward sweep recorded in clip (StageBufs::clip): an edge whose value was clipped passes its
// adjoint to the cell whose value it took (from that cell's own edge loop: its own value when the
// bound was its own), an unclipped one to the upwind reconstruction as without the limiter.
template <typename T, int S, bool ACC, int EPI, bool CLIP = false>
__global__ void __launch_bounds__(kTileCells, sizeof(T) == 4 ? 3 : 2)
    k_adv_T_ring(Geo<T> g, RingTiles rt, const int16_t *__restrict__ lnb, const int8_t *__restrict__ rev, int Wv,
                 int Wg, const T *__restrict__ L, T lscale, T *__restrict__ out, const T *__restrict__ f,
                 const T *__restrict__ tau1, T a_dt, double *__restrict__ dth, T rho0, AdjBufs<T> ab,
                 StepPar<T> p, const uint64_t *__restrict__ clip = nullptr) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *V = reinterpret_cast<T *>(smem);
    T *Gl = V + 8 * Wv;
    T *Mi = Gl + 16 * Wg;
    // FP64 triangles form the coefficient of a neighbour's edge pointing back, c_(j->t) = w M_j^-1 (-d),
    // from M_j^-1 in LDS; FP32 gathers it from the stored coefficients, the ones its forward uses
    constexpr bool FORM = S == 3 && sizeof(T) == 8;
    // the stage-2 transpose runs the tiles descending, the others ascending (see ring_tile)
    const int tile = ring_tile<EPI != 2>();
    const int start = tile * kTileCells;
    const int ncell = min(kTileCells, g.n - start);
    const int x0 = rt.ptr[tile], nx = rt.ptr[tile + 1] - x0, n1 = rt.n1[tile];
    const int t = threadIdx.x;
    const int n = g.n;
    const bool own = t < ncell, ext = t < nx, ring1 = t < n1;
    const int c = start + t;

    // ---- phase 0 ----
    T mu[9], Lc[9];   // Lc: the cell's input values, kept for the stage-2 / 3 reverse (same arrays)
    int nb[S], col[S];
    T nlx[S], nly[S], rx[S], ry[S], qx[S], qy[S], cxs[S], cys[S], cbx[S], cby[S];
    if (own) {
        T mi[3], ia;
        cell_edges<T, S>(g, lnb, n, c, c, col, nb, nlx, nly, rx, ry, qx, qy, cxs, cys, mi, ia);
        if constexpr (EPI == 2 || EPI == 3) Lc[0] = L[c];
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            Lc[a] = L[(size_t)a * n + c];
            mu[a] = -(lscale * Lc[a]) * ia;
            V[t * 8 + (a - 1)] = mu[a];
        }
        if constexpr (FORM) {
#pragma unroll
            for (int k = 0; k < 3; ++k) Mi[t * 3 + k] = mi[k];
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const size_t si = (size_t)s * n + c;
                cbx[s] = cby[s] = T(0);
                if (nb[s] >= 0) {
                    const size_t sj = (size_t)rev[si] * n + g.nbr[si];
                    cbx[s] = g.cx[sj];
                    cby[s] = g.cy[sj];
                }
            }
        }
    }
    T hmu[9];
    int hnb[S], hcol[S];
    T hnlx[S], hnly[S], hrx[S], hry[S];
    if (ext) {
        const int hc = rt.cell[x0 + t];
        T hqx[S], hqy[S], hcx[S], hcy[S], hmi[3], hia;
        if (ring1) {
            cell_edges<T, S>(g, rt.lnb, rt.n_ext, x0 + t, hc, hcol, hnb, hnlx, hnly, hrx, hry, hqx, hqy, hcx, hcy, hmi,
                             hia);
            if constexpr (FORM) {
#pragma unroll
                for (int k = 0; k < 3; ++k) Mi[(kTileCells + t) * 3 + k] = hmi[k];
            }
        } else {
            hia = g.inv_area[hc];
        }
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            hmu[a] = -(lscale * L[(size_t)a * n + hc]) * hia;
            V[(kTileCells + t) * 8 + (a - 1)] = hmu[a];
        }
    }
    // ring-2 cells beyond one per thread (tiles of stretched cells): their values only
    for (int e = t + kTileCells; e < nx; e += kTileCells) {
        const int ec = rt.cell[x0 + e];
        const T eia = g.inv_area[ec];
#pragma unroll
        for (int a = 1; a < 9; ++a) V[(kTileCells + e) * 8 + (a - 1)] = -(lscale * L[(size_t)a * n + ec]) * eia;
    }
    __syncthreads();

    // ---- phase 1: adv_T1 ----
    // weights of the edges whose face value cell x reconstructs: interior edges (mu_x - mu_N) and
    // outgoing directions of open boundaries (mu_x); gd: the part on g_x itself.  With CLIP, cm holds
    // x's recorded clip states: a clipped edge puts its weight on g_x when the bound was x's value
    // (either upwind side), and nothing on x's gradient
    auto t1 = [&](const T m[9], const int *nbs, const int *cols, const T *nx_, const T *ny_, const T *rx_,
                  const T *ry_, uint64_t cm, T gd[9], T Gx[9], T Gy[9]) {
#pragma unroll
        for (int a = 0; a < 9; ++a) gd[a] = Gx[a] = Gy[a] = T(0);
        bool bnd = false;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bool in = nbs[s] >= 0;
            bnd = bnd || nbs[s] <= -2;
            const int r = in ? cols[s] : 0;
            const T mx = in ? nx_[s] : T(0), my = in ? ny_[s] : T(0);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T en = T(ex(a)) * mx + T(ey(a)) * my;
                if constexpr (CLIP) {
                    const int bit = 2 * (8 * s + a - 1);
                    const bool clipped = (cm >> bit) & 1, self = (cm >> (bit + 1)) & 1;
                    const T wa = en * (m[a] - V[r * 8 + (a - 1)]);
                    const T wr = (!clipped && en > T(0)) ? wa : T(0);
                    gd[a] += clipped ? (self ? wa : T(0)) : wr;
                    Gx[a] += wr * rx_[s];
                    Gy[a] += wr * ry_[s];
                } else {
                    const T w = en > T(0) ? en * (m[a] - V[r * 8 + (a - 1)]) : T(0);
                    gd[a] += w;
                    Gx[a] += w * rx_[s];
                    Gy[a] += w * ry_[s];
                }
            }
        }
        if (bnd) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (nbs[s] > -2) continue;
                const int kind = g.b_kind[-2 - nbs[s]];
                if (kind == kWall || kind == kMovingWall) continue;
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    const T en = T(ex(a)) * nx_[s] + T(ey(a)) * ny_[s];
                    if (en >= T(0)) {
                        const T w = en * m[a];
                        gd[a] += w;
                        Gx[a] += w * rx_[s];
                        Gy[a] += w * ry_[s];
                    }
                }
            }
        }
    };
    if (ring1) {
        T gd[9], Gx[9], Gy[9];
        t1(hmu, hnb, hcol, hnlx, hnly, hrx, hry, CLIP ? clip[rt.cell[x0 + t]] : 0, gd, Gx, Gy);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            Gl[(kTileCells + t) * 16 + 2 * (a - 1)] = Gx[a];
            Gl[(kTileCells + t) * 16 + 2 * (a - 1) + 1] = Gy[a];
        }
    }
    T gd[9], Gx[9], Gy[9];
    if (own) {
        t1(mu, nb, col, nlx, nly, rx, ry, CLIP ? clip[c] : 0, gd, Gx, Gy);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            Gl[t * 16 + 2 * (a - 1)] = Gx[a];
            Gl[t * 16 + 2 * (a - 1) + 1] = Gy[a];
        }
    }
    __syncthreads();
    if (!own) return;

    // ---- phase 2: own LSQ part, then adv_T2 ----
    T sx = 0, sy = 0;
    bool bnd = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        sx += cxs[s];   // zero on unused slots
        sy += cys[s];
        bnd = bnd || nb[s] <= -2;
    }
#pragma unroll
    for (int a = 1; a < 9; ++a) gd[a] -= sx * Gx[a] + sy * Gy[a];
    T acc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) acc[a] = T(0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool in = nb[s] >= 0;
        const int r = in ? col[s] : 0;
        T bx, by;
        if constexpr (FORM) {
            // neighbour r's LSQ coefficient of its edge back to this cell: w M_r^-1 (-d)
            const T dx = rx[s] - qx[s], dy = ry[s] - qy[s];
            const T w = in ? recip(dx * dx + dy * dy) : T(0);
            bx = -w * (Mi[r * 3] * dx + Mi[r * 3 + 1] * dy);
            by = -w * (Mi[r * 3 + 1] * dx + Mi[r * 3 + 2] * dy);
        } else {
            bx = in ? cbx[s] : T(0);
            by = in ? cby[s] : T(0);
        }
#pragma unroll
        for (int a = 1; a < 9; ++a) acc[a] += bx * Gl[r * 16 + 2 * (a - 1)] + by * Gl[r * 16 + 2 * (a - 1) + 1];
    }
    T lf[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        if constexpr (ACC)
            lf[a] = (out[(size_t)a * n + c] + gd[a]) + acc[a];
        else
            lf[a] = gd[a] + acc[a];
    }
    if (bnd) {
        // ghost part of a cell with boundary edges: the face values on walls and incoming
        // directions and the ghosts' use in the cell's own LSQ gradient, through the closed-form
        // Jacobian of the ghost states (the field is f, or its stage solve with a = a_dt / tau1);
        // mu and the cell's gradient adjoint are read back from LDS
        T gj[9], gdb[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            gj[a] = f[(size_t)a * n + c];
            gdb[a] = T(0);
        }
        if (tau1) {
            T f1[9], fe[9];
            stage_collide(gj, a_dt * recip(tau1[c]), rho0, f1, fe);
#pragma unroll
            for (int a = 0; a < 9; ++a) gj[a] = f1[a];
        }
        T th = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] > -2) continue;
            const int b = -2 - nb[s];
            const int kind = g.b_kind[b];
            const bool wall = (kind == kWall || kind == kMovingWall);
            const size_t si = (size_t)s * n + c;
            const T bnx = g.nlx[si], bny = g.nly[si];
            T gb_bar[9];
            gb_bar[0] = T(0);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const T en = T(ex(a)) * bnx + T(ey(a)) * bny;
                gb_bar[a] = cxs[s] * Gl[t * 16 + 2 * (a - 1)] + cys[s] * Gl[t * 16 + 2 * (a - 1) + 1] +
                            ((wall || en < T(0)) ? en * V[t * 8 + (a - 1)] : T(0));
            }
            th += ghost_vjp(g, b, bnx, bny, gj, rho0, gb_bar, gdb);
        }
        dth[c] += (double)th;
#pragma unroll
        for (int a = 0; a < 9; ++a) lf[a] += gdb[a];
    }
    if constexpr (EPI == 0) {
#pragma unroll
        for (int a = 0; a < 9; ++a) out[(size_t)a * n + c] = lf[a];
    } else {
        adj_stage_epilogue<T, EPI>(c, n, lf, ab, p, Lc);
    }
}

// ----------------------------------------------------------------------------------------------
// SST, reversed.  Cell data x = (rho, u, v, k, omega, dk/dx, dk/dy, domega/dx, domega/dy, Gamma_k,
// Gamma_omega); lx its adjoint [11][n]; lnet [2][n] the adjoint of the net k / omega inflow; lown
// [4][n] the adjoint of (dt P / rho, dt (P_w + cross) / rho, beta, S); lgrad [8][n] the adjoint of
// the LSQ gradients of u, v, k, omega; pbar [5][n] (FP64) per-cell parameter adjoints in the order
// (theta, sigma_k1, sigma_w1, beta*, a1).
// ----------------------------------------------------------------------------------------------
struct SstAdj {
    const int32_t *bzg;
    double *pbar;
};

// SB1: reverse of the point-implicit update and of tau = 3 (nu + nu_t) (cell-local: the net
// inflows are aux planes 10, 11 of the forward).
template <typename T>
__global__ void __launch_bounds__(256) k_adj_sst_update(Geo<T> g, SstAdj sa, const T *__restrict__ M,
                                                        const T *__restrict__ K, const T *__restrict__ W,
                                                        const T *__restrict__ aux, const T *__restrict__ lk1,
                                                        const T *__restrict__ lw1, const T *__restrict__ ltau,
                                                        T *__restrict__ lx, T *__restrict__ lnet, T *__restrict__ lown,
                                                        StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T xb[3] = {0, 0, 0}, ob[6];
    SstParBar<T> pb;
    sst_update_rev<T>(p.rho0 + M[c], K[c], W[c], aux[(size_t)10 * n + c], aux[(size_t)11 * n + c], aux[(size_t)6 * n + c],
                      aux[(size_t)7 * n + c], aux[(size_t)8 * n + c], aux[(size_t)9 * n + c], T(g.wdist[c]), g.inv_area[c],
                      p, sst_params(p), lk1[c], lw1[c], T(3) * ltau[c], xb, ob, pb);
    lx[c] += xb[0];
    lx[(size_t)3 * n + c] += xb[1];
    lx[(size_t)4 * n + c] += xb[2];
    lnet[c] = ob[0];
    lnet[(size_t)n + c] = ob[1];
#pragma unroll
    for (int i = 0; i < 4; ++i) lown[(size_t)i * n + c] = ob[2 + i];
    sa.pbar[(size_t)4 * n + c] += (double)pb.a1;
    sa.pbar[(size_t)3 * n + c] += (double)pb.bstar;
}

// SB2: reverse of the face fluxes, gathered per cell j from its own edges and, through the same
// edges seen from the neighbour, from the neighbours' net inflows.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_sst_faces(Geo<T> g, SstAdj sa, const T *__restrict__ M,
                                                       const T *__restrict__ K, const T *__restrict__ W,
                                                       const T *__restrict__ aux, const T *__restrict__ lnet,
                                                       T *__restrict__ lx, StepPar<T> p) {
    const int j = cell_index();
    if (j >= g.n) return;
    const int n = g.n;
    T xj[11], acc[11];
    sst_cell_x(n, j, p.rho0, M, K, W, aux, xj);
#pragma unroll
    for (int i = 0; i < 11; ++i) acc[i] = T(0);
    const T lk = lnet[j], lw = lnet[(size_t)n + j];
    T th = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + j;
        const int nb = g.nbr[si];
        if (nb == -1) continue;
        const T nlx = g.nlx[si], nly = g.nly[si], rx = g.rfx[si], ry = g.rfy[si], qx = g.qx[si], qy = g.qy[si];
        if (nb >= 0) {
            T xn[11], unused[11];
            sst_cell_x(n, nb, p.rho0, M, K, W, aux, xn);
#pragma unroll
            for (int i = 0; i < 11; ++i) unused[i] = T(0);
            sst_face_rev<T>(xj, xn, nlx, nly, rx, ry, qx, qy, lk, lw, acc, unused);               // j's net inflow
            sst_face_rev<T>(xn, xj, -nlx, -nly, qx, qy, rx, ry, lnet[nb], lnet[(size_t)n + nb], unused, acc);  // N's
        } else {
            const int b = -2 - nb;
            const int kind = g.b_kind[b];
            th += sst_bface_rev<T>(xj, sa.bzg[b] != 0, kind == kInlet || kind == kFarfield, T(g.b_ux[b]), T(g.b_uy[b]),
                                   T(g.b_k[b]), T(g.b_w[b]), nlx, nly, rx, ry, T(g.b_l[b] / g.b_dperp[b]), lk, lw, acc);
        }
    }
#pragma unroll
    for (int i = 0; i < 11; ++i) lx[(size_t)i * n + j] += acc[i];
    sa.pbar[j] += (double)th;
}

// SA1: reverse of the cell-local closure.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_sst_local(Geo<T> g, SstAdj sa, const T *__restrict__ M,
                                                       const T *__restrict__ K, const T *__restrict__ W,
                                                       const T *__restrict__ lown, T *__restrict__ lx,
                                                       T *__restrict__ lgrad, StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T gu[2], gv[2], gk[2], gw[2];
    sst_gradients(g, sa.bzg, M, K, W, c, gu, gv, gk, gw);
    T l[11];
#pragma unroll
    for (int i = 0; i < 11; ++i) l[i] = T(0);
    SstParBar<T> pb;
    sst_local_rev<T>(p.rho0 + M[c], K[c], W[c], gu[0], gu[1], gv[0], gv[1], gk[0], gk[1], gw[0], gw[1], T(g.wdist[c]), p,
                     sst_params(p), lx[(size_t)9 * n + c], lx[(size_t)10 * n + c], lown[c], lown[(size_t)n + c],
                     lown[(size_t)2 * n + c], lown[(size_t)3 * n + c], l, pb);
    lx[c] += l[0];
    lx[(size_t)3 * n + c] += l[1];
    lx[(size_t)4 * n + c] += l[2];
    // gradients of u, v (closure only), of k, omega (closure + the face reconstructions)
    lgrad[c] = l[3];
    lgrad[(size_t)1 * n + c] = l[4];
    lgrad[(size_t)2 * n + c] = l[5];
    lgrad[(size_t)3 * n + c] = l[6];
    lgrad[(size_t)4 * n + c] = l[7] + lx[(size_t)5 * n + c];
    lgrad[(size_t)5 * n + c] = l[8] + lx[(size_t)6 * n + c];
    lgrad[(size_t)6 * n + c] = l[9] + lx[(size_t)7 * n + c];
    lgrad[(size_t)7 * n + c] = l[10] + lx[(size_t)8 * n + c];
    sa.pbar[(size_t)4 * n + c] += (double)pb.a1;
    sa.pbar[(size_t)3 * n + c] += (double)pb.bstar;
    sa.pbar[(size_t)1 * n + c] += (double)pb.sk1;
    sa.pbar[(size_t)2 * n + c] += (double)pb.sw1;
}

// SA2: transposed LSQ gradients of u, v, k, omega, then the macro transpose onto f^n:
// u = j_x / rho gives d u / d f_a = (e_x,a - u) / rho; rho - rho0 = sum f.  Writes the adjoints of
// k^n, omega^n and adds to lfn.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_sst_grad(Geo<T> g, SstAdj sa, const int8_t *__restrict__ rev,
                                                      const T *__restrict__ M, const T *__restrict__ lgrad,
                                                      const T *__restrict__ lx, T *__restrict__ lfn,
                                                      T *__restrict__ lk, T *__restrict__ lw, T rho0) {
    const int s0 = cell_index();
    if (s0 >= g.n) return;
    const int n = g.n;
    T acc[4] = {0, 0, 0, 0};      // u, v, k, omega
    T own[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) own[i] = lgrad[(size_t)i * n + s0];
    T th = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t si = (size_t)k * n + s0;
        const int j = g.nbr[si];
        if (j == -1) continue;
        const T cx = g.cx[si], cy = g.cy[si];
        if (j >= 0) {
            const size_t sj = (size_t)rev[si] * n + j;
            const T cjx = g.cx[sj], cjy = g.cy[sj];
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[v] += cjx * lgrad[(size_t)(2 * v) * n + j] + cjy * lgrad[(size_t)(2 * v + 1) * n + j];
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] -= cx * own[2 * v] + cy * own[2 * v + 1];
        } else {
            const int b = -2 - j;
            if (sa.bzg[b]) continue;      // zero-gradient ghost: no contribution
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] -= cx * own[2 * v] + cy * own[2 * v + 1];
            const int kind = g.b_kind[b];
            if (kind == kInlet || kind == kFarfield) {
                const T lu = cx * own[0] + cy * own[1], lv = cx * own[2] + cy * own[3];
                th += lu * (-T(g.b_uy[b])) + lv * T(g.b_ux[b]);
            }
        }
    }
    sa.pbar[s0] += (double)th;
    const T lrho = lx[s0], lu = lx[(size_t)n + s0] + acc[0], lv = lx[(size_t)2 * n + s0] + acc[1];
    lk[s0] = lx[(size_t)3 * n + s0] + acc[2];
    lw[s0] = lx[(size_t)4 * n + s0] + acc[3];
    const T rho = rho0 + M[s0], ux = M[(size_t)n + s0], uy = M[(size_t)2 * n + s0];
    const T ir = recip(rho);
#pragma unroll
    for (int a = 0; a < 9; ++a)
        lfn[(size_t)a * n + s0] += lrho + (T(ex(a)) - ux) * ir * lu + (T(ey(a)) - uy) * ir * lv;
}

// ---- reverse of the implicit SST variant (params.sst_sweeps = m > 0, reading r34) ----
// The forward (sst_row_edge, sst_row_bedge, sst_row_finish, k_sst_jacobi), per cell and phi in
// {k, omega} with explicit source s (sk or sw) and sink dst (dt beta* omega or dt beta omega):
//   R' = (fac net + s - dst phi) q,  C_s = c_s fac q,  q = 1 / (sigma + fac d),  fac = dt / (A rho),
//   sigma = 1 + dst + max(-s, 0) / phi,  d = sum_s (out_s + D_s) + the boundary parts,
//   c_s = in_s + D_s,  out_s = max(mdot_s, 0),  in_s = max(-mdot_s, 0),  D_s = (Gamma_c + Gamma_N) hn_s / 2,
//   delta^1 = R',  delta^{i+1} = R' + sum_s C_s delta^i_N,  phi^{n+1} = max(phi + delta^m, floor),
// then nu_t from k^{n+1}, omega^{n+1} and the strain rate S.  Its reverse replaces that of the
// point-implicit update (k_adj_sst_update): it writes the adjoints of net, of s, beta, S (lown) and
// adds those of the cell values (lx: rho, u, v, k, omega, Gamma_k, Gamma_omega) before the face,
// closure and gradient reverses run as for the point-implicit update.

// The floor and nu_t: from the adjoints of k^{n+1}, omega^{n+1}, tau to that of delta^m (ld) and of
// k^n, omega^n (lx); the strain rate's (aux plane 9) goes to lown[3].  dm: delta^m [2][n].
template <typename T>
__global__ void __launch_bounds__(256) k_adj_impl_fin(Geo<T> g, SstAdj sa, const T *__restrict__ aux,
                                                      const T *__restrict__ dm, const T *__restrict__ K,
                                                      const T *__restrict__ W, const T *__restrict__ lk1,
                                                      const T *__restrict__ lw1, const T *__restrict__ ltau,
                                                      T *__restrict__ ld, T *__restrict__ lx, T *__restrict__ lown,
                                                      StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const size_t n = (size_t)g.n;
    const T kr = K[c] + dm[c], wr = W[c] + dm[n + c];
    const bool kpass = kr >= T(1e-20), wpass = wr >= T(1e-20);
    const T k1 = kpass ? kr : T(1e-20), w1 = wpass ? wr : T(1e-20);
    T kb = lk1[c], wb = lw1[c], Srb = 0;
    SstParBar<T> pb;
    sst_nut_rev(k1, w1, aux[9 * n + c], T(g.wdist[c]), p, sst_params(p), T(3) * ltau[c], kb, wb, Srb, pb);
    kb = kpass ? kb : T(0);
    wb = wpass ? wb : T(0);
    ld[c] = kb;
    ld[n + c] = wb;
    lx[3 * n + c] += kb;
    lx[4 * n + c] += wb;
    lown[3 * n + c] = Srb;
    sa.pbar[4 * n + c] += (double)pb.a1;
}

// One transposed Jacobi sweep: lin = the adjoint of delta^i.  Adds lin to lR (the adjoint of R'),
// lin_c delta^{i-1}_N to lC (the adjoints of the couplings C_s, [8][n] as in J), and gathers the
// adjoint of delta^{i-1} through the couplings that point back: lout_j = sum_s C_(N, rev) lin_N.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_impl_sweep(Geo<T> g, const int8_t *__restrict__ rev,
                                                        const T *__restrict__ J, const T *__restrict__ lin,
                                                        const T *__restrict__ dprev, T *__restrict__ lR,
                                                        T *__restrict__ lC, T *__restrict__ lout) {
    const int c = cell_index();
    if (c >= g.n) return;
    const size_t n = (size_t)g.n;
    const T lk = lin[c], lw = lin[n + c];
    lR[c] += lk;
    lR[n + c] += lw;
    T ok = T(0), ow = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        if (nb < 0) continue;
        lC[si] += lk * dprev[nb];
        lC[4 * n + si] += lw * dprev[n + nb];
        const size_t sj = (size_t)rev[si] * n + nb;
        ok += J[sj] * lin[nb];
        ow += J[4 * n + sj] * lin[n + nb];
    }
    if (lout) {
        lout[c] = ok;
        lout[n + c] = ow;
    }
}

// The row of cell c, formed again from the solve's recorded inputs (as sst_row_edge, sst_row_bedge
// and sst_row_finish form it): M, K, W the macro variables and k, omega the solve started from;
// aux its closure outputs (Gamma in planes 4, 5, s in 6, 7, beta in 8) and net inflows (10, 11).
// Slots without an interior neighbour keep mdot = hn = c = 0.
template <typename T>
struct ImplRow {
    T rho, ux, uy, kc, wc, Gk, Gw, sk, sw, beta, net_k, net_w;
    T dk, dw, fac, dstk, dstw, mk, mw, ik_k, ik_w, qk, qw, Nk, Nw;
    T mdot[4], hn[4], ck[4], cw[4];
};

template <typename T>
__device__ __forceinline__ void impl_row(const Geo<T> &g, const SstAdj &sa, const T *__restrict__ M,
                                         const T *__restrict__ K, const T *__restrict__ W, const T *__restrict__ aux,
                                         int c, const StepPar<T> &p, ImplRow<T> &r) {
    const size_t n = (size_t)g.n;
    const T zero = T(0), one = T(1), dt = p.dt;
    r.rho = p.rho0 + M[c];
    r.ux = M[n + c];
    r.uy = M[2 * n + c];
    r.kc = K[c];
    r.wc = W[c];
    r.Gk = aux[4 * n + c];
    r.Gw = aux[5 * n + c];
    r.sk = aux[6 * n + c];
    r.sw = aux[7 * n + c];
    r.beta = aux[8 * n + c];
    r.net_k = aux[10 * n + c];
    r.net_w = aux[11 * n + c];
    r.dk = r.dw = zero;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        r.mdot[s] = r.hn[s] = r.ck[s] = r.cw[s] = zero;
        if (nb >= 0) {
            const T rn = p.rho0 + M[nb], un = M[n + nb], vn = M[2 * n + nb];
            const T nlx = g.nlx[si], nly = g.nly[si];
            r.mdot[s] = T(0.5) * ((r.rho * r.ux + rn * un) * nlx + (r.rho * r.uy + rn * vn) * nly);
            const T ddx = g.rfx[si] - g.qx[si], ddy = g.rfy[si] - g.qy[si];
            r.hn[s] = (ddx * nlx + ddy * nly) * recip(ddx * ddx + ddy * ddy);
            const T Dk = T(0.5) * (r.Gk + aux[4 * n + nb]) * r.hn[s], Dw = T(0.5) * (r.Gw + aux[5 * n + nb]) * r.hn[s];
            const T out = tmax(r.mdot[s], zero), in = tmax(-r.mdot[s], zero);
            r.dk = r.dk + out + Dk;
            r.dw = r.dw + out + Dw;
            r.ck[s] = in + Dk;
            r.cw[s] = in + Dw;
        } else if (nb <= -2) {
            const int b = -2 - nb;
            const bool zg = sa.bzg[b] != 0;
            const T bux = zg ? r.ux : T(g.b_ux[b]), buy = zg ? r.uy : T(g.b_uy[b]);
            const T mb = r.rho * (bux * g.nlx[si] + buy * g.nly[si]);
            const T own = (zg || mb >= zero) ? mb : zero;
            r.dk = r.dk + own;
            r.dw = r.dw + own;
            if (!zg) {
                const T lod = T(g.b_l[b] / g.b_dperp[b]);
                r.dk = r.dk + r.Gk * lod;
                r.dw = r.dw + r.Gw * lod;
            }
        }
    }
    // a periodic cell that is its own neighbour across an edge: that coupling is on the diagonal
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (g.nbr[(size_t)s * n + c] == c) {
            r.dk = r.dk - r.ck[s];
            r.dw = r.dw - r.cw[s];
            r.ck[s] = r.cw[s] = zero;
        }
    r.fac = T(dt * g.inv_area[c]) * recip(r.rho);
    r.dstk = dt * p.bstar * r.wc;
    r.dstw = dt * r.beta * r.wc;
    r.mk = tmax(-r.sk, zero);
    r.mw = tmax(-r.sw, zero);
    r.ik_k = recip(r.kc);
    r.ik_w = recip(r.wc);
    r.qk = recip(one + r.dstk + r.mk * r.ik_k + r.fac * r.dk);
    r.qw = recip(one + r.dstw + r.mw * r.ik_w + r.fac * r.dw);
    r.Nk = r.fac * r.net_k + r.sk - r.dstk * r.kc;
    r.Nw = r.fac * r.net_w + r.sw - r.dstw * r.wc;
}

// The system again (planes 0-9 of the forward's J: the couplings of k and omega per slot, R' of
// both), for the recomputed sweeps and their transposes.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_impl_sys(Geo<T> g, SstAdj sa, const T *__restrict__ M,
                                                      const T *__restrict__ K, const T *__restrict__ W,
                                                      const T *__restrict__ aux, T *__restrict__ J, StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const size_t n = (size_t)g.n;
    ImplRow<T> r;
    impl_row(g, sa, M, K, W, aux, c, p, r);
    const T gk = r.fac * r.qk, gw = r.fac * r.qw;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        J[(size_t)s * n + c] = r.ck[s] * gk;
        J[(size_t)(4 + s) * n + c] = r.cw[s] * gw;
    }
    J[8 * n + c] = r.Nk * r.qk;
    J[9 * n + c] = r.Nw * r.qw;
}

// The rows' reverse, cell c: from the adjoints of R' (lR) and of the couplings (lC) to those of net
// (lnet), s and beta (lown[0..2]), of the cell's rho, u, v, k, omega, Gamma_k, Gamma_omega (lx) and
// of beta* and theta (pbar); the parts that belong to the neighbours' rho, u, v (through mdot) and
// Gamma (through D) go per edge slot to lslot [4][4][n]: (dJ/dmdot) nl / 2 (x, y), and
// (dJ/dD) hn / 2 for k and omega.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_impl_rows(Geo<T> g, SstAdj sa, const T *__restrict__ M,
                                                       const T *__restrict__ K, const T *__restrict__ W,
                                                       const T *__restrict__ aux, const T *__restrict__ lR,
                                                       const T *__restrict__ lC, T *__restrict__ lx,
                                                       T *__restrict__ lnet, T *__restrict__ lown,
                                                       T *__restrict__ lslot, StepPar<T> p) {
    const int c = cell_index();
    if (c >= g.n) return;
    const size_t n = (size_t)g.n;
    const T zero = T(0), dt = p.dt;
    ImplRow<T> r;
    impl_row(g, sa, M, K, W, aux, c, p, r);
    const T gk = r.fac * r.qk, gw = r.fac * r.qw;
    // R' = N q and C_s = c_s fac q
    const T lRk = lR[c], lRw = lR[n + c];
    T lgk = zero, lgw = zero, lck[4], lcw[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const T a = lC[(size_t)s * n + c], b = lC[(size_t)(4 + s) * n + c];
        lgk += a * r.ck[s];
        lgw += b * r.cw[s];
        lck[s] = a * gk;
        lcw[s] = b * gw;
    }
    const T lNk = lRk * r.qk, lNw = lRw * r.qw;
    const T lqk = lRk * r.Nk + lgk * r.fac, lqw = lRw * r.Nw + lgw * r.fac;
    T lfac = lgk * r.qk + lgw * r.qw;
    // q = 1 / (sigma + fac d): the adjoint of the denominator is that of sigma
    const T lsk_ = -lqk * r.qk * r.qk, lsw_ = -lqw * r.qw * r.qw;
    lfac += lsk_ * r.dk + lsw_ * r.dw;
    const T ldk = lsk_ * r.fac, ldw = lsw_ * r.fac;
    // a self-neighbour slot's in + D enters the diagonal with a minus sign; its coupling is zero
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (g.nbr[(size_t)s * n + c] == c) {
            lck[s] = -ldk;
            lcw[s] = -ldw;
        }
    // N = fac net + s - dst phi
    lfac += lNk * r.net_k + lNw * r.net_w;
    T lsk = lNk, lsw = lNw;
    const T ldstk = -lNk * r.kc + lsk_, ldstw = -lNw * r.wc + lsw_;
    T lk = -lNk * r.dstk, lw = -lNw * r.dstw;
    // sigma = 1 + dst + max(-s, 0) / phi
    if (-r.sk >= zero) lsk -= lsk_ * r.ik_k;
    lk -= lsk_ * r.mk * r.ik_k * r.ik_k;
    if (-r.sw >= zero) lsw -= lsw_ * r.ik_w;
    lw -= lsw_ * r.mw * r.ik_w * r.ik_w;
    // dst = dt beta* omega (k), dt beta omega (omega)
    lw += ldstk * dt * p.bstar + ldstw * dt * r.beta;
    const T lbeta = ldstw * dt * r.wc;
    const double lbstar = (double)(ldstk * dt * r.wc);
    // fac = dt / (A rho)
    T lrho = -lfac * r.fac * recip(r.rho), lu = zero, lv = zero, lGk = zero, lGw = zero;
    double lth = 0.0;
    // d = sum (out + D) + the boundary parts, c = in + D
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + c;
        const int nb = g.nbr[si];
        T sA = zero, sB = zero, sK = zero, sW = zero;
        if (nb >= 0) {
            const T lDk = ldk + lck[s], lDw = ldw + lcw[s];
            T lm = zero;
            if (r.mdot[s] >= zero) lm += ldk + ldw;          // out = max(mdot, 0)
            if (-r.mdot[s] >= zero) lm -= lck[s] + lcw[s];   // in = max(-mdot, 0)
            const T nlx = g.nlx[si], nly = g.nly[si];
            // mdot = (rho u + rho_N u_N) . nl / 2
            lrho += T(0.5) * lm * (r.ux * nlx + r.uy * nly);
            lu += T(0.5) * lm * r.rho * nlx;
            lv += T(0.5) * lm * r.rho * nly;
            sA = T(0.5) * lm * nlx;
            sB = T(0.5) * lm * nly;
            // D = (Gamma_c + Gamma_N) hn / 2
            sK = T(0.5) * r.hn[s] * lDk;
            sW = T(0.5) * r.hn[s] * lDw;
            lGk += sK;
            lGw += sW;
        } else if (nb <= -2) {
            const int b = -2 - nb;
            const bool zg = sa.bzg[b] != 0;
            const T bux = zg ? r.ux : T(g.b_ux[b]), buy = zg ? r.uy : T(g.b_uy[b]);
            const T nlx = g.nlx[si], nly = g.nly[si];
            const T mb = r.rho * (bux * nlx + buy * nly);
            if (zg || mb >= zero) {
                const T lm = ldk + ldw;
                lrho += lm * (bux * nlx + buy * nly);
                if (zg) {
                    lu += lm * r.rho * nlx;
                    lv += lm * r.rho * nly;
                } else {
                    const int kind = g.b_kind[b];
                    if (kind == kInlet || kind == kFarfield)   // the rotated inflow: d ub / d theta = (-ub_y, ub_x)
                        lth += (double)(lm * r.rho * (-T(g.b_uy[b]) * nlx + T(g.b_ux[b]) * nly));
                }
            }
            if (!zg) {
                const T lod = T(g.b_l[b] / g.b_dperp[b]);
                lGk += ldk * lod;
                lGw += ldw * lod;
            }
        }
        lslot[si] = sA;
        lslot[4 * n + si] = sB;
        lslot[8 * n + si] = sK;
        lslot[12 * n + si] = sW;
    }
    lnet[c] = lNk * r.fac;
    lnet[n + c] = lNw * r.fac;
    lown[c] = lsk;
    lown[n + c] = lsw;
    lown[2 * n + c] = lbeta;
    lx[c] += lrho;
    lx[n + c] += lu;
    lx[2 * n + c] += lv;
    lx[3 * n + c] += lk;
    lx[4 * n + c] += lw;
    lx[9 * n + c] += lGk;
    lx[10 * n + c] += lGw;
    sa.pbar[3 * n + c] += lbstar;
    sa.pbar[c] += lth;
}

// The neighbours' parts of the rows' reverse, gathered per cell j: each interior edge's slot seen
// from the neighbour N (through rev) gives the adjoint of j's rho, u, v through N's mdot and of j's
// Gamma through N's D.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_impl_gather(Geo<T> g, const int8_t *__restrict__ rev,
                                                         const T *__restrict__ M, const T *__restrict__ lslot,
                                                         T *__restrict__ lx, T rho0) {
    const int j = cell_index();
    if (j >= g.n) return;
    const size_t n = (size_t)g.n;
    const T rho = rho0 + M[j], ux = M[n + j], uy = M[2 * n + j];
    T lrho = 0, lu = 0, lv = 0, lGk = 0, lGw = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t si = (size_t)s * n + j;
        const int nb = g.nbr[si];
        if (nb < 0) continue;
        const size_t sn = (size_t)rev[si] * n + nb;
        const T A = lslot[sn], B = lslot[4 * n + sn];
        lrho += A * ux + B * uy;
        lu += A * rho;
        lv += B * rho;
        lGk += lslot[8 * n + sn];
        lGw += lslot[12 * n + sn];
    }
    lx[j] += lrho;
    lx[n + j] += lu;
    lx[2 * n + j] += lv;
    lx[9 * n + j] += lGk;
    lx[10 * n + j] += lGw;
}

// ---- ring-tiled SST reverse: update, faces, closure and LSQ gradients in one launch ----
// The layout of the ring-tiled forward kernels.  x = the 11 cell values of the face fluxes
// (rho, u, v, k, omega, grad k, grad omega, Gamma_k, Gamma_omega).
//   phase 0: tile cell t and ext cell t: x and the reverse of the cell-local update (the adjoints
//            of the net inflows into LDS, those of rho, k, omega and of the closure outputs kept);
//   phase 1: tile cell t and ring-1 cell t: reverse of its face fluxes (both edge perspectives,
//            neighbours from LDS) and of its closure (gradients recomputed from LDS): the adjoints
//            of its LSQ gradients into LDS;
//   phase 2: tile cell t: transposed LSQ gradients from its neighbours' gradient adjoints in LDS,
//            the macro transpose onto f^n; the adjoints of k^n, omega^n go to lk_out, lw_out
//            (the adjoints of k, omega of the step's output are read from lk1, lw1).
// LDS, cell-major: X [Wv][12] (the 11 cell values at row positions xpos), Ln [Wv][2] (net-inflow
// adjoints), Lg [Wg][8] (gradient adjoints), Mi [Wg][3] (triangle meshes: inverse LSQ matrices,
// from which the neighbours' LSQ coefficients pointing back are formed; other meshes gather them).
template <typename T, int S>
__global__ void __launch_bounds__(kTileCells, sizeof(T) == 4 ? 3 : 2)
    k_adj_sst_ring(Geo<T> g, RingTiles rt, const int16_t *__restrict__ lnb, const int8_t *__restrict__ rev, int Wv,
                   int Wg, SstAdj sa, const T *__restrict__ M, const T *__restrict__ K, const T *__restrict__ W,
                   const T *__restrict__ aux, const T *__restrict__ lk1, const T *__restrict__ lw1,
                   const T *__restrict__ ltau, T *__restrict__ lfn, T *__restrict__ lk_out, T *__restrict__ lw_out,
                   StepPar<T> p) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *X = reinterpret_cast<T *>(smem);
    T *Ln = X + 12 * Wv;
    T *Lg = Ln + 2 * Wv;
    T *Mi = Lg + 8 * Wg;   // [Wg][3] inverse LSQ matrices (S = 3)
    // FP64 triangles form the coefficient of a neighbour's edge pointing back, c_(j->t) = w M_j^-1 (-d),
    // from M_j^-1 in LDS; FP32 gathers it from the stored coefficients, the ones its forward uses
    constexpr bool FORM = S == 3 && sizeof(T) == 8;
    const int tile = ring_tile<false>();   // descending, after the ascending stage-1 transpose
    const int start = tile * kTileCells;
    const int ncell = min(kTileCells, g.n - start);
    const int x0 = rt.ptr[tile], nx = rt.ptr[tile + 1] - x0, n1 = rt.n1[tile];
    const int t = threadIdx.x;
    const int n = g.n;
    const bool own = t < ncell, ext = t < nx, ring1 = t < n1;
    const int c = start + t;
    const SstParams<T> q = sst_params(p);

    // phase 0: cell values and the update's reverse of cell `cell`, stored at LDS row `col`
    auto load_update = [&](int cell, int col, T x[11], T lxu[3], T lown[4], SstParBar<T> &pb) {
        x[0] = p.rho0 + M[cell];
        x[1] = M[(size_t)n + cell];
        x[2] = M[(size_t)2 * n + cell];
        x[3] = K[cell];
        x[4] = W[cell];
#pragma unroll
        for (int i = 0; i < 6; ++i) x[5 + i] = aux[(size_t)i * n + cell];
#pragma unroll
        for (int i = 0; i < 11; ++i) X[col * 12 + xpos(i)] = x[i];
        T ob[6];
        lxu[0] = lxu[1] = lxu[2] = T(0);
        sst_update_rev<T>(x[0], x[3], x[4], aux[(size_t)10 * n + cell], aux[(size_t)11 * n + cell],
                          aux[(size_t)6 * n + cell], aux[(size_t)7 * n + cell], aux[(size_t)8 * n + cell],
                          aux[(size_t)9 * n + cell], T(g.wdist[cell]), g.inv_area[cell], p, q, lk1[cell], lw1[cell],
                          T(3) * ltau[cell], lxu, ob, pb);
        Ln[col * 2] = ob[0];
        Ln[col * 2 + 1] = ob[1];
#pragma unroll
        for (int i = 0; i < 4; ++i) lown[i] = ob[2 + i];
    };
    T xc[11], lxc[3], lownc[4];
    SstParBar<T> pbc;
    int nb[S], col[S];
    T nlx[S], nly[S], rx[S], ry[S], qx[S], qy[S], cxs[S], cys[S], cbx[S], cby[S];
    if (own) {
        load_update(c, t, xc, lxc, lownc, pbc);
        T mi[3], ia;
        cell_edges<T, S>(g, lnb, n, c, c, col, nb, nlx, nly, rx, ry, qx, qy, cxs, cys, mi, ia);
        if constexpr (FORM) {
#pragma unroll
            for (int k = 0; k < 3; ++k) Mi[t * 3 + k] = mi[k];
        } else {
            // the LSQ coefficient of the neighbour's slot that points back, gathered
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const size_t si = (size_t)s * n + c;
                cbx[s] = cby[s] = T(0);
                if (nb[s] >= 0) {
                    const size_t sj = (size_t)rev[si] * n + g.nbr[si];
                    cbx[s] = g.cx[sj];
                    cby[s] = g.cy[sj];
                }
            }
        }
    }
    T xh[11], lxh[3], lownh[4];
    SstParBar<T> pbh;    // ring-1 cells: their constants' adjoints are their own tile's
    int hc = 0;
    int hnb[S], hcol[S];
    T hnx[S], hny[S], hrx[S], hry[S], hqx[S], hqy[S], hcx[S], hcy[S];
    if (ext) {
        hc = rt.cell[x0 + t];
        load_update(hc, kTileCells + t, xh, lxh, lownh, pbh);
        if (ring1) {
            T hmi[3], hia;
            cell_edges<T, S>(g, rt.lnb, rt.n_ext, x0 + t, hc, hcol, hnb, hnx, hny, hrx, hry, hqx, hqy, hcx, hcy, hmi,
                             hia);
            if constexpr (FORM) {
#pragma unroll
                for (int k = 0; k < 3; ++k) Mi[(kTileCells + t) * 3 + k] = hmi[k];
            }
        }
    }
    // ring-2 cells beyond one per thread (tiles of stretched cells): their LDS rows only (the
    // other outputs of a ring-2 cell are not used)
    for (int e = t + kTileCells; e < nx; e += kTileCells) {
        T ex[11], elx[3], eown[4];
        SstParBar<T> epb;
        load_update(rt.cell[x0 + e], kTileCells + e, ex, elx, eown, epb);
    }
    __syncthreads();

    // phase 1: faces and closure of a cell with edge data e*, LDS column cl; returns the 11 x
    // adjoints (lx) and the theta part, adds the constants' adjoints to pb
    auto faces_closure = [&](int cell, int cl, const T x[11], const T lxu[3], const T lown[4], const int *enb,
                             const int *ecol, const T *enx, const T *eny, const T *erx, const T *ery, const T *eqx,
                             const T *eqy, const T *ecx, const T *ecy, T lg[8], T lx[11], SstParBar<T> &pb) {
        T th = 0;
#pragma unroll
        for (int i = 0; i < 11; ++i) lx[i] = T(0);
        const T lk = Ln[cl * 2], lw = Ln[cl * 2 + 1];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (enb[s] == -1) continue;
            if (enb[s] >= 0) {
                T xn[11], unused[11];
#pragma unroll
                for (int i = 0; i < 11; ++i) {
                    xn[i] = X[ecol[s] * 12 + xpos(i)];
                    unused[i] = T(0);
                }
                sst_face_rev<T>(x, xn, enx[s], eny[s], erx[s], ery[s], eqx[s], eqy[s], lk, lw, lx, unused);
                sst_face_rev<T>(xn, x, -enx[s], -eny[s], eqx[s], eqy[s], erx[s], ery[s], Ln[ecol[s] * 2],
                                Ln[ecol[s] * 2 + 1], unused, lx);
            } else {
                const int b = -2 - enb[s];
                const int kind = g.b_kind[b];
                th += sst_bface_rev<T>(x, sa.bzg[b] != 0, kind == kInlet || kind == kFarfield, T(g.b_ux[b]),
                                       T(g.b_uy[b]), T(g.b_k[b]), T(g.b_w[b]), enx[s], eny[s], erx[s], ery[s],
                                       T(g.b_l[b] / g.b_dperp[b]), lk, lw, lx);
            }
        }
        lx[0] += lxu[0];
        lx[3] += lxu[1];
        lx[4] += lxu[2];
        T gu[2], gv[2], gk[2], gw[2];
        sst_grad_ring<T, S, 12>(g, sa.bzg, enb, ecol, ecx, ecy, X, x[1], x[2], x[3], x[4], gu, gv, gk, gw);
        T l[11];
#pragma unroll
        for (int i = 0; i < 11; ++i) l[i] = T(0);
        sst_local_rev<T>(x[0], x[3], x[4], gu[0], gu[1], gv[0], gv[1], gk[0], gk[1], gw[0], gw[1], T(g.wdist[cell]), p, q,
                         lx[9], lx[10], lown[0], lown[1], lown[2], lown[3], l, pb);
        lx[0] += l[0];
        lx[3] += l[1];
        lx[4] += l[2];
        lg[0] = l[3];
        lg[1] = l[4];
        lg[2] = l[5];
        lg[3] = l[6];
        lg[4] = l[7] + lx[5];
        lg[5] = l[8] + lx[6];
        lg[6] = l[9] + lx[7];
        lg[7] = l[10] + lx[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) Lg[cl * 8 + i] = lg[i];
        return th;
    };
    if (ring1) {
        T lg[8], lx[11];
        faces_closure(hc, kTileCells + t, xh, lxh, lownh, hnb, hcol, hnx, hny, hrx, hry, hqx, hqy, hcx, hcy, lg, lx, pbh);
    }
    T lgc[8], lx[11], th = 0;
    if (own)
        th = faces_closure(c, t, xc, lxc, lownc, nb, col, nlx, nly, rx, ry, qx, qy, cxs, cys, lgc, lx, pbc);
    __syncthreads();
    if (!own) return;

    // phase 2: transposed LSQ gradients (interior edges straight-line, boundary edges after) and
    // the macro transpose
    T acc[4] = {0, 0, 0, 0};
    bool bnd = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool in = nb[s] >= 0;
        bnd = bnd || nb[s] <= -2;
        const int r = in ? col[s] : 0;
        T bx, by;
        if constexpr (FORM) {
            // neighbour r's LSQ coefficient of its edge back to this cell: w M_r^-1 (-d)
            const T dx = rx[s] - qx[s], dy = ry[s] - qy[s];
            const T w = in ? recip(dx * dx + dy * dy) : T(0);
            bx = -w * (Mi[r * 3] * dx + Mi[r * 3 + 1] * dy);
            by = -w * (Mi[r * 3 + 1] * dx + Mi[r * 3 + 2] * dy);
        } else {
            bx = in ? cbx[s] : T(0);
            by = in ? cby[s] : T(0);
        }
        const T wx = in ? cxs[s] : T(0), wy = in ? cys[s] : T(0);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += bx * Lg[r * 8 + 2 * v] + by * Lg[r * 8 + 2 * v + 1];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] -= wx * lgc[2 * v] + wy * lgc[2 * v + 1];
    }
    if (bnd) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (nb[s] > -2) continue;
            const int b = -2 - nb[s];
            if (sa.bzg[b]) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] -= cxs[s] * lgc[2 * v] + cys[s] * lgc[2 * v + 1];
            const int kind = g.b_kind[b];
            if (kind == kInlet || kind == kFarfield) {
                const T lu = cxs[s] * lgc[0] + cys[s] * lgc[1], lv = cxs[s] * lgc[2] + cys[s] * lgc[3];
                th += lu * (-T(g.b_uy[b])) + lv * T(g.b_ux[b]);
            }
        }
    }
    sa.pbar[c] += (double)th;
    sa.pbar[(size_t)1 * n + c] += (double)pbc.sk1;
    sa.pbar[(size_t)2 * n + c] += (double)pbc.sw1;
    sa.pbar[(size_t)3 * n + c] += (double)pbc.bstar;
    sa.pbar[(size_t)4 * n + c] += (double)pbc.a1;
    const T lrho = lx[0], lu = lx[1] + acc[0], lv = lx[2] + acc[1];
    lk_out[c] = lx[3] + acc[2];
    lw_out[c] = lx[4] + acc[3];
    const T ir = recip(xc[0]), ux = xc[1], uy = xc[2];
#pragma unroll
    for (int a = 0; a < 9; ++a)
        lfn[(size_t)a * n + c] += lrho + (T(ex(a)) - ux) * ir * lu + (T(ey(a)) - uy) * ir * lv;
}

// Forces and the reversed-flow length at the final state, reversed onto f (through rho, u of the
// wall cells): seed = (dJ/dF_x, dJ/dF_y, dJ/dJ_R).
template <typename T>
__global__ void __launch_bounds__(256) k_adj_forces(Geo<T> g, const T *__restrict__ F, unsigned long long mask,
                                                    int jr_group, double jr_xmin, double eps, double nu, double sx,
                                                    double sy, double sj, T rho0, T *__restrict__ lfn) {
    const int c = cell_index();
    if (c >= g.n) return;
    const int n = g.n;
    T d[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = F[(size_t)a * n + c];
    using D = Dual<double, 3>;
    D acc[3];
    bool any = false;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int nb = g.nbr[(size_t)s * n + c];
        if (nb >= -1) continue;
        const int b = -2 - nb;
        const int kind = g.b_kind[b];
        if (kind != kWall && kind != kMovingWall) continue;
        const int grp = g.b_group[b];
        const bool inF = (mask >> grp) & 1ull, inJ = (grp == jr_group && g.b_xfx[b] > jr_xmin);
        if (!inF && !inJ) continue;
        if (!any) {
            T m0, mx, my;
            raw_moments(d, m0, mx, my);
            const D dr = D::var((double)m0, 0), jx = D::var((double)mx, 1), jy = D::var((double)my, 2);
            const D rho = D((double)rho0) + dr;
            acc[0] = rho;
            acc[1] = jx / rho;
            acc[2] = jy / rho;
            any = true;
        }
        const D rho = acc[0], ux = acc[1], uy = acc[2];
        const double nx = g.b_nx[b], ny = g.b_ny[b], l = g.b_l[b], dp = g.b_dperp[b];
        const D rux = ux - g.b_ux[b], ruy = uy - g.b_uy[b];
        const D un = rux * nx + ruy * ny;
        const D mu = rho * nu;
        const D tx = mu * (rux - un * nx) / dp, ty = mu * (ruy - un * ny) / dp;
        const D dpres = (rho - (double)rho0) / 3.0;
        D J(0.0);
        if (inF) J = J + (sx * l) * (dpres * nx + tx) + (sy * l) * (dpres * ny + ty);
        if (inJ) J = J + (sj * l * 0.5) * (1.0 - dtanh(tx / eps));
        // accumulate dJ/d(m) into lfn below
        const double j0 = J.d[0], j1 = J.d[1], j2 = J.d[2];
#pragma unroll
        for (int a = 0; a < 9; ++a) lfn[(size_t)a * n + c] += T(j0 + ex(a) * j1 + ey(a) * j2);
    }
}

}  // namespace fvlbm
