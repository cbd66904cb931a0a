// Reverse mode of the cell-local SST pieces (sst_local, sst_face, sst_bface, sst_update in
// kernels.h), written out by hand: given the adjoints of a piece's outputs, the adjoints of its
// inputs and of the constants a1, beta*, sigma_k1, sigma_omega1 (and theta on boundary edges).
// Branches follow the forward pieces exactly: max / min pass the adjoint to the argument the
// forward selected (the first on ties), sqrt has derivative 0 at 0, tanh' = 1 / cosh^2.
#pragma once

#include "kernels.h"

namespace fvlbm {

// Adjoints of the SST constants the reverse differentiates.
template <typename T>
struct SstParBar {
    T a1 = T(0), bstar = T(0), sk1 = T(0), sw1 = T(0);
};

// 1 / cosh^2 x = 4 e / (1 + e)^2 with e = exp(-2 |x|) (no overflow, no cancellation).
template <typename T>
__device__ __forceinline__ T sech2(T x) {
    const T e = sexp(T(-2) * fabs(x));
    const T s = T(1) + e;
    return T(4) * e * recip(s * s);
}

// Reverse of sst_local.  In: the cell values and gradients of the forward call; out-adjoints
// lGk, lGw, lsk, lsw, lbeta, lSr.  Adds to xb[0..10] = (rho, k, w, dux, duy, dvx, dvy, dkx, dky,
// dwx, dwy) and to pb.
template <typename T>
__device__ __forceinline__ void sst_local_rev(T rho, T k, T w, T dux, T duy, T dvx, T dvy, T dkx, T dky, T dwx, T dwy,
                                              T d, const StepPar<T> &p, const SstParams<T> &q, T lGk, T lGw, T lsk,
                                              T lsw, T lbeta, T lSr, T xb[11], SstParBar<T> &pb) {
    // ---- forward, keeping the intermediates (the expressions of sst_local) ----
    const T kap2 = p.kappa * p.kappa;
    const T sb = ssqrt(q.bstar), ib = recip(q.bstar), isb = recip(sb);
    const T cw1 = p.b1 * ib - q.sw1 * kap2 * isb;
    const T cw2 = p.b2 * ib - p.sw2 * p.kappa * p.kappa * isb;
    const T s11 = dux, s22 = dvy, s12 = T(0.5) * (duy + dvx);
    const T S2 = T(2) * (s11 * s11 + s22 * s22 + T(2) * s12 * s12);
    const T Sr = ssqrt(S2);
    const T div = dux + dvy;
    const T gkgw = dkx * dwx + dky * dwy;
    const T iw = recip(w);
    const T CDa = T(2) * rho * p.sw2 * iw * gkgw;
    const bool cd_pass = CDa >= T(1e-20);
    const T CD = cd_pass ? CDa : T(1e-20);
    const T sk = ssqrt(k);
    const T idd = recip(d), idd2 = idd * idd;
    const T visc = T(500) * p.nu * iw * idd2;
    const T t1 = sk * iw * idd * T(1.0 / 0.09);
    const bool m1_first = t1 >= visc;
    const T m1 = m1_first ? t1 : visc;
    const T iCD = recip(CD);
    const T t2 = T(4) * rho * p.sw2 * k * iCD * idd2;
    const bool a1_first = m1 <= t2;
    const T arg1 = a1_first ? m1 : t2;
    const T a2 = arg1 * arg1;
    const T F1 = stanh(a2 * a2);
    const T t3 = T(2) * t1;
    const bool arg2_first = t3 >= visc;
    const T arg2 = arg2_first ? t3 : visc;
    const T F2 = stanh(arg2 * arg2);
    const bool den_first = q.a1 * w >= Sr * F2;
    const T den = den_first ? q.a1 * w : Sr * F2;
    const T iden = recip(den);
    const T mut = q.a1 * rho * k * iden;
    const T one = T(1);
    const T sig_k = F1 * q.sk1 + (one - F1) * p.sk2;
    const T sig_w = F1 * q.sw1 + (one - F1) * p.sw2;
    const T gam = F1 * cw1 + (one - F1) * cw2;
    const T tt = T(2.0 / 3.0);
    const T E = S2 - tt * div * div;
    const T ia1 = recip(q.a1);
    const T Hh = den * ia1;
    const T P = mut * E - tt * rho * k * div;
    const T Pw = gam * rho * E - tt * gam * rho * Hh * div;
    const T cross = T(2) * (one - F1) * rho * p.sw2 * gkgw * iw;
    const T irho = recip(rho), dtr = p.dt * irho;
    const T sko = dtr * P;
    const T swo = dtr * (Pw + cross);
    // ---- reverse ----
    T rho_b = 0, k_b = 0, w_b = 0, div_b = 0, S2_b = 0, gkgw_b = 0, F1_b = 0, den_b = 0, mut_b = 0, Sr_b = lSr;
    T a1_b = 0, cw1_b = 0, cw2_b = 0, sk1_b = 0, sw1_b = 0;
    // Gk = mu + sig_k mut, Gw = mu + sig_w mut, mu = rho nu
    rho_b += (lGk + lGw) * p.nu;
    const T sigk_b = lGk * mut, sigw_b = lGw * mut;
    mut_b += lGk * sig_k + lGw * sig_w;
    // sk = dt / rho P, sw = dt / rho (Pw + cross)
    const T P_b = lsk * dtr;
    const T Pwc_b = lsw * dtr;
    rho_b -= (lsk * sko + lsw * swo) * irho;
    // beta = F1 b1 + (1 - F1) b2
    F1_b += lbeta * (p.b1 - p.b2);
    // cross = 2 (1 - F1) rho sw2 gkgw / w
    F1_b -= Pwc_b * T(2) * rho * p.sw2 * gkgw * iw;
    rho_b += Pwc_b * T(2) * (one - F1) * p.sw2 * gkgw * iw;
    gkgw_b += Pwc_b * T(2) * (one - F1) * rho * p.sw2 * iw;
    w_b -= Pwc_b * cross * iw;
    // Pw = gam rho E - tt gam rho H div
    const T gam_b = Pwc_b * (rho * E - tt * rho * Hh * div);
    rho_b += Pwc_b * (gam * E - tt * gam * Hh * div);
    T E_b = Pwc_b * gam * rho;
    const T H_b = -Pwc_b * tt * gam * rho * div;
    div_b -= Pwc_b * tt * gam * rho * Hh;
    den_b += H_b * ia1;
    a1_b -= H_b * den * ia1 * ia1;
    // P = mut E - tt rho k div
    mut_b += P_b * E;
    E_b += P_b * mut;
    rho_b -= P_b * tt * k * div;
    k_b -= P_b * tt * rho * div;
    div_b -= P_b * tt * rho * k;
    // E = S2 - tt div^2
    S2_b += E_b;
    div_b -= E_b * T(2) * tt * div;
    // blends
    F1_b += gam_b * (cw1 - cw2) + sigw_b * (q.sw1 - p.sw2) + sigk_b * (q.sk1 - p.sk2);
    cw1_b += gam_b * F1;
    cw2_b += gam_b * (one - F1);
    sw1_b += sigw_b * F1;
    sk1_b += sigk_b * F1;
    // mut = a1 rho k / den
    a1_b += mut_b * rho * k * iden;
    rho_b += mut_b * q.a1 * k * iden;
    k_b += mut_b * q.a1 * rho * iden;
    den_b -= mut_b * mut * iden;
    // den = max(a1 w, Sr F2)
    T F2_b = 0;
    if (den_first) {
        a1_b += den_b * w;
        w_b += den_b * q.a1;
    } else {
        Sr_b += den_b * F2;
        F2_b += den_b * Sr;
    }
    // F2 = tanh(arg2^2), arg2 = max(t3, visc)
    const T arg2_b = F2_b * sech2(arg2 * arg2) * T(2) * arg2;
    T visc_b = 0, sk_b = 0;
    if (arg2_first) {
        sk_b += arg2_b * T(2.0 / 0.09) * iw * idd;
        w_b -= arg2_b * t3 * iw;
    } else {
        visc_b += arg2_b;
    }
    // F1 = tanh(a2^2), a2 = arg1^2, arg1 = min(m1, t2)
    const T a2_b = F1_b * sech2(a2 * a2) * T(2) * a2;
    const T arg1_b = a2_b * T(2) * arg1;
    if (a1_first) {
        // m1 = max(t1, visc)
        if (m1_first) {
            sk_b += arg1_b * T(1.0 / 0.09) * iw * idd;
            w_b -= arg1_b * t1 * iw;
        } else {
            visc_b += arg1_b;
        }
    } else {
        // t2 = 4 rho sw2 k / (CD d^2)
        rho_b += arg1_b * T(4) * p.sw2 * k * iCD * idd2;
        k_b += arg1_b * T(4) * rho * p.sw2 * iCD * idd2;
        const T CD_b = -arg1_b * t2 * iCD;
        if (cd_pass) {
            // CDa = 2 rho sw2 / w gkgw
            rho_b += CD_b * T(2) * p.sw2 * iw * gkgw;
            w_b -= CD_b * CDa * iw;
            gkgw_b += CD_b * T(2) * rho * p.sw2 * iw;
        }
    }
    // visc = 500 nu / (w d^2)
    w_b -= visc_b * visc * iw;
    // sk = sqrt(k)
    k_b += sk > T(0) ? sk_b * T(0.5) * recip(sk) : T(0);
    // Sr = sqrt(S2), S2 = 2 (s11^2 + s22^2 + 2 s12^2)
    S2_b += Sr > T(0) ? Sr_b * T(0.5) * recip(Sr) : T(0);
    const T s12_b = S2_b * T(8) * s12;
    // gradients
    xb[0] += rho_b;
    xb[1] += k_b;
    xb[2] += w_b;
    xb[3] += div_b + S2_b * T(4) * s11;           // dux
    xb[4] += T(0.5) * s12_b;                      // duy
    xb[5] += T(0.5) * s12_b;                      // dvx
    xb[6] += div_b + S2_b * T(4) * s22;           // dvy
    xb[7] += gkgw_b * dwx;                        // dkx
    xb[8] += gkgw_b * dwy;                        // dky
    xb[9] += gkgw_b * dkx;                        // dwx
    xb[10] += gkgw_b * dky;                       // dwy
    // constants: cw1 = b1 / b* - sw1 kap^2 / sqrt(b*), cw2 = b2 / b* - sw2 kap^2 / sqrt(b*)
    const T sb_b = (cw1_b * q.sw1 + cw2_b * p.sw2) * kap2 * isb * isb;
    pb.bstar += -(cw1_b * p.b1 + cw2_b * p.b2) * ib * ib + (sb > T(0) ? sb_b * T(0.5) * isb : T(0));
    pb.sw1 += sw1_b - cw1_b * kap2 * isb;
    pb.sk1 += sk1_b;
    pb.a1 += a1_b;
}

// Bounded upwind face value bound(v0, up) = min(max(v0, 0), 2 up): the adjoints of v0 and of up
// for the result's adjoint vb.
template <typename T>
struct BoundRev {
    T v, up;
};

template <typename T>
__device__ __forceinline__ BoundRev<T> bound_face_rev(T v0, T up, T vb) {
    const T lo = v0 >= T(0) ? v0 : T(0);
    if (lo <= T(2) * up) return BoundRev<T>{v0 >= T(0) ? vb : T(0), T(0)};
    return BoundRev<T>{T(0), T(2) * vb};
}

// Adds the adjoint of the reconstruction phi + g_x x + g_y y, bounded with up = phi, to the
// adjoints of phi (i) and of its gradient (ig, ig + 1).
template <typename T>
__device__ __forceinline__ void recon_rev(const BoundRev<T> &r, T x, T y, T &phi_b, T &gx_b, T &gy_b) {
    phi_b += r.v + r.up;
    gx_b += r.v * x;
    gy_b += r.v * y;
}

// Reverse of sst_face for the edge seen from cell c: given the adjoints lk, lw of (Tk, Tw), adds
// to the adjoints of c's and N's 11 cell values.
template <typename T>
__device__ __forceinline__ void sst_face_rev(const T xc[11], const T xn[11], T nlx, T nly, T rx, T ry, T qx, T qy, T lk,
                                             T lw, T xcb[11], T xnb[11]) {
    const T mdot = T(0.5) * ((xc[0] * xc[1] + xn[0] * xn[1]) * nlx + (xc[0] * xc[2] + xn[0] * xn[2]) * nly);
    const bool up_c = mdot >= T(0);
    const T vk = up_c ? xc[3] + xc[5] * rx + xc[6] * ry : xn[3] + xn[5] * qx + xn[6] * qy;
    const T vw = up_c ? xc[4] + xc[7] * rx + xc[8] * ry : xn[4] + xn[7] * qx + xn[8] * qy;
    const T kf = bound_face(vk, up_c ? xc[3] : xn[3]);
    const T wf = bound_face(vw, up_c ? xc[4] : xn[4]);
    const T ddx = rx - qx, ddy = ry - qy;
    const T hn = (ddx * nlx + ddy * nly) * recip(ddx * ddx + ddy * ddy);
    // Tk = -mdot kf + 0.5 (Gk_c + Gk_N) (k_N - k_c) hn, likewise Tw
    const T mdot_b = -lk * kf - lw * wf;
    const T kf_b = -lk * mdot, wf_b = -lw * mdot;
    const T gk = T(0.5) * lk * (xn[3] - xc[3]) * hn, gw = T(0.5) * lw * (xn[4] - xc[4]) * hn;
    xcb[9] += gk;
    xnb[9] += gk;
    xcb[10] += gw;
    xnb[10] += gw;
    const T dk = T(0.5) * (xc[9] + xn[9]) * hn * lk, dw = T(0.5) * (xc[10] + xn[10]) * hn * lw;
    xnb[3] += dk;
    xcb[3] -= dk;
    xnb[4] += dw;
    xcb[4] -= dw;
    if (up_c) {
        recon_rev(bound_face_rev(vk, xc[3], kf_b), rx, ry, xcb[3], xcb[5], xcb[6]);
        recon_rev(bound_face_rev(vw, xc[4], wf_b), rx, ry, xcb[4], xcb[7], xcb[8]);
    } else {
        recon_rev(bound_face_rev(vk, xn[3], kf_b), qx, qy, xnb[3], xnb[5], xnb[6]);
        recon_rev(bound_face_rev(vw, xn[4], wf_b), qx, qy, xnb[4], xnb[7], xnb[8]);
    }
    // mdot = 0.5 ((rho_c u_c + rho_N u_N) nlx + (rho_c v_c + rho_N v_N) nly)
    const T h = T(0.5) * mdot_b;
    xcb[0] += h * (xc[1] * nlx + xc[2] * nly);
    xcb[1] += h * xc[0] * nlx;
    xcb[2] += h * xc[0] * nly;
    xnb[0] += h * (xn[1] * nlx + xn[2] * nly);
    xnb[1] += h * xn[0] * nlx;
    xnb[2] += h * xn[0] * nly;
}

// Reverse of sst_bface: adds to the cell's adjoints and returns the theta adjoint (rot: the
// boundary velocity is the rotated inflow, d ub / d theta = (-ub_y, ub_x)).
template <typename T>
__device__ __forceinline__ T sst_bface_rev(const T xc[11], bool zg, bool rot, T ubx, T uby, T kb, T wb, T nlx, T nly, T rx,
                                           T ry, T l_over_dp, T lk, T lw, T xcb[11]) {
    const T bux = zg ? xc[1] : ubx, buy = zg ? xc[2] : uby;
    const T bk = zg ? xc[3] : kb, bw = zg ? xc[4] : wb;
    const T mdot = xc[0] * (bux * nlx + buy * nly);
    const bool up_c = mdot >= T(0);
    const T vk = xc[3] + xc[5] * rx + xc[6] * ry, vw = xc[4] + xc[7] * rx + xc[8] * ry;
    const T kf = up_c ? bound_face(vk, xc[3]) : bk;
    const T wf = up_c ? bound_face(vw, xc[4]) : bw;
    const T mdot_b = -lk * kf - lw * wf;
    const T kf_b = -lk * mdot, wf_b = -lw * mdot;
    if (!zg) {
        xcb[9] += lk * (bk - xc[3]) * l_over_dp;
        xcb[3] -= lk * xc[9] * l_over_dp;
        xcb[10] += lw * (bw - xc[4]) * l_over_dp;
        xcb[4] -= lw * xc[10] * l_over_dp;
    }
    if (up_c) {
        recon_rev(bound_face_rev(vk, xc[3], kf_b), rx, ry, xcb[3], xcb[5], xcb[6]);
        recon_rev(bound_face_rev(vw, xc[4], wf_b), rx, ry, xcb[4], xcb[7], xcb[8]);
    } else if (zg) {
        xcb[3] += kf_b;
        xcb[4] += wf_b;
    }
    xcb[0] += mdot_b * (bux * nlx + buy * nly);
    const T bux_b = mdot_b * xc[0] * nlx, buy_b = mdot_b * xc[0] * nly;
    if (zg) {
        xcb[1] += bux_b;
        xcb[2] += buy_b;
        return T(0);
    }
    return rot ? bux_b * (-uby) + buy_b * ubx : T(0);
}

// Reverse of sst_nut: given the adjoint of nu_t, adds to the adjoints of k1, omega1 (kb, wb) and of
// the strain rate (Sr_b), and to that of a1.
template <typename T>
__device__ __forceinline__ void sst_nut_rev(T k1, T w1, T Sr, T d, const StepPar<T> &p, const SstParams<T> &q, T nut_bar,
                                            T &kb, T &wb, T &Sr_b, SstParBar<T> &pb) {
    const T idd = recip(d);
    const T sk1 = ssqrt(k1);
    const T iw1 = recip(w1);
    const T A = T(2.0 / 0.09) * sk1 * iw1 * idd;
    const T B = T(500) * p.nu * iw1 * idd * idd;
    const bool a_first = A >= B;
    const T arg2 = a_first ? A : B;
    const T F2 = stanh(arg2 * arg2);
    const bool den_first = q.a1 * w1 >= Sr * F2;
    const T den = den_first ? q.a1 * w1 : Sr * F2;
    const T iden = recip(den);
    const T nut = q.a1 * k1 * iden;
    kb += nut_bar * q.a1 * iden;
    pb.a1 += nut_bar * k1 * iden;
    const T den_b = -nut_bar * nut * iden;
    T F2_b = 0;
    if (den_first) {
        pb.a1 += den_b * w1;
        wb += den_b * q.a1;
    } else {
        Sr_b += den_b * F2;
        F2_b += den_b * Sr;
    }
    const T arg2_b = F2_b * sech2(arg2 * arg2) * T(2) * arg2;
    if (a_first) {
        const T sk1_b = arg2_b * T(2.0 / 0.09) * iw1 * idd;
        wb -= arg2_b * A * iw1;
        kb += sk1 > T(0) ? sk1_b * T(0.5) * recip(sk1) : T(0);
    } else {
        wb -= arg2_b * B * iw1;
    }
}

// Reverse of sst_update: given the adjoints of k1, omega1 and nu_t, adds to the adjoints of rho,
// k, omega (xb[0..2]) and returns those of net_k, net_w, sk, sw, beta, Sr in ob[0..5].
template <typename T>
__device__ __forceinline__ void sst_update_rev(T rho, T k, T w, T net_k, T net_w, T sk, T sw, T beta, T Sr, T d, T inv_area,
                                               const StepPar<T> &p, const SstParams<T> &q, T k1_bar, T w1_bar, T nut_bar,
                                               T xb[3], T ob[6], SstParBar<T> &pb) {
    // forward, in the expressions of sst_update
    const T dt = p.dt;
    const T irho = recip(rho);
    const T fac = dt * inv_area * irho;
    const T skp = sk >= T(0) ? sk : T(0), skm = -sk >= T(0) ? -sk : T(0);
    const T swp = sw >= T(0) ? sw : T(0), swm = -sw >= T(0) ? -sw : T(0);
    const T ik = recip(k), iw = recip(w);
    const T kn = k + fac * net_k + skp, kd = T(1) + dt * q.bstar * w + skm * ik;
    const T wn = w + fac * net_w + swp, wd = T(1) + dt * beta * w + swm * iw;
    const T ikd = recip(kd), iwd = recip(wd);
    const T kr = kn * ikd, wr = wn * iwd;
    const bool kpass = kr >= T(1e-20), wpass = wr >= T(1e-20);
    const T k1 = kpass ? kr : T(1e-20), w1 = wpass ? wr : T(1e-20);
    // reverse
    T kb = k1_bar, wb = w1_bar, Sr_b = 0;
    sst_nut_rev(k1, w1, Sr, d, p, q, nut_bar, kb, wb, Sr_b, pb);
    const T kr_b = kpass ? kb : T(0), wr_b = wpass ? wb : T(0);
    const T kn_b = kr_b * ikd, kd_b = -kr_b * kr * ikd;
    const T wn_b = wr_b * iwd, wd_b = -wr_b * wr * iwd;
    T rho_b = 0, k_b = kn_b, w_b = wn_b, fac_b = kn_b * net_k + wn_b * net_w;
    ob[0] = kn_b * fac;
    ob[1] = wn_b * fac;
    T sk_b = sk >= T(0) ? kn_b : T(0);
    T sw_b = sw >= T(0) ? wn_b : T(0);
    // kd = 1 + dt b* w + max(-sk, 0) / k
    pb.bstar += kd_b * dt * w;
    w_b += kd_b * dt * q.bstar;
    if (-sk >= T(0)) sk_b -= kd_b * ik;
    k_b -= kd_b * skm * ik * ik;
    // wd = 1 + dt beta w + max(-sw, 0) / w
    const T beta_b = wd_b * dt * w;
    w_b += wd_b * dt * beta;
    if (-sw >= T(0)) sw_b -= wd_b * iw;
    w_b -= wd_b * swm * iw * iw;
    // fac = dt ia / rho
    rho_b -= fac_b * fac * irho;
    xb[0] += rho_b;
    xb[1] += k_b;
    xb[2] += w_b;
    ob[2] = sk_b;
    ob[3] = sw_b;
    ob[4] = beta_b;
    ob[5] = Sr_b;
}

}  // namespace fvlbm
