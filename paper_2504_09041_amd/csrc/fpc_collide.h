// Node-local collision of the Fokker-Planck central-moment LBM (device code).
//
// Method (Schupbach & Premnath, arXiv 2504.09041):
//  * fluid: central moments kappa_mnp of f, relaxed as
//      kappa~ = kappa + w (kappa^Mv - kappa) + (1 - w/2) sigma        (App. A Step 3)
//    toward the Markovian attractors of the FP recurrence with the diffusion
//    tensor c_s^2 I up to second order and the renormalised kappa~_ab / rho
//    above (Eq. Dij2Dselection, Eq. diffusion-tensor-parameter-3D), which
//    gives zero attractors at orders 1 and 3 and products of post-collision
//    lower moments at orders 4-6 (Eq. D2Q9attractors, Sec. 5.2 list);
//    body-force sources sigma_m = sum_i m_i (F_i / rho) kappa_{m - e_i} with
//    pre-collision moments and the first order taken as zero
//    (Eq. sourceCM2D, Sec. 5.2);
//  * thermal (option A, Eq. Dij2D_goptionA): eta~_0 = T, first order relaxed
//    toward 0, second order toward c^_s^2 T (App. B / App. C Step 3), on the
//    D2Q5 / D3Q7 moment sets; the paper's D2Q9 / D3Q15 thermal lattices, with
//    option A or B and the MCM comparator above second order, further below.
//
// GPU design (not the paper's):
//  * The raw -> central map F(u) P and its inverse are applied as products of
//    1D shifts along x, y, z (the velocity sets are tensor products of
//    {-1, 0, 1}), 8 flops per 1D triple instead of a dense 27x27 product.
//  * Every quantity is carried as a deviation from a reference state: the
//    stored populations are s = f - rho_r w and s_g = g - T_r w^T, and the
//    collision works on delta kappa = kappa - rho_r kappa_rest(u), where
//    kappa_rest(u) = prod_d c_{m_d}(u_d) (c_0 = 1, c_1 = -u, c_2 = c_s^2 + u^2)
//    are the central moments of the weights.  Because F(u) P is linear,
//    delta kappa = F(u) P s, and the attractors are rewritten so that no
//    O(1) quantities are subtracted.  rho_r = T_r = 0 gives the plain FP64
//    algorithm; rho_r = rho0, T_r = T0 gives the FP32 deviation form.
#pragma once

#include <hip/hip_runtime.h>

#include "fpc_lattice.h"

namespace fpc {

template <class R>
struct CollParams {
  R om[27];   // fluid rates in the paper's slot order (see fpclbm.h)
  R omg[15];  // thermal rates (moment order of the thermal lattice)
  R cs2T;     // thermal diffusion parameter c^_s^2
  R gbeta;    // buoyancy per unit temperature along the up axis
  R T0;       // Boussinesq reference temperature
  R rho_r;    // storage offset of f (0: plain populations)
  R T_r;      // storage offset of g at the box centre (0: plain populations)
  int model;  // 0: FP attractors; 1: Maxwellian central moments (MCM comparator, Sec. 7)
  int topt;   // thermal higher-order attractors: 0 option A, 1 option B (Sec. 4.3)
};

// Macros of the time level, produced by the collision for diagnostics.
template <class R>
struct Macros {
  R rho, ux, uy, uz, T;
};

// 1D central moments of a triple (a_-, a_0, a_+) about velocity u:
// k_p = sum_e a_e (e - u)^p, p = 0, 1, 2.
template <class R>
__device__ __forceinline__ void shift_fwd(R am, R a0, R ap, R u, R& k0, R& k1, R& k2) {
  const R s = ap + am;
  const R d = ap - am;
  k0 = a0 + s;
  k1 = d - u * k0;
  k2 = s - R(2) * u * d + u * u * k0;
}

// Inverse of shift_fwd: raw moments r1 = k1 + u k0, r2 = k2 + 2u k1 + u^2 k0,
// then a_0 = k0 - r2, a_+- = (r2 +- r1) / 2.
template <class R>
__device__ __forceinline__ void shift_inv(R k0, R k1, R k2, R u, R& am, R& a0, R& ap) {
  const R r1 = k1 + u * k0;
  const R r2 = k2 + R(2) * u * k1 + u * u * k0;
  a0 = k0 - r2;
  ap = R(0.5) * (r2 + r1);
  am = R(0.5) * (r2 - r1);
}

// X*Y - rr^2 RX RY for X = rr RX + dx, Y = rr RY + dy.
template <class R>
__device__ __forceinline__ R dprod(R rr, R RX, R dx, R RY, R dy) {
  return rr * (RX * dy + RY * dx) + dx * dy;
}

// Relaxation rates.  STD = true: the standard rate set, where only the slots
// carrying the viscosity (2D: 20-02 and 11; 3D: the off-diagonals and the two
// deviators) and the thermal first-order slots relax at the runtime rates
// c.om[4] and c.omg[1], and every other slot at 1 (compile-time, so the
// algebra of those slots folds).  STD = false: every slot at its own rate.
template <int D, bool STD, class R>
__device__ __forceinline__ R rate_f(const CollParams<R>& c, int k) {
  if (!STD) return c.om[k];
  const bool nu = D == 2 ? (k == 4 || k == 5) : (k == 4 || k == 5 || k == 6 || k == 8 || k == 9);
  return nu ? c.om[4] : R(1);
}
// Relaxation of fluid slot K toward the attractor deviation dmv with source
// s (App. A Step 3): k~ = k + w (dmv - k) + (1 - w/2) s.  A slot whose rate
// is the compile-time 1 of the standard set lands on dmv + s/2 directly (the
// same value, without keeping its pre-collision moment).
template <int D>
__device__ __forceinline__ constexpr bool viscous_slot(int k) {
  return D == 2 ? (k == 4 || k == 5) : (k == 4 || k == 5 || k == 6 || k == 8 || k == 9);
}
template <int D, bool STD, int K, class R>
__device__ __forceinline__ R relax_slot(const CollParams<R>& c, R k, R dmv, R s) {
  if constexpr (STD && !viscous_slot<D>(K)) {
    return dmv + R(0.5) * s;
  } else {
    const R w = rate_f<D, STD>(c, K);
    return k + w * (dmv - k) + (R(1) - R(0.5) * w) * s;
  }
}
// The same for a slot without a source (s = 0 written out: a zero source
// would still cost instructions, as IEEE arithmetic cannot drop it).
template <int D, bool STD, int K, class R>
__device__ __forceinline__ R relax_slot(const CollParams<R>& c, R k, R dmv) {
  if constexpr (STD && !viscous_slot<D>(K)) {
    return dmv;
  } else {
    const R w = rate_f<D, STD>(c, K);
    return k + w * (dmv - k);
  }
}
// With the source only when HAS_S (a source known to vanish at compile time).
template <int D, bool STD, int K, bool HAS_S, class R>
__device__ __forceinline__ R relax_src(const CollParams<R>& c, R k, R dmv, R s) {
  if constexpr (HAS_S)
    return relax_slot<D, STD, K>(c, k, dmv, s);
  else
    return relax_slot<D, STD, K>(c, k, dmv);
}
// Whether the force source sigma_m = m_up (F / rho) kappa_{m - e_up} of
// moment (m, n, p) can be non-zero: m_up > 0 and m - e_up not of order 1
// (first-order central moments taken as zero).
__device__ __forceinline__ constexpr bool has_sig(int up, int m, int n, int p) {
  const int mu = up == 0 ? m : (up == 1 ? n : p);
  return mu != 0 && (m + n + p - 1) != 1;
}

// The standard build (STD) also fixes the FP attractors and thermal option
// A at compile time; the MCM comparator and option B run the general build.
template <bool STD, class R>
__device__ __forceinline__ bool mcm(const CollParams<R>& c) {
  return !STD && c.model != 0;
}
template <bool STD, class R>
__device__ __forceinline__ bool option_b(const CollParams<R>& c) {
  return !STD && c.topt != 0;
}

template <int D, bool STD, class R>
__device__ __forceinline__ R rate_g(const CollParams<R>& c, int k) {
  if (!STD) return c.omg[k];
  return (k >= 1 && k <= D) ? c.omg[1] : R(1);
}

// FP32 storage holds deviations from rho_r; FP64 storage holds the plain
// populations (rho_r = 0, folded at compile time).
template <class R>
__device__ __forceinline__ R rho_ref(const CollParams<R>& c) {
  if constexpr (sizeof(R) == 4) return c.rho_r;
  return R(0);
}


// ---------------------------------------------------------------------------
// The paper's thermal lattices, on plain populations (FP64 storage) or on
// the deviations g - w^T Tr (FP32 storage, see thermal_d2q9):
// D2Q9 (Sec. 4.3-4.4, App. B) and D3Q15 (Sec. 5.3-5.4, App. C).
// Higher-order attractors (Eq. Mvcmattractor2D_g with Eq. Dij2D_goptionA /
// Dij2D_g, and their 3D forms): option A uses c^_s^2 I at every order, option
// B the post-collision second-order moments over T above second order; the
// MCM comparator uses the Maxwellian moments T prod c(m_d).  The first- and
// second-order rules are common to all three.
// ---------------------------------------------------------------------------

// D2Q9 thermal: central moments by 1D shifts (x per row, then y), as for f.
// In the FP32 deviation form g holds g - w^T Tr (Tr: the node's storage
// reference): the shifts are linear, so they give the central moments of the
// deviations, e - Tr kw with kw_ij = c_i(u_x) c_j(u_y) the central moments of
// w^T (c_0 = 1, c_1 = -u, c_2 = c^_s^2 + u^2), and the moments relax as
// deviations toward attractor deviations m - Tr kw formed analytically; the
// inverse shifts of those give the stored post-collision deviations.
// T = Tr + dT, with dT the sum of the stored deviations.
template <class R, bool STD>
__device__ __forceinline__ void thermal_d2q9(R (&g)[kQ2], R ux, R uy, R T, R Tr, R dT, const CollParams<R>& c) {
  R x0m, x1m, x2m, x0z, x1z, x2z, x0p, x1p, x2p;
  shift_fwd(g[7], g[4], g[8], ux, x0m, x1m, x2m);  // ey = -1
  shift_fwd(g[3], g[0], g[1], ux, x0z, x1z, x2z);  // ey =  0
  shift_fwd(g[6], g[2], g[5], ux, x0p, x1p, x2p);  // ey = +1
  R e00, e01, e02, e10, e11, e12, e20, e21, e22;
  shift_fwd(x0m, x0z, x0p, uy, e00, e01, e02);
  shift_fwd(x1m, x1z, x1p, uy, e10, e11, e12);
  shift_fwd(x2m, x2z, x2p, uy, e20, e21, e22);
  (void)e00;  // equals T (the deviation T - Tr in the deviation form)
  auto og = [&](int k) -> R { return rate_g<2, STD>(c, k); };
  const R cT = c.cs2T;
  R t00, t10, t01, t20, t02, t11, t21, t12, t22;
  if constexpr (sizeof(R) == 8) {  // FP64 storage: plain populations
    (void)Tr;
    (void)dT;
    // orders 1-2 (App. B Step 3): first order and 11 toward 0; 2s toward 2 c^2 T, 2d toward 0
    t00 = T;
    t10 = (R(1) - og(1)) * e10;
    t01 = (R(1) - og(2)) * e01;
    const R s2 = e20 + e02, d2 = e20 - e02;
    const R ts = s2 + og(3) * (R(2) * cT * T - s2), td = (R(1) - og(4)) * d2;
    t20 = R(0.5) * (ts + td);
    t02 = R(0.5) * (ts - td);
    t11 = (R(1) - og(5)) * e11;
    R m21, m12, m22;
    if (mcm<STD>(c)) {  // MCM
      m21 = R(0);
      m12 = R(0);
      m22 = cT * cT * T;
    } else if (option_b<STD>(c)) {  // option B (Eq. MvT2DoptionB)
      const R iT = R(1) / T;
      m21 = R(2) / R(3) * iT * (t20 * t01 + R(2) * t11 * t10);
      m12 = R(2) / R(3) * iT * (t02 * t10 + R(2) * t11 * t01);
      m22 = iT * (t20 * t02 + R(2) * t11 * t11);
    } else {  // option A (Eq. MvT2D)
      m21 = R(2) / R(3) * cT * t01;
      m12 = R(2) / R(3) * cT * t10;
      m22 = R(0.5) * cT * (t20 + t02);
    }
    t21 = e21 + og(6) * (m21 - e21);
    t12 = e12 + og(7) * (m12 - e12);
    t22 = e22 + og(8) * (m22 - e22);
  } else {
    const R uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    const R ax = cT + uxx, ay = cT + uyy;  // kw_20, kw_02
    t00 = dT;
    t10 = e10 + og(1) * (Tr * ux - e10);
    t01 = e01 + og(2) * (Tr * uy - e01);
    const R s2 = e20 + e02, d2 = e20 - e02;
    const R ts = s2 + og(3) * ((R(2) * cT * dT - Tr * (uxx + uyy)) - s2);
    const R td = d2 + og(4) * (-Tr * (uxx - uyy) - d2);
    t20 = R(0.5) * (ts + td);
    t02 = R(0.5) * (ts - td);
    t11 = e11 + og(5) * (-Tr * uxy - e11);
    // third- and fourth-order attractor deviations (kw_21 = -u_y ax,
    // kw_12 = -u_x ay, kw_22 = ax ay)
    R d21, d12, d22;
    if (mcm<STD>(c)) {  // MCM
      d21 = Tr * uy * ax;
      d12 = Tr * ux * ay;
      d22 = cT * cT * dT - Tr * (cT * (uxx + uyy) + uxx * uyy);
    } else if (option_b<STD>(c)) {  // option B, from the full post-collision moments
      const R iT = R(1) / T;
      const R f10 = t10 - Tr * ux, f01 = t01 - Tr * uy, f11 = t11 + Tr * uxy;
      const R f20 = t20 + Tr * ax, f02 = t02 + Tr * ay;
      d21 = R(2) / R(3) * iT * (f20 * f01 + R(2) * f11 * f10) + Tr * uy * ax;
      d12 = R(2) / R(3) * iT * (f02 * f10 + R(2) * f11 * f01) + Tr * ux * ay;
      // (f20 f02 + 2 f11^2) / T - Tr ax ay without the cancellation of its
      // leading Tr^2 ax ay terms
      d22 = iT * ((Tr * (ax * t02 + ay * t20) - Tr * ax * ay * dT) + t20 * t02 + R(2) * f11 * f11);
    } else {  // option A
      d21 = R(2) / R(3) * cT * t01 + Tr * uy * (cT / R(3) + uxx);
      d12 = R(2) / R(3) * cT * t10 + Tr * ux * (cT / R(3) + uyy);
      d22 = R(0.5) * cT * (t20 + t02) - Tr * (R(0.5) * cT * (uxx + uyy) + uxx * uyy);
    }
    t21 = e21 + og(6) * (d21 - e21);
    t12 = e12 + og(7) * (d12 - e12);
    t22 = e22 + og(8) * (d22 - e22);
  }
  shift_inv(t00, t01, t02, uy, x0m, x0z, x0p);
  shift_inv(t10, t11, t12, uy, x1m, x1z, x1p);
  shift_inv(t20, t21, t22, uy, x2m, x2z, x2p);
  shift_inv(x0m, x1m, x2m, ux, g[7], g[4], g[8]);
  shift_inv(x0z, x1z, x2z, ux, g[3], g[0], g[1]);
  shift_inv(x0p, x1p, x2p, ux, g[6], g[2], g[5]);
}

// D3Q15 moment set in the paper's order (Sec. 5.4):
// 000 100 010 001 110 101 011 200 020 002 120 012 201 111 220.
namespace t15 {
constexpr int kM[kQ15][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {2, 0, 0},
                             {0, 2, 0}, {0, 0, 2}, {1, 2, 0}, {0, 1, 2}, {2, 0, 1}, {1, 1, 1}, {2, 2, 0}};
// On D3Q15 every raw moment with exponents <= 2 equals one of the set: with
// at most one non-zero exponent it is in the set itself; with two or more
// only the corners contribute, and a corner moment depends only on the
// exponent parities (s^2 = 1).  Index of that set member.
constexpr int alias(int a, int b, int c) {
  const int nz = (a > 0) + (b > 0) + (c > 0);
  if (nz <= 1) {
    if (a + b + c == 0) return 0;
    if (a) return a == 1 ? 1 : 7;
    if (b) return b == 1 ? 2 : 8;
    return c == 1 ? 3 : 9;
  }
  const int p = (a & 1) + 2 * (b & 1) + 4 * (c & 1);
  constexpr int byp[8] = {14, 10, 11, 4, 12, 5, 6, 13};  // parity x + 2y + 4z -> set index
  return byp[p];
}
constexpr int binom(int m, int i) { return (m == 2 && i == 1) ? 2 : 1; }
}  // namespace t15

// sum over i <= m (componentwise) of prod_d binom(m_d, i_d) (-u_d)^(m_d - i_d) r[alias(i)],
// leaving out i == m when SKIP_SELF
template <class R, int K, bool SKIP_SELF>
__device__ __forceinline__ R t15_shift(const R (&r)[kQ15], const R (&nux)[3], const R (&nuy)[3], const R (&nuz)[3]) {
  constexpr int mx = t15::kM[K][0], my = t15::kM[K][1], mz = t15::kM[K][2];
  R acc = R(0);
#pragma unroll
  for (int i = 0; i <= mx; ++i)
#pragma unroll
    for (int j = 0; j <= my; ++j)
#pragma unroll
      for (int k = 0; k <= mz; ++k) {
        if (SKIP_SELF && i == mx && j == my && k == mz) continue;
        const R cf = R(t15::binom(mx, i) * t15::binom(my, j) * t15::binom(mz, k)) * nux[mx - i] * nuy[my - j] *
                     nuz[mz - k];
        acc += cf * r[t15::alias(i, j, k)];
      }
  return acc;
}

template <class R, bool STD>
__device__ __forceinline__ void thermal_d3q15(R (&g)[kQ15], R ux, R uy, R uz, R T, R Tr, R dT,
                                              const CollParams<R>& c) {
  // raw moments: corner Walsh-Hadamard transform h[px + 2py + 4pz] =
  // sum_corners g s_x^px s_y^py s_z^pz, plus the axis pairs and the rest
  R h[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) h[j] = g[7 + j];  // corner j: s_x = -1 if j&1, s_y if j&2, s_z if j&4
#pragma unroll
  for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (!(j & bit)) {
        const R p = h[j], q = h[j | bit];
        h[j] = p + q;
        h[j | bit] = p - q;
      }
  const R Sx = g[1] + g[2], Dx = g[1] - g[2], Sy = g[3] + g[4], Dy = g[3] - g[4];
  const R Sz = g[5] + g[6], Dz = g[5] - g[6];
  R r[kQ15];
  r[0] = g[0] + Sx + Sy + Sz + h[0];
  r[1] = Dx + h[1];
  r[2] = Dy + h[2];
  r[3] = Dz + h[4];
  r[4] = h[3];   // 110
  r[5] = h[5];   // 101
  r[6] = h[6];   // 011
  r[7] = Sx + h[0];
  r[8] = Sy + h[0];
  r[9] = Sz + h[0];
  r[10] = h[1];  // 120
  r[11] = h[2];  // 012
  r[12] = h[4];  // 201
  r[13] = h[7];  // 111
  r[14] = h[0];  // 220
  // central moments (App. C Step 2): binomial expansion about u
  const R nux[3] = {R(1), -ux, ux * ux}, nuy[3] = {R(1), -uy, uy * uy}, nuz[3] = {R(1), -uz, uz * uz};
  R e[kQ15];
#define FPC_T15(K) e[K] = t15_shift<R, K, false>(r, nux, nuy, nuz);
  FPC_T15(1) FPC_T15(2) FPC_T15(3) FPC_T15(4) FPC_T15(5) FPC_T15(6) FPC_T15(7) FPC_T15(8) FPC_T15(9)
  FPC_T15(10) FPC_T15(11) FPC_T15(12) FPC_T15(13) FPC_T15(14)
#undef FPC_T15
  // relaxation (App. C Step 3), moment by moment
  auto og = [&](int k) -> R { return rate_g<3, STD>(c, k); };
  const R cT = c.cs2T;
  R t[kQ15];
  if constexpr (sizeof(R) == 8) {  // FP64 storage: plain populations
    (void)Tr;
    (void)dT;
    t[0] = T;
#pragma unroll
    for (int k = 1; k <= 6; ++k) t[k] = (R(1) - og(k)) * e[k];  // first order, off-diagonal second order
#pragma unroll
    for (int k = 7; k <= 9; ++k) t[k] = e[k] + og(k) * (cT * T - e[k]);
    R m120, m012, m201, m111, m220;
    if (mcm<STD>(c)) {  // MCM
      m120 = m012 = m201 = m111 = R(0);
      m220 = cT * cT * T;
    } else if (option_b<STD>(c)) {  // option B
      const R f = R(2) / (R(3) * T);
      m120 = f * (t[8] * t[1] + R(2) * t[4] * t[2]);
      m012 = f * (t[9] * t[2] + R(2) * t[6] * t[3]);
      m201 = f * (t[7] * t[3] + R(2) * t[5] * t[1]);
      m111 = f * (t[4] * t[3] + t[5] * t[2] + t[6] * t[1]);
      m220 = (t[7] * t[8] + R(2) * t[4] * t[4]) / T;
    } else {  // option A
      m120 = R(2) / R(3) * cT * t[1];
      m012 = R(2) / R(3) * cT * t[2];
      m201 = R(2) / R(3) * cT * t[3];
      m111 = R(0);
      m220 = R(0.5) * cT * (t[7] + t[8]);
    }
    t[10] = e[10] + og(10) * (m120 - e[10]);
    t[11] = e[11] + og(11) * (m012 - e[11]);
    t[12] = e[12] + og(12) * (m201 - e[12]);
    t[13] = e[13] + og(13) * (m111 - e[13]);
    t[14] = e[14] + og(14) * (m220 - e[14]);
  } else {
    // deviation form (g holds g - w^T Tr): e are the central moments of the
    // deviations, e - Tr kw with kw_m = prod_d c_(m_d)(u_d) the central
    // moments of w^T (c_0 = 1, c_1 = -u, c_2 = c^_s^2 + u^2); relax toward
    // the attractor deviations m - Tr kw, formed analytically
    const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
    const R ax = cT + uxx, ay = cT + uyy, az = cT + uzz;
    t[0] = dT;
    t[1] = e[1] + og(1) * (Tr * ux - e[1]);
    t[2] = e[2] + og(2) * (Tr * uy - e[2]);
    t[3] = e[3] + og(3) * (Tr * uz - e[3]);
    t[4] = e[4] + og(4) * (-Tr * (ux * uy) - e[4]);
    t[5] = e[5] + og(5) * (-Tr * (ux * uz) - e[5]);
    t[6] = e[6] + og(6) * (-Tr * (uy * uz) - e[6]);
    t[7] = e[7] + og(7) * ((cT * dT - Tr * uxx) - e[7]);
    t[8] = e[8] + og(8) * ((cT * dT - Tr * uyy) - e[8]);
    t[9] = e[9] + og(9) * ((cT * dT - Tr * uzz) - e[9]);
    const R uxyz = ux * uy * uz;
    R d120, d012, d201, d111, d220;
    if (mcm<STD>(c)) {  // MCM
      d120 = Tr * ux * ay;
      d012 = Tr * uy * az;
      d201 = Tr * uz * ax;
      d111 = Tr * uxyz;
      d220 = cT * cT * dT - Tr * (cT * (uxx + uyy) + uxx * uyy);
    } else if (option_b<STD>(c)) {  // option B, from the full post-collision moments
      const R f = R(2) / (R(3) * T);
      const R F1 = t[1] - Tr * ux, F2 = t[2] - Tr * uy, F3 = t[3] - Tr * uz;
      const R F4 = t[4] + Tr * (ux * uy), F5 = t[5] + Tr * (ux * uz), F6 = t[6] + Tr * (uy * uz);
      const R F7 = t[7] + Tr * ax, F8 = t[8] + Tr * ay, F9 = t[9] + Tr * az;
      d120 = f * (F8 * F1 + R(2) * F4 * F2) + Tr * ux * ay;
      d012 = f * (F9 * F2 + R(2) * F6 * F3) + Tr * uy * az;
      d201 = f * (F7 * F3 + R(2) * F5 * F1) + Tr * uz * ax;
      d111 = f * (F4 * F3 + F5 * F2 + F6 * F1) + Tr * uxyz;
      // (F7 F8 + 2 F4^2) / T - Tr ax ay without the cancellation of its
      // leading Tr^2 ax ay terms
      d220 = ((Tr * (ax * t[8] + ay * t[7]) - Tr * ax * ay * dT) + t[7] * t[8] + R(2) * F4 * F4) / T;
    } else {  // option A
      d120 = R(2) / R(3) * cT * t[1] + Tr * ux * (cT / R(3) + uyy);
      d012 = R(2) / R(3) * cT * t[2] + Tr * uy * (cT / R(3) + uzz);
      d201 = R(2) / R(3) * cT * t[3] + Tr * uz * (cT / R(3) + uxx);
      d111 = Tr * uxyz;
      d220 = R(0.5) * cT * (t[7] + t[8]) - Tr * (R(0.5) * cT * (uxx + uyy) + uxx * uyy);
    }
    t[10] = e[10] + og(10) * (d120 - e[10]);
    t[11] = e[11] + og(11) * (d012 - e[11]);
    t[12] = e[12] + og(12) * (d201 - e[12]);
    t[13] = e[13] + og(13) * (d111 - e[13]);
    t[14] = e[14] + og(14) * (d220 - e[14]);
  }
  // raw moments back: the central map is unit lower triangular in this order,
  // so r_m = t_m - (terms of lower members), member by member
  r[0] = t[0];
#define FPC_T15I(K) r[K] = t[K] - t15_shift<R, K, true>(r, nux, nuy, nuz);
  FPC_T15I(1) FPC_T15I(2) FPC_T15I(3) FPC_T15I(4) FPC_T15I(5) FPC_T15I(6) FPC_T15I(7) FPC_T15I(8) FPC_T15I(9)
  FPC_T15I(10) FPC_T15I(11) FPC_T15I(12) FPC_T15I(13) FPC_T15I(14)
#undef FPC_T15I
  // populations: corners by the inverse Hadamard transform of
  // (220, 120, 012, 110, 201, 101, 011, 111); axis pairs and rest from the rest
  h[0] = r[14];
  h[1] = r[10];
  h[2] = r[11];
  h[3] = r[4];
  h[4] = r[12];
  h[5] = r[5];
  h[6] = r[6];
  h[7] = r[13];
#pragma unroll
  for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (!(j & bit)) {
        const R p = h[j], q = h[j | bit];
        h[j] = p + q;
        h[j | bit] = p - q;
      }
#pragma unroll
  for (int j = 0; j < 8; ++j) g[7 + j] = R(0.125) * h[j];
  g[1] = R(0.5) * ((r[7] - r[14]) + (r[1] - r[10]));
  g[2] = R(0.5) * ((r[7] - r[14]) - (r[1] - r[10]));
  g[3] = R(0.5) * ((r[8] - r[14]) + (r[2] - r[11]));
  g[4] = R(0.5) * ((r[8] - r[14]) - (r[2] - r[11]));
  g[5] = R(0.5) * ((r[9] - r[14]) + (r[3] - r[12]));
  g[6] = R(0.5) * ((r[9] - r[14]) - (r[3] - r[12]));
  g[0] = r[0] - r[7] - r[8] - r[9] + R(2) * r[14];
}

// ---------------------------------------------------------------------------
// 2D: D2Q9 fluid + D2Q5 thermal.  f, g hold the pulled (pre-collision) stored
// values on entry and the post-collision stored values on exit.
// ---------------------------------------------------------------------------
// Tr: storage reference of g at this node (g is stored as g - w^T Tr).
// QG: thermal lattice, D2Q5 (5, deviation form) or D2Q9 (9, plain populations).
template <class R, int UP, bool STD = false, int QG = kQ2T>
__device__ __forceinline__ void collide2d(R (&f)[kQ2], R (&g)[QG], const CollParams<R>& c, R Tr,
                                          Macros<R>* mac) {
  constexpr R cs2 = R(1) / R(3);
  const R rr = rho_ref(c);
  const R drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  R dT;
  if constexpr (QG == kQ2T) {
    dT = ((g[0] + g[1]) + (g[2] + g[3])) + g[4];
  } else {
    dT = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  }
  const R T = Tr + dT;
  const R rho = rr + drho;
  const R Fb = c.gbeta * (T - c.T0);
  const R Fx = UP == 0 ? Fb : R(0);
  const R Fy = UP == 1 ? Fb : R(0);
  const R irho = R(1) / rho;
  const R ux = (jx + R(0.5) * Fx) * irho;
  const R uy = (jy + R(0.5) * Fy) * irho;
  if (mac) {
    mac->rho = rho;
    mac->ux = ux;
    mac->uy = uy;
    mac->uz = R(0);
    mac->T = T;
  }
  const R uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
  const R A = cs2 + uxx, B = cs2 + uyy;  // c_2(u_x), c_2(u_y)

  // f -> central moment deviations: x shifts per row ey, then y shifts per mx
  R x0m, x1m, x2m, x0z, x1z, x2z, x0p, x1p, x2p;
  shift_fwd(f[7], f[4], f[8], ux, x0m, x1m, x2m);  // ey = -1
  shift_fwd(f[3], f[0], f[1], ux, x0z, x1z, x2z);  // ey =  0
  shift_fwd(f[6], f[2], f[5], ux, x0p, x1p, x2p);  // ey = +1
  R k00, k01, k02, k10, k11, k12, k20, k21, k22;
  shift_fwd(x0m, x0z, x0p, uy, k00, k01, k02);
  shift_fwd(x1m, x1z, x1p, uy, k10, k11, k12);
  shift_fwd(x2m, x2z, x2p, uy, k20, k21, k22);

  // sources: sigma_m = m_up (F/rho) kappa_{m - e_up}, full pre-collision moments
  const R Fr = Fb * irho;
  R s21, s12, s22;
  if (UP == 1) {
    s21 = Fr * (rr * A + k20);                    // kappa_20
    s12 = R(2) * Fr * (rr * uxy + k11);           // kappa_11
    s22 = R(2) * Fr * (rr * (-A * uy) + k21);     // kappa_21
  } else {
    s21 = R(2) * Fr * (rr * uxy + k11);           // kappa_11
    s12 = Fr * (rr * B + k02);                    // kappa_02
    s22 = R(2) * Fr * (rr * (-ux * B) + k12);     // kappa_12
  }

  // relaxation (deviation form; attractor deviations dMv = Mv - rho_r kappa_rest)
  const R t10 = relax_src<2, STD, 1, UP == 0>(c, k10, rr * ux, Fx);
  const R t01 = relax_src<2, STD, 2, UP == 1>(c, k01, rr * uy, Fy);
  const R k2s = k20 + k02, k2d = k20 - k02;
  const R t2s = relax_slot<2, STD, 3>(c, k2s, R(2) * cs2 * drho - rr * (uxx + uyy));
  const R t2d = relax_slot<2, STD, 4>(c, k2d, -rr * (uxx - uyy));
  const R t11 = relax_slot<2, STD, 5>(c, k11, -rr * uxy);
  const R t20 = R(0.5) * (t2s + t2d);
  const R t02 = R(0.5) * (t2s - t2d);
  const R t21 = relax_slot<2, STD, 6>(c, k21, rr * A * uy, s21);
  const R t12 = relax_slot<2, STD, 7>(c, k12, rr * ux * B, s12);
  // kappa^Mv_22 = (kappa~20 kappa~02 + 2 kappa~11^2) / rho (FP); rho c_s^4 (MCM)
  R mv22;
  if (mcm<STD>(c))
    mv22 = drho * (cs2 * cs2) - rr * (cs2 * (uxx + uyy) + uxx * uyy);
  else
    mv22 = (dprod(rr, A, t20, B, t02) + R(2) * dprod(rr, uxy, t11, uxy, t11) + rr * rr * (R(2) * uxx * uyy) -
            rr * A * B * drho) * irho;
  const R t22 = relax_slot<2, STD, 8>(c, k22, mv22, s22);

  // central -> populations: y shifts per mx, then x shifts per row ey
  shift_inv(drho, t01, t02, uy, x0m, x0z, x0p);
  shift_inv(t10, t11, t12, uy, x1m, x1z, x1p);
  shift_inv(t20, t21, t22, uy, x2m, x2z, x2p);
  shift_inv(x0m, x1m, x2m, ux, f[7], f[4], f[8]);
  shift_inv(x0z, x1z, x2z, ux, f[3], f[0], f[1]);
  shift_inv(x0p, x1p, x2p, ux, f[6], f[2], f[5]);

  if constexpr (QG != kQ2T) {
    thermal_d2q9<R, STD>(g, ux, uy, T, Tr, dT, c);
    return;
  } else {
  // thermal D2Q5: raw moments (00, 10, 01, 20, 02) -> central -> relax -> back
  const R cT = c.cs2T;
  auto og = [&](int k) -> R { return rate_g<2, STD>(c, k); };
  const R n10 = g[1] - g[3], n01 = g[2] - g[4], n20 = g[1] + g[3], n02 = g[2] + g[4];
  const R e10 = n10 - ux * dT;
  const R e01 = n01 - uy * dT;
  const R e20 = n20 - R(2) * ux * n10 + uxx * dT;
  const R e02 = n02 - R(2) * uy * n01 + uyy * dT;
  const R te10 = e10 + og(1) * (Tr * ux - e10);
  const R te01 = e01 + og(2) * (Tr * uy - e01);
  const R e2s = e20 + e02, e2d = e20 - e02;
  const R te2s = e2s + og(3) * ((R(2) * cT * dT - Tr * (uxx + uyy)) - e2s);
  const R te2d = e2d + og(4) * (-Tr * (uxx - uyy) - e2d);
  const R te20 = R(0.5) * (te2s + te2d);
  const R te02 = R(0.5) * (te2s - te2d);
  const R m10 = te10 + ux * dT;
  const R m01 = te01 + uy * dT;
  const R m20 = te20 + R(2) * ux * te10 + uxx * dT;
  const R m02 = te02 + R(2) * uy * te01 + uyy * dT;
  g[0] = dT - m20 - m02;
  g[1] = R(0.5) * (m20 + m10);
  g[3] = R(0.5) * (m20 - m10);
  g[2] = R(0.5) * (m02 + m01);
  g[4] = R(0.5) * (m02 - m01);
  }
}

// ---------------------------------------------------------------------------
// 3D: D3Q27 fluid + D3Q7 thermal.
// ---------------------------------------------------------------------------

// position of (i, j, k) in a 3x3x3 work array (i, j, k in {0, 1, 2})
__device__ constexpr int I3(int i, int j, int k) { return i * 9 + j * 3 + k; }

template <class R>
__device__ __forceinline__ R cpow(int m, R u, R cs2) {
  return m == 0 ? R(1) : (m == 1 ? -u : cs2 + u * u);
}

// QG: thermal lattice, D3Q7 (7, deviation form) or D3Q15 (15, plain populations).
template <class R, int UP, bool STD = false, int QG = kQ3T>
__device__ __forceinline__ void collide3d(R (&f)[kQ3], R (&g)[QG], const CollParams<R>& c, R Tr,
                                          Macros<R>* mac) {
  constexpr R cs2 = R(1) / R(3);
  const R rr = rho_ref(c);

  // macros (each sum starts from its first term: an explicit 0 + x would
  // cost an IEEE add)
  R drho = f[0], jx = R(0), jy = R(0), jz = R(0);
  bool hx = false, hy = false, hz = false;
#pragma unroll
  for (int a = 1; a < kQ3; ++a) {
    drho += f[a];
    if (D3_EX[a] != 0) {
      jx = hx ? (D3_EX[a] > 0 ? jx + f[a] : jx - f[a]) : (D3_EX[a] > 0 ? f[a] : -f[a]);
      hx = true;
    }
    if (D3_EY[a] != 0) {
      jy = hy ? (D3_EY[a] > 0 ? jy + f[a] : jy - f[a]) : (D3_EY[a] > 0 ? f[a] : -f[a]);
      hy = true;
    }
    if (D3_EZ[a] != 0) {
      jz = hz ? (D3_EZ[a] > 0 ? jz + f[a] : jz - f[a]) : (D3_EZ[a] > 0 ? f[a] : -f[a]);
      hz = true;
    }
  }
  R dT = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + g[6]);
  if constexpr (QG != kQ3T) {
    R dc = R(0);
#pragma unroll
    for (int q = 7; q < QG; ++q) dc += g[q];
    dT += dc;
  }
  const R T = Tr + dT;
  const R rho = rr + drho;
  const R Fb = c.gbeta * (T - c.T0);
  const R Fx = UP == 0 ? Fb : R(0);
  const R Fy = UP == 1 ? Fb : R(0);
  const R Fz = UP == 2 ? Fb : R(0);
  const R irho = R(1) / rho;
  const R ux = (jx + R(0.5) * Fx) * irho;
  const R uy = (jy + R(0.5) * Fy) * irho;
  const R uz = (jz + R(0.5) * Fz) * irho;
  if (mac) {
    mac->rho = rho;
    mac->ux = ux;
    mac->uy = uy;
    mac->uz = uz;
    mac->T = T;
  }
  const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
  const R uxy = ux * uy, uxz = ux * uz, uyz = uy * uz;
  const R A = cs2 + uxx, B = cs2 + uyy, C = cs2 + uzz;

  // f -> central moment deviations, work array w[I3(., ., .)]:
  // after the x pass w[I3(mx, ey+1, ez+1)], after y w[I3(mx, my, ez+1)],
  // after z w[I3(mx, my, mz)].
  R w[27];
#pragma unroll
  for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
    for (int ez = -1; ez <= 1; ++ez)
      shift_fwd(f[d3_index(-1, ey, ez)], f[d3_index(0, ey, ez)], f[d3_index(1, ey, ez)], ux,
                w[I3(0, ey + 1, ez + 1)], w[I3(1, ey + 1, ez + 1)], w[I3(2, ey + 1, ez + 1)]);
#pragma unroll
  for (int mx = 0; mx < 3; ++mx)
#pragma unroll
    for (int ez = 0; ez < 3; ++ez) {
      R a = w[I3(mx, 0, ez)], b = w[I3(mx, 1, ez)], d = w[I3(mx, 2, ez)];
      shift_fwd(a, b, d, uy, w[I3(mx, 0, ez)], w[I3(mx, 1, ez)], w[I3(mx, 2, ez)]);
    }
#pragma unroll
  for (int mx = 0; mx < 3; ++mx)
#pragma unroll
    for (int my = 0; my < 3; ++my) {
      R a = w[I3(mx, my, 0)], b = w[I3(mx, my, 1)], d = w[I3(mx, my, 2)];
      shift_fwd(a, b, d, uz, w[I3(mx, my, 0)], w[I3(mx, my, 1)], w[I3(mx, my, 2)]);
    }

  // rest central moments kappa_rest(u) = c_m(ux) c_n(uy) c_p(uz)
  auto Rst = [&](int m, int n, int p) -> R { return cpow(m, ux, cs2) * cpow(n, uy, cs2) * cpow(p, uz, cs2); };
  // full pre-collision moment (for the sources)
  auto Kfull = [&](int m, int n, int p) -> R { return rr * Rst(m, n, p) + w[I3(m, n, p)]; };
  const R Fr = Fb * irho;
  // sigma_m = m_up (F/rho) kappa_{m - e_up}; zero when m_up = 0; first order taken as zero
  auto sig = [&](int m, int n, int p) -> R {
    const int mu = UP == 0 ? m : (UP == 1 ? n : p);
    if (mu == 0) return R(0);
    const int m2 = m - (UP == 0), n2 = n - (UP == 1), p2 = p - (UP == 2);
    if (m2 + n2 + p2 == 1) return R(0);
    return R(mu) * Fr * Kfull(m2, n2, p2);
  };

  // sources of orders 3-6 from pre-collision moments, before anything is overwritten
  const R s120 = sig(1, 2, 0), s102 = sig(1, 0, 2), s210 = sig(2, 1, 0), s012 = sig(0, 1, 2);
  const R s201 = sig(2, 0, 1), s021 = sig(0, 2, 1), s111 = sig(1, 1, 1);
  const R s220 = sig(2, 2, 0), s202 = sig(2, 0, 2), s022 = sig(0, 2, 2);
  const R s211 = sig(2, 1, 1), s121 = sig(1, 2, 1), s112 = sig(1, 1, 2);
  const R s122 = sig(1, 2, 2), s212 = sig(2, 1, 2), s221 = sig(2, 2, 1), s222 = sig(2, 2, 2);

  // order 0 and 1
  w[I3(0, 0, 0)] = drho;
  w[I3(1, 0, 0)] = relax_src<3, STD, 1, UP == 0>(c, w[I3(1, 0, 0)], rr * ux, Fx);
  w[I3(0, 1, 0)] = relax_src<3, STD, 2, UP == 1>(c, w[I3(0, 1, 0)], rr * uy, Fy);
  w[I3(0, 0, 1)] = relax_src<3, STD, 3, UP == 2>(c, w[I3(0, 0, 1)], rr * uz, Fz);
  // order 2: off-diagonal, then trace and the two deviators
  w[I3(1, 1, 0)] = relax_slot<3, STD, 4>(c, w[I3(1, 1, 0)], -rr * uxy);
  w[I3(1, 0, 1)] = relax_slot<3, STD, 5>(c, w[I3(1, 0, 1)], -rr * uxz);
  w[I3(0, 1, 1)] = relax_slot<3, STD, 6>(c, w[I3(0, 1, 1)], -rr * uyz);
  {
    const R a = w[I3(2, 0, 0)], b = w[I3(0, 2, 0)], d = w[I3(0, 0, 2)];
    const R ts = relax_slot<3, STD, 7>(c, a + b + d, R(3) * cs2 * drho - rr * (uxx + uyy + uzz));
    const R t1 = relax_slot<3, STD, 8>(c, a - b, -rr * (uxx - uyy));
    const R t2 = relax_slot<3, STD, 9>(c, a - d, -rr * (uxx - uzz));
    const R t200 = (ts + t1 + t2) * (R(1) / R(3));
    w[I3(2, 0, 0)] = t200;
    w[I3(0, 2, 0)] = t200 - t1;
    w[I3(0, 0, 2)] = t200 - t2;
  }
  // order 3: attractors zero, deviation -rho_r kappa_rest
  w[I3(1, 2, 0)] = relax_src<3, STD, 10, has_sig(UP, 1, 2, 0)>(c, w[I3(1, 2, 0)], -rr * Rst(1, 2, 0), s120);
  w[I3(1, 0, 2)] = relax_src<3, STD, 11, has_sig(UP, 1, 0, 2)>(c, w[I3(1, 0, 2)], -rr * Rst(1, 0, 2), s102);
  w[I3(2, 1, 0)] = relax_src<3, STD, 12, has_sig(UP, 2, 1, 0)>(c, w[I3(2, 1, 0)], -rr * Rst(2, 1, 0), s210);
  w[I3(0, 1, 2)] = relax_src<3, STD, 13, has_sig(UP, 0, 1, 2)>(c, w[I3(0, 1, 2)], -rr * Rst(0, 1, 2), s012);
  w[I3(2, 0, 1)] = relax_src<3, STD, 14, has_sig(UP, 2, 0, 1)>(c, w[I3(2, 0, 1)], -rr * Rst(2, 0, 1), s201);
  w[I3(0, 2, 1)] = relax_src<3, STD, 15, has_sig(UP, 0, 2, 1)>(c, w[I3(0, 2, 1)], -rr * Rst(0, 2, 1), s021);
  w[I3(1, 1, 1)] = relax_src<3, STD, 16, has_sig(UP, 1, 1, 1)>(c, w[I3(1, 1, 1)], -rr * Rst(1, 1, 1), s111);

  // order 4: products of post-collision second-order moments
  const R rr2 = rr * rr;
  auto P = [&](int m1, int n1, int p1, int m2, int n2, int p2) -> R {
    return dprod(rr, Rst(m1, n1, p1), w[I3(m1, n1, p1)], Rst(m2, n2, p2), w[I3(m2, n2, p2)]);
  };
  {
    // FP: products of post-collision second-order moments; MCM: rho c_s^4 or 0
    R mv220, mv202, mv022, mv211, mv121, mv112;
    if (mcm<STD>(c)) {
      constexpr R cs4 = cs2 * cs2;
      mv220 = drho * cs4 - rr * (cs2 * (uxx + uyy) + uxx * uyy);
      mv202 = drho * cs4 - rr * (cs2 * (uxx + uzz) + uxx * uzz);
      mv022 = drho * cs4 - rr * (cs2 * (uyy + uzz) + uyy * uzz);
      mv211 = -rr * A * uyz;
      mv121 = -rr * B * uxz;
      mv112 = -rr * C * uxy;
    } else {
      mv220 = (P(2, 0, 0, 0, 2, 0) + R(2) * P(1, 1, 0, 1, 1, 0) + rr2 * (R(2) * uxx * uyy) - rr * A * B * drho) * irho;
      mv202 = (P(2, 0, 0, 0, 0, 2) + R(2) * P(1, 0, 1, 1, 0, 1) + rr2 * (R(2) * uxx * uzz) - rr * A * C * drho) * irho;
      mv022 = (P(0, 2, 0, 0, 0, 2) + R(2) * P(0, 1, 1, 0, 1, 1) + rr2 * (R(2) * uyy * uzz) - rr * B * C * drho) * irho;
      mv211 = (P(2, 0, 0, 0, 1, 1) + R(2) * P(1, 1, 0, 1, 0, 1) + rr2 * (R(2) * uxx * uyz) - rr * A * uyz * drho) * irho;
      mv121 = (P(0, 2, 0, 1, 0, 1) + R(2) * P(1, 1, 0, 0, 1, 1) + rr2 * (R(2) * uyy * uxz) - rr * B * uxz * drho) * irho;
      mv112 = (P(0, 0, 2, 1, 1, 0) + R(2) * P(0, 1, 1, 1, 0, 1) + rr2 * (R(2) * uzz * uxy) - rr * C * uxy * drho) * irho;
    }
    w[I3(2, 2, 0)] = relax_src<3, STD, 17, has_sig(UP, 2, 2, 0)>(c, w[I3(2, 2, 0)], mv220, s220);
    w[I3(2, 0, 2)] = relax_src<3, STD, 18, has_sig(UP, 2, 0, 2)>(c, w[I3(2, 0, 2)], mv202, s202);
    w[I3(0, 2, 2)] = relax_src<3, STD, 19, has_sig(UP, 0, 2, 2)>(c, w[I3(0, 2, 2)], mv022, s022);
    w[I3(2, 1, 1)] = relax_src<3, STD, 20, has_sig(UP, 2, 1, 1)>(c, w[I3(2, 1, 1)], mv211, s211);
    w[I3(1, 2, 1)] = relax_src<3, STD, 21, has_sig(UP, 1, 2, 1)>(c, w[I3(1, 2, 1)], mv121, s121);
    w[I3(1, 1, 2)] = relax_src<3, STD, 22, has_sig(UP, 1, 1, 2)>(c, w[I3(1, 1, 2)], mv112, s112);
  }
  // order 5: (2 / 5 rho) [...] from post-collision second x third order (FP);
  // zero for MCM (deviation -rho_r kappa_rest)
  {
    R mv122, mv212, mv221;
    if (mcm<STD>(c)) {
      mv122 = -rr * Rst(1, 2, 2);
      mv212 = -rr * Rst(2, 1, 2);
      mv221 = -rr * Rst(2, 2, 1);
    } else {
      const R f25 = R(2) / R(5);
      const R r122 = f25 * (Rst(0, 2, 0) * Rst(1, 0, 2) + Rst(0, 0, 2) * Rst(1, 2, 0) + R(4) * Rst(0, 1, 1) * Rst(1, 1, 1) +
                            R(2) * (Rst(1, 0, 1) * Rst(0, 2, 1) + Rst(1, 1, 0) * Rst(0, 1, 2))) - Rst(1, 2, 2);
      const R r212 = f25 * (Rst(2, 0, 0) * Rst(0, 1, 2) + Rst(0, 0, 2) * Rst(2, 1, 0) + R(4) * Rst(1, 0, 1) * Rst(1, 1, 1) +
                            R(2) * (Rst(1, 1, 0) * Rst(1, 0, 2) + Rst(0, 1, 1) * Rst(2, 0, 1))) - Rst(2, 1, 2);
      const R r221 = f25 * (Rst(2, 0, 0) * Rst(0, 2, 1) + Rst(0, 2, 0) * Rst(2, 0, 1) + R(4) * Rst(1, 1, 0) * Rst(1, 1, 1) +
                            R(2) * (Rst(0, 1, 1) * Rst(2, 1, 0) + Rst(1, 0, 1) * Rst(1, 2, 0))) - Rst(2, 2, 1);
      mv122 = (f25 * (P(0, 2, 0, 1, 0, 2) + P(0, 0, 2, 1, 2, 0) + R(4) * P(0, 1, 1, 1, 1, 1) +
                       R(2) * (P(1, 0, 1, 0, 2, 1) + P(1, 1, 0, 0, 1, 2))) +
               rr2 * r122 - rr * Rst(1, 2, 2) * drho) * irho;
      mv212 = (f25 * (P(2, 0, 0, 0, 1, 2) + P(0, 0, 2, 2, 1, 0) + R(4) * P(1, 0, 1, 1, 1, 1) +
                       R(2) * (P(1, 1, 0, 1, 0, 2) + P(0, 1, 1, 2, 0, 1))) +
               rr2 * r212 - rr * Rst(2, 1, 2) * drho) * irho;
      mv221 = (f25 * (P(2, 0, 0, 0, 2, 1) + P(0, 2, 0, 2, 0, 1) + R(4) * P(1, 1, 0, 1, 1, 1) +
                       R(2) * (P(0, 1, 1, 2, 1, 0) + P(1, 0, 1, 1, 2, 0))) +
               rr2 * r221 - rr * Rst(2, 2, 1) * drho) * irho;
    }
    w[I3(1, 2, 2)] = relax_src<3, STD, 23, has_sig(UP, 1, 2, 2)>(c, w[I3(1, 2, 2)], mv122, s122);
    w[I3(2, 1, 2)] = relax_src<3, STD, 24, has_sig(UP, 2, 1, 2)>(c, w[I3(2, 1, 2)], mv212, s212);
    w[I3(2, 2, 1)] = relax_src<3, STD, 25, has_sig(UP, 2, 2, 1)>(c, w[I3(2, 2, 1)], mv221, s221);
  }
  // order 6: (1 / 3 rho) [...] from post-collision second x fourth order (FP);
  // rho c_s^6 for MCM
  {
    R mv222;
    if (mcm<STD>(c)) {
      constexpr R cs4 = cs2 * cs2;
      mv222 = drho * (cs4 * cs2) -
              rr * (cs4 * (uxx + uyy + uzz) + cs2 * (uxx * uyy + uxx * uzz + uyy * uzz) + uxx * uyy * uzz);
    } else {
      const R f13 = R(1) / R(3);
      mv222 = (f13 * (P(2, 0, 0, 0, 2, 2) + P(0, 2, 0, 2, 0, 2) + P(0, 0, 2, 2, 2, 0) +
                      R(4) * (P(1, 1, 0, 1, 1, 2) + P(1, 0, 1, 1, 2, 1) + P(0, 1, 1, 2, 1, 1))) +
               rr2 * (R(4) / R(3)) * (uxx * uyy * C + uxx * uzz * B + uyy * uzz * A) - rr * A * B * C * drho) *
              irho;
    }
    w[I3(2, 2, 2)] = relax_src<3, STD, 26, has_sig(UP, 2, 2, 2)>(c, w[I3(2, 2, 2)], mv222, s222);
  }

  // central -> populations: z shifts, then y, then x
#pragma unroll
  for (int mx = 0; mx < 3; ++mx)
#pragma unroll
    for (int my = 0; my < 3; ++my) {
      R a = w[I3(mx, my, 0)], b = w[I3(mx, my, 1)], d = w[I3(mx, my, 2)];
      shift_inv(a, b, d, uz, w[I3(mx, my, 0)], w[I3(mx, my, 1)], w[I3(mx, my, 2)]);
    }
#pragma unroll
  for (int mx = 0; mx < 3; ++mx)
#pragma unroll
    for (int ez = 0; ez < 3; ++ez) {
      R a = w[I3(mx, 0, ez)], b = w[I3(mx, 1, ez)], d = w[I3(mx, 2, ez)];
      shift_inv(a, b, d, uy, w[I3(mx, 0, ez)], w[I3(mx, 1, ez)], w[I3(mx, 2, ez)]);
    }
#pragma unroll
  for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
    for (int ez = -1; ez <= 1; ++ez)
      shift_inv(w[I3(0, ey + 1, ez + 1)], w[I3(1, ey + 1, ez + 1)], w[I3(2, ey + 1, ez + 1)], ux,
                f[d3_index(-1, ey, ez)], f[d3_index(0, ey, ez)], f[d3_index(1, ey, ez)]);

  if constexpr (QG != kQ3T) {
    thermal_d3q15<R, STD>(g, ux, uy, uz, T, Tr, dT, c);
    return;
  } else {
  // thermal D3Q7: links 1/2 = +-x, 3/4 = +-y, 5/6 = +-z
  const R cT = c.cs2T;
  auto og = [&](int k) -> R { return rate_g<3, STD>(c, k); };
  const R n100 = g[1] - g[2], n010 = g[3] - g[4], n001 = g[5] - g[6];
  const R n200 = g[1] + g[2], n020 = g[3] + g[4], n002 = g[5] + g[6];
  const R e100 = n100 - ux * dT, e010 = n010 - uy * dT, e001 = n001 - uz * dT;
  const R e200 = n200 - R(2) * ux * n100 + uxx * dT;
  const R e020 = n020 - R(2) * uy * n010 + uyy * dT;
  const R e002 = n002 - R(2) * uz * n001 + uzz * dT;
  const R te100 = e100 + og(1) * (Tr * ux - e100);
  const R te010 = e010 + og(2) * (Tr * uy - e010);
  const R te001 = e001 + og(3) * (Tr * uz - e001);
  const R te200 = e200 + og(4) * ((cT * dT - Tr * uxx) - e200);
  const R te020 = e020 + og(5) * ((cT * dT - Tr * uyy) - e020);
  const R te002 = e002 + og(6) * ((cT * dT - Tr * uzz) - e002);
  const R m100 = te100 + ux * dT, m010 = te010 + uy * dT, m001 = te001 + uz * dT;
  const R m200 = te200 + R(2) * ux * te100 + uxx * dT;
  const R m020 = te020 + R(2) * uy * te010 + uyy * dT;
  const R m002 = te002 + R(2) * uz * te001 + uzz * dT;
  g[0] = dT - m200 - m020 - m002;
  g[1] = R(0.5) * (m200 + m100);
  g[2] = R(0.5) * (m200 - m100);
  g[3] = R(0.5) * (m020 + m010);
  g[4] = R(0.5) * (m020 - m010);
  g[5] = R(0.5) * (m002 + m001);
  g[6] = R(0.5) * (m002 - m001);
  }
}

}  // namespace fpc
