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
//    D2Q5 / D3Q7 moment sets.
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
  R omg[7];   // thermal rates
  R cs2T;     // thermal diffusion parameter c^_s^2
  R gbeta;    // buoyancy per unit temperature along the up axis
  R T0;       // Boussinesq reference temperature
  R rho_r;    // storage offset of f (0: plain populations)
  R T_r;      // storage offset of g at the box centre (0: plain populations)
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
// 2D: D2Q9 fluid + D2Q5 thermal.  f, g hold the pulled (pre-collision) stored
// values on entry and the post-collision stored values on exit.
// ---------------------------------------------------------------------------
// Tr: storage reference of g at this node (g is stored as g - w^T Tr).
template <class R, int UP, bool STD = false>
__device__ __forceinline__ void collide2d(R (&f)[kQ2], R (&g)[kQ2T], const CollParams<R>& c, R Tr,
                                          Macros<R>* mac) {
  constexpr R cs2 = R(1) / R(3);
  const R rr = rho_ref(c);
  const R drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const R dT = ((g[0] + g[1]) + (g[2] + g[3])) + g[4];
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
  auto om = [&](int k) -> R { return rate_f<2, STD>(c, k); };
  const R t10 = k10 + om(1) * (rr * ux - k10) + (R(1) - R(0.5) * om(1)) * Fx;
  const R t01 = k01 + om(2) * (rr * uy - k01) + (R(1) - R(0.5) * om(2)) * Fy;
  const R k2s = k20 + k02, k2d = k20 - k02;
  const R t2s = k2s + om(3) * ((R(2) * cs2 * drho - rr * (uxx + uyy)) - k2s);
  const R t2d = k2d + om(4) * (-rr * (uxx - uyy) - k2d);
  const R t11 = k11 + om(5) * (-rr * uxy - k11);
  const R t20 = R(0.5) * (t2s + t2d);
  const R t02 = R(0.5) * (t2s - t2d);
  const R t21 = k21 + om(6) * (rr * A * uy - k21) + (R(1) - R(0.5) * om(6)) * s21;
  const R t12 = k12 + om(7) * (rr * ux * B - k12) + (R(1) - R(0.5) * om(7)) * s12;
  // kappa^Mv_22 = (kappa~20 kappa~02 + 2 kappa~11^2) / rho
  const R mv22 = (dprod(rr, A, t20, B, t02) + R(2) * dprod(rr, uxy, t11, uxy, t11) +
                  rr * rr * (R(2) * uxx * uyy) - rr * A * B * drho) * irho;
  const R t22 = k22 + om(8) * (mv22 - k22) + (R(1) - R(0.5) * om(8)) * s22;

  // central -> populations: y shifts per mx, then x shifts per row ey
  shift_inv(drho, t01, t02, uy, x0m, x0z, x0p);
  shift_inv(t10, t11, t12, uy, x1m, x1z, x1p);
  shift_inv(t20, t21, t22, uy, x2m, x2z, x2p);
  shift_inv(x0m, x1m, x2m, ux, f[7], f[4], f[8]);
  shift_inv(x0z, x1z, x2z, ux, f[3], f[0], f[1]);
  shift_inv(x0p, x1p, x2p, ux, f[6], f[2], f[5]);

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

// ---------------------------------------------------------------------------
// 3D: D3Q27 fluid + D3Q7 thermal.
// ---------------------------------------------------------------------------

// position of (i, j, k) in a 3x3x3 work array (i, j, k in {0, 1, 2})
__device__ constexpr int I3(int i, int j, int k) { return i * 9 + j * 3 + k; }

template <class R>
__device__ __forceinline__ R cpow(int m, R u, R cs2) {
  return m == 0 ? R(1) : (m == 1 ? -u : cs2 + u * u);
}

template <class R, int UP, bool STD = false>
__device__ __forceinline__ void collide3d(R (&f)[kQ3], R (&g)[kQ3T], const CollParams<R>& c, R Tr,
                                          Macros<R>* mac) {
  constexpr R cs2 = R(1) / R(3);
  const R rr = rho_ref(c);

  // macros
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int a = 0; a < kQ3; ++a) {
    drho += f[a];
    if (D3_EX[a] != 0) jx += D3_EX[a] > 0 ? f[a] : -f[a];
    if (D3_EY[a] != 0) jy += D3_EY[a] > 0 ? f[a] : -f[a];
    if (D3_EZ[a] != 0) jz += D3_EZ[a] > 0 ? f[a] : -f[a];
  }
  const R dT = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + g[6]);
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
  auto om = [&](int k) -> R { return rate_f<3, STD>(c, k); };
  auto relax = [&](R k, R dmv, R w_, R s) -> R { return k + w_ * (dmv - k) + (R(1) - R(0.5) * w_) * s; };

  // sources of orders 3-6 from pre-collision moments, before anything is overwritten
  const R s120 = sig(1, 2, 0), s102 = sig(1, 0, 2), s210 = sig(2, 1, 0), s012 = sig(0, 1, 2);
  const R s201 = sig(2, 0, 1), s021 = sig(0, 2, 1), s111 = sig(1, 1, 1);
  const R s220 = sig(2, 2, 0), s202 = sig(2, 0, 2), s022 = sig(0, 2, 2);
  const R s211 = sig(2, 1, 1), s121 = sig(1, 2, 1), s112 = sig(1, 1, 2);
  const R s122 = sig(1, 2, 2), s212 = sig(2, 1, 2), s221 = sig(2, 2, 1), s222 = sig(2, 2, 2);

  // order 0 and 1
  w[I3(0, 0, 0)] = drho;
  w[I3(1, 0, 0)] = relax(w[I3(1, 0, 0)], rr * ux, om(1), Fx);
  w[I3(0, 1, 0)] = relax(w[I3(0, 1, 0)], rr * uy, om(2), Fy);
  w[I3(0, 0, 1)] = relax(w[I3(0, 0, 1)], rr * uz, om(3), Fz);
  // order 2: off-diagonal, then trace and the two deviators
  w[I3(1, 1, 0)] = relax(w[I3(1, 1, 0)], -rr * uxy, om(4), R(0));
  w[I3(1, 0, 1)] = relax(w[I3(1, 0, 1)], -rr * uxz, om(5), R(0));
  w[I3(0, 1, 1)] = relax(w[I3(0, 1, 1)], -rr * uyz, om(6), R(0));
  {
    const R a = w[I3(2, 0, 0)], b = w[I3(0, 2, 0)], d = w[I3(0, 0, 2)];
    const R ts = relax(a + b + d, R(3) * cs2 * drho - rr * (uxx + uyy + uzz), om(7), R(0));
    const R t1 = relax(a - b, -rr * (uxx - uyy), om(8), R(0));
    const R t2 = relax(a - d, -rr * (uxx - uzz), om(9), R(0));
    const R t200 = (ts + t1 + t2) * (R(1) / R(3));
    w[I3(2, 0, 0)] = t200;
    w[I3(0, 2, 0)] = t200 - t1;
    w[I3(0, 0, 2)] = t200 - t2;
  }
  // order 3: attractors zero, deviation -rho_r kappa_rest
  w[I3(1, 2, 0)] = relax(w[I3(1, 2, 0)], -rr * Rst(1, 2, 0), om(10), s120);
  w[I3(1, 0, 2)] = relax(w[I3(1, 0, 2)], -rr * Rst(1, 0, 2), om(11), s102);
  w[I3(2, 1, 0)] = relax(w[I3(2, 1, 0)], -rr * Rst(2, 1, 0), om(12), s210);
  w[I3(0, 1, 2)] = relax(w[I3(0, 1, 2)], -rr * Rst(0, 1, 2), om(13), s012);
  w[I3(2, 0, 1)] = relax(w[I3(2, 0, 1)], -rr * Rst(2, 0, 1), om(14), s201);
  w[I3(0, 2, 1)] = relax(w[I3(0, 2, 1)], -rr * Rst(0, 2, 1), om(15), s021);
  w[I3(1, 1, 1)] = relax(w[I3(1, 1, 1)], -rr * Rst(1, 1, 1), om(16), s111);

  // order 4: products of post-collision second-order moments
  const R rr2 = rr * rr;
  auto P = [&](int m1, int n1, int p1, int m2, int n2, int p2) -> R {
    return dprod(rr, Rst(m1, n1, p1), w[I3(m1, n1, p1)], Rst(m2, n2, p2), w[I3(m2, n2, p2)]);
  };
  {
    const R mv220 = (P(2, 0, 0, 0, 2, 0) + R(2) * P(1, 1, 0, 1, 1, 0) + rr2 * (R(2) * uxx * uyy) - rr * A * B * drho) * irho;
    const R mv202 = (P(2, 0, 0, 0, 0, 2) + R(2) * P(1, 0, 1, 1, 0, 1) + rr2 * (R(2) * uxx * uzz) - rr * A * C * drho) * irho;
    const R mv022 = (P(0, 2, 0, 0, 0, 2) + R(2) * P(0, 1, 1, 0, 1, 1) + rr2 * (R(2) * uyy * uzz) - rr * B * C * drho) * irho;
    const R mv211 = (P(2, 0, 0, 0, 1, 1) + R(2) * P(1, 1, 0, 1, 0, 1) + rr2 * (R(2) * uxx * uyz) - rr * A * uyz * drho) * irho;
    const R mv121 = (P(0, 2, 0, 1, 0, 1) + R(2) * P(1, 1, 0, 0, 1, 1) + rr2 * (R(2) * uyy * uxz) - rr * B * uxz * drho) * irho;
    const R mv112 = (P(0, 0, 2, 1, 1, 0) + R(2) * P(0, 1, 1, 1, 0, 1) + rr2 * (R(2) * uzz * uxy) - rr * C * uxy * drho) * irho;
    w[I3(2, 2, 0)] = relax(w[I3(2, 2, 0)], mv220, om(17), s220);
    w[I3(2, 0, 2)] = relax(w[I3(2, 0, 2)], mv202, om(18), s202);
    w[I3(0, 2, 2)] = relax(w[I3(0, 2, 2)], mv022, om(19), s022);
    w[I3(2, 1, 1)] = relax(w[I3(2, 1, 1)], mv211, om(20), s211);
    w[I3(1, 2, 1)] = relax(w[I3(1, 2, 1)], mv121, om(21), s121);
    w[I3(1, 1, 2)] = relax(w[I3(1, 1, 2)], mv112, om(22), s112);
  }
  // order 5: (2 / 5 rho) [...] from post-collision second x third order
  {
    const R f25 = R(2) / R(5);
    const R r122 = f25 * (Rst(0, 2, 0) * Rst(1, 0, 2) + Rst(0, 0, 2) * Rst(1, 2, 0) + R(4) * Rst(0, 1, 1) * Rst(1, 1, 1) +
                          R(2) * (Rst(1, 0, 1) * Rst(0, 2, 1) + Rst(1, 1, 0) * Rst(0, 1, 2))) - Rst(1, 2, 2);
    const R r212 = f25 * (Rst(2, 0, 0) * Rst(0, 1, 2) + Rst(0, 0, 2) * Rst(2, 1, 0) + R(4) * Rst(1, 0, 1) * Rst(1, 1, 1) +
                          R(2) * (Rst(1, 1, 0) * Rst(1, 0, 2) + Rst(0, 1, 1) * Rst(2, 0, 1))) - Rst(2, 1, 2);
    const R r221 = f25 * (Rst(2, 0, 0) * Rst(0, 2, 1) + Rst(0, 2, 0) * Rst(2, 0, 1) + R(4) * Rst(1, 1, 0) * Rst(1, 1, 1) +
                          R(2) * (Rst(0, 1, 1) * Rst(2, 1, 0) + Rst(1, 0, 1) * Rst(1, 2, 0))) - Rst(2, 2, 1);
    const R mv122 = (f25 * (P(0, 2, 0, 1, 0, 2) + P(0, 0, 2, 1, 2, 0) + R(4) * P(0, 1, 1, 1, 1, 1) +
                            R(2) * (P(1, 0, 1, 0, 2, 1) + P(1, 1, 0, 0, 1, 2))) +
                     rr2 * r122 - rr * Rst(1, 2, 2) * drho) * irho;
    const R mv212 = (f25 * (P(2, 0, 0, 0, 1, 2) + P(0, 0, 2, 2, 1, 0) + R(4) * P(1, 0, 1, 1, 1, 1) +
                            R(2) * (P(1, 1, 0, 1, 0, 2) + P(0, 1, 1, 2, 0, 1))) +
                     rr2 * r212 - rr * Rst(2, 1, 2) * drho) * irho;
    const R mv221 = (f25 * (P(2, 0, 0, 0, 2, 1) + P(0, 2, 0, 2, 0, 1) + R(4) * P(1, 1, 0, 1, 1, 1) +
                            R(2) * (P(0, 1, 1, 2, 1, 0) + P(1, 0, 1, 1, 2, 0))) +
                     rr2 * r221 - rr * Rst(2, 2, 1) * drho) * irho;
    w[I3(1, 2, 2)] = relax(w[I3(1, 2, 2)], mv122, om(23), s122);
    w[I3(2, 1, 2)] = relax(w[I3(2, 1, 2)], mv212, om(24), s212);
    w[I3(2, 2, 1)] = relax(w[I3(2, 2, 1)], mv221, om(25), s221);
  }
  // order 6: (1 / 3 rho) [...] from post-collision second x fourth order
  {
    const R f13 = R(1) / R(3);
    const R mv222 = (f13 * (P(2, 0, 0, 0, 2, 2) + P(0, 2, 0, 2, 0, 2) + P(0, 0, 2, 2, 2, 0) +
                            R(4) * (P(1, 1, 0, 1, 1, 2) + P(1, 0, 1, 1, 2, 1) + P(0, 1, 1, 2, 1, 1))) +
                     rr2 * (R(4) / R(3)) * (uxx * uyy * C + uxx * uzz * B + uyy * uzz * A) -
                     rr * A * B * C * drho) * irho;
    w[I3(2, 2, 2)] = relax(w[I3(2, 2, 2)], mv222, om(26), s222);
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

}  // namespace fpc
