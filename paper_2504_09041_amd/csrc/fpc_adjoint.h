// Reverse-mode (adjoint) of the node-local collision, written by hand.
//
// The forward map differentiated here is the same collision as in
// fpc_collide.h (Sec. 4.1-4.2, 5.1-5.2 and App. A for f; Sec. 4.3-4.4, 5.3 and
// App. B/C, option A, for g), evaluated on plain populations:
//   rho = sum f, j = sum f e, T = sum g, F = g beta (T - T0) e_up,
//   u = (j + F/2) / rho                                         (App. A Step 7)
//   kappa = C(u) f        (central moments, tensor product of 1D shifts)
//   kappa~: relaxation order by order, attractors from the recurrence with
//           D' = c_s^2 I up to second order and D'_ab = kappa~_ab / rho above
//           (FP), or the Maxwellian central moments rho prod c(m_d) (MCM),
//           sources sigma_m = m_up (F/rho) kappa_{m - e_up}     (Eq. sourceCM2D)
//   f~ = C(u)^-1 kappa~
//   eta = C_g(u) g, eta~ (option A), g~ = C_g(u)^-1 eta~.
//
// Reverse-mode identities used (no intermediate of the shift passes is kept):
//   d kappa_m / d u_i = -m_i kappa_{m - e_i}, so for kappa = C(u) f
//     fbar = C(u)^T kappabar,  ubar_i -= sum_m kappabar_m m_i kappa_{m - e_i};
//   for f~ = C(u)^-1 kappa~ (C(u) f~ = kappa~):
//     kappa~bar = C(u)^-T f~bar,  ubar_i += sum_m kappa~bar_m m_i kappa~_{m - e_i}.
// C(u)^T and C(u)^-T are applied as the transposed 1D maps in reverse pass order.
#pragma once

#include "fpc_collide.h"

namespace fpc {
namespace adj {

// Moment / population work space of the tensor-product lattice (3^D entries):
// entry (a, b, c) with a, b, c in {0, 1, 2} is either the link (a-1, b-1, c-1)
// or the central moment with exponents (a, b, c).
template <int D>
struct MS {
  static constexpr int NM = D == 2 ? 9 : 27;
  static constexpr int at(int a, int b, int c) { return D == 2 ? a * 3 + b : a * 9 + b * 3 + c; }
  static constexpr int ma(int i) { return D == 2 ? i / 3 : i / 9; }
  static constexpr int mb(int i) { return D == 2 ? i % 3 : (i / 3) % 3; }
  static constexpr int mc(int i) { return D == 2 ? 0 : i % 3; }
  static constexpr int m(int i, int ax) { return ax == 0 ? ma(i) : (ax == 1 ? mb(i) : mc(i)); }
  static constexpr int order(int i) { return ma(i) + mb(i) + mc(i); }
  // index of the moment m - e_ax (caller guarantees m_ax > 0)
  static constexpr int down(int i, int ax) {
    return at(ma(i) - (ax == 0), mb(i) - (ax == 1), mc(i) - (ax == 2));
  }
  // population index (paper order) of entry i read as a link
  static constexpr int pop(int i) {
    return D == 2 ? d2_index(ma(i) - 1, mb(i) - 1) : d3_index(ma(i) - 1, mb(i) - 1, mc(i) - 1);
  }
  // relaxation-rate slot of moment i (paper order of the moment vector; the
  // diagonal second-order slots hold the rates of their combinations)
  static constexpr int slot(int i) {
    if (D == 2) {
      constexpr int s2[9] = {0, 2, 4, 1, 5, 7, 3, 6, 8};  // at(a,b) -> slot
      return s2[i];
    }
    constexpr int list[27][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
                                 {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 2, 0}, {1, 0, 2}, {2, 1, 0}, {0, 1, 2},
                                 {2, 0, 1}, {0, 2, 1}, {1, 1, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1},
                                 {1, 2, 1}, {1, 1, 2}, {1, 2, 2}, {2, 1, 2}, {2, 2, 1}, {2, 2, 2}};
    for (int k = 0; k < 27; ++k)
      if (list[k][0] == ma(i) && list[k][1] == mb(i) && list[k][2] == mc(i)) return k;
    return -1;
  }
};

// Slots whose rate is the compile-time 1 of the standard rate set (STD): the
// moment lands on its attractor (plus half its source), so its pre-collision
// value drops out of the forward map and of its adjoint.
template <int D, bool STD>
__device__ __forceinline__ constexpr bool unit_f(int slot) {
  return STD && !viscous_slot<D>(slot);
}
template <int D, bool STD>
__device__ __forceinline__ constexpr bool unit_g(int k) {
  return STD && !(k >= 1 && k <= D);
}

// Transposed 1D maps.  S(u): (a-, a0, a+) -> (k0, k1, k2) is shift_fwd.
template <class R>
__device__ __forceinline__ void shift_fwd_T(R k0, R k1, R k2, R u, R& am, R& a0, R& ap) {
  am = k0 + (R(-1) - u) * k1 + (R(1) + u) * (R(1) + u) * k2;
  a0 = k0 - u * k1 + u * u * k2;
  ap = k0 + (R(1) - u) * k1 + (R(1) - u) * (R(1) - u) * k2;
}
// S(u)^-1: (k0, k1, k2) -> (a-, a0, a+) is shift_inv; its transpose maps
// (a-bar, a0bar, a+bar) -> (k0bar, k1bar, k2bar).
template <class R>
__device__ __forceinline__ void shift_inv_T(R am, R a0, R ap, R u, R& k0, R& k1, R& k2) {
  k0 = (R(1) - u * u) * a0 + R(0.5) * (u * u + u) * ap + R(0.5) * (u * u - u) * am;
  k1 = R(-2) * u * a0 + R(0.5) * (R(2) * u + R(1)) * ap + R(0.5) * (R(2) * u - R(1)) * am;
  k2 = -a0 + R(0.5) * ap + R(0.5) * am;
}

// Apply C(u) (mode 0), C(u)^-1 (mode 1), C(u)^T (mode 2) or C(u)^-T (mode 3)
// in place to a work array of the tensor-product lattice.
template <class R, int D, int MODE>
__device__ __forceinline__ void apply(R (&w)[MS<D>::NM], const R (&u)[3]) {
  using M = MS<D>;
  auto pass = [&](int ax) {
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < (D == 2 ? 1 : 3); ++q) {
        int i0, i1, i2;
        if (D == 2) {
          i0 = ax == 0 ? M::at(0, p, 0) : M::at(p, 0, 0);
          i1 = ax == 0 ? M::at(1, p, 0) : M::at(p, 1, 0);
          i2 = ax == 0 ? M::at(2, p, 0) : M::at(p, 2, 0);
        } else {
          i0 = ax == 0 ? M::at(0, p, q) : (ax == 1 ? M::at(p, 0, q) : M::at(p, q, 0));
          i1 = ax == 0 ? M::at(1, p, q) : (ax == 1 ? M::at(p, 1, q) : M::at(p, q, 1));
          i2 = ax == 0 ? M::at(2, p, q) : (ax == 1 ? M::at(p, 2, q) : M::at(p, q, 2));
        }
        const R a = w[i0], b = w[i1], c = w[i2];
        if (MODE == 0) shift_fwd(a, b, c, u[ax], w[i0], w[i1], w[i2]);
        if (MODE == 1) shift_inv(a, b, c, u[ax], w[i0], w[i1], w[i2]);
        if (MODE == 2) shift_fwd_T(a, b, c, u[ax], w[i0], w[i1], w[i2]);
        if (MODE == 3) shift_inv_T(a, b, c, u[ax], w[i0], w[i1], w[i2]);
      }
  };
  // C = Z Y X (x pass first); C^-1 = X^-1 Y^-1 Z^-1 (z pass first);
  // C^T = X^T Y^T Z^T (z pass first); C^-T = Z^-T Y^-T X^-T (x pass first).
  if (MODE == 0 || MODE == 3) {
    pass(0);
    pass(1);
    if (D == 3) pass(2);
  } else {
    if (D == 3) pass(2);
    pass(1);
    pass(0);
  }
}

// Attractor terms of the recurrence (Eq. Mvcmattractor2D / 3D) for moment i of
// order s >= 3 with D'_ab = kappa~_ab / rho: Mv_i = sum_t c_t kt[A_t] kt[B_t] / (s rho)
// over t = (axis pair), A_t the second-order moment, B_t = i - A_t; terms whose
// B_t has order 1 vanish (first-order moments taken as zero).
template <int D>
struct Terms {
  using M = MS<D>;
  // enumerate: t in [0, D*(D+1)/2): (i, i) then (i, j) i < j
  static constexpr int npairs = D == 2 ? 3 : 6;
  static constexpr int axA(int t) { return D == 2 ? (t == 0 ? 0 : (t == 1 ? 1 : 0)) : (t < 3 ? t : (t == 3 ? 0 : (t == 4 ? 0 : 1))); }
  static constexpr int axB(int t) { return D == 2 ? (t == 0 ? 0 : (t == 1 ? 1 : 1)) : (t < 3 ? t : (t == 3 ? 1 : 2)); }
  static constexpr int coef(int i, int t) {
    const int a = axA(t), b = axB(t);
    return a == b ? M::m(i, a) * (M::m(i, a) - 1) : 2 * M::m(i, a) * M::m(i, b);
  }
  static constexpr int A(int t) {
    const int a = axA(t), b = axB(t);
    return M::at((a == 0) + (b == 0), (a == 1) + (b == 1), (a == 2) + (b == 2));
  }
  static constexpr bool valid(int i, int t) {
    if (coef(i, t) == 0) return false;
    const int a = axA(t), b = axB(t);
    const int ra = M::m(i, 0) - (a == 0) - (b == 0), rb = M::m(i, 1) - (a == 1) - (b == 1),
              rc = M::m(i, 2) - (a == 2) - (b == 2);
    return ra >= 0 && rb >= 0 && rc >= 0 && ra + rb + rc != 1;
  }
  static constexpr int B(int i, int t) {
    const int a = axA(t), b = axB(t);
    return M::at(M::m(i, 0) - (a == 0) - (b == 0), M::m(i, 1) - (a == 1) - (b == 1), M::m(i, 2) - (a == 2) - (b == 2));
  }
};

// Maxwellian central moment of exponents m over rho (the MCM comparator's
// attractor, Sec. 7): prod_d c(m_d) with c(0) = 1, c(1) = 0, c(2) = c_s^2.
template <int D>
__device__ constexpr double maxwell_cm(int i) {
  double v = 1.0;
  for (int ax = 0; ax < D; ++ax) {
    const int m = MS<D>::m(i, ax);
    v *= m == 0 ? 1.0 : (m == 1 ? 0.0 : 1.0 / 3.0);
  }
  return v;
}

// Forward collision on plain populations with everything the reverse needs.
// QG: thermal lattice, 2D + 1 (D2Q5 / D3Q7), 9 (the paper's D2Q9, whose
// moments use the work layout of MS<2>) or 15 (the paper's D3Q15, moments in
// the order of t15::kM).
template <class R, int D, int QG = 2 * D + 1>
struct Tape {
  static constexpr int NM = MS<D>::NM;
  // D3Q15: the 15 moments of the set and, last, the central moment 210
  static constexpr int NG = QG == kQ15 ? QG + 1 : QG;
  R rho, ir, T, Fb, u[3];  // ir = 1 / rho
  R k[NM];   // pre-collision central moments
  R kt[NM];  // post-collision central moments
  R e[NG];   // thermal central moments (D2Q5 / D3Q7: 0, +-axis order 1, order 2 per axis)
  R et[NG];  // post-collision thermal central moments
};

// ---- the paper's D3Q15 thermal lattice (App. C) ----
// Raw moments r = H g (H[m][q] = prod_d e_qd^m_d over the moment set) and
// central moments e = S(u) r, S unit lower triangular in the set's order
// (binomial shift about u, raw moments aliased into the set).  For the
// reverse, H^T, H^-T and S(u)^T, S(u)^-T; H^-1 is inverted at compile time.
namespace q15 {
struct Mat {
  double a[kQ15][kQ15];
};
constexpr int ipow(int e, int m) { return m == 0 ? 1 : (m == 1 ? e : e * e); }
constexpr Mat raw_matrix() {
  Mat H{};
  for (int m = 0; m < kQ15; ++m)
    for (int q = 0; q < kQ15; ++q)
      H.a[m][q] = ipow(T15_EX[q], t15::kM[m][0]) * ipow(T15_EY[q], t15::kM[m][1]) * ipow(T15_EZ[q], t15::kM[m][2]);
  return H;
}
constexpr double cabs(double v) { return v < 0 ? -v : v; }
// Gauss-Jordan elimination with partial pivoting (H is an invertible integer matrix)
constexpr Mat inverse(Mat A) {
  Mat I{};
  for (int i = 0; i < kQ15; ++i) I.a[i][i] = 1.0;
  for (int c = 0; c < kQ15; ++c) {
    int p = c;
    for (int r = c + 1; r < kQ15; ++r)
      if (cabs(A.a[r][c]) > cabs(A.a[p][c])) p = r;
    for (int j = 0; j < kQ15; ++j) {
      const double ta = A.a[c][j], ti = I.a[c][j];
      A.a[c][j] = A.a[p][j];
      I.a[c][j] = I.a[p][j];
      A.a[p][j] = ta;
      I.a[p][j] = ti;
    }
    const double d = A.a[c][c];
    for (int j = 0; j < kQ15; ++j) {
      A.a[c][j] /= d;
      I.a[c][j] /= d;
    }
    for (int r = 0; r < kQ15; ++r) {
      if (r == c) continue;
      const double f = A.a[r][c];
      if (f == 0.0) continue;
      for (int j = 0; j < kQ15; ++j) {
        A.a[r][j] -= f * A.a[c][j];
        I.a[r][j] -= f * I.a[c][j];
      }
    }
  }
  return I;
}
struct Tables {
  static constexpr Mat H = raw_matrix();
  static constexpr Mat Hi = inverse(raw_matrix());
};
// index in the set of the exponents (a, b, c), or kQ15 for (2, 1, 0) (the
// only m - e_d of a member that is not a member), -1 otherwise
constexpr int index_of(int a, int b, int c) {
  for (int k = 0; k < kQ15; ++k)
    if (t15::kM[k][0] == a && t15::kM[k][1] == b && t15::kM[k][2] == c) return k;
  return (a == 2 && b == 1 && c == 0) ? kQ15 : -1;
}
constexpr int m(int k, int ax) { return k == kQ15 ? (ax == 0 ? 2 : (ax == 1 ? 1 : 0)) : t15::kM[k][ax]; }
constexpr int down(int k, int ax) {
  return index_of(m(k, 0) - (ax == 0), m(k, 1) - (ax == 1), m(k, 2) - (ax == 2));
}
// central moment (MX, MY, MZ) from raw moments r (the self term left out when SKIP_SELF)
template <class R, int MX, int MY, int MZ, bool SKIP_SELF>
__device__ __forceinline__ R shift(const R (&r)[kQ15], const R (&nux)[3], const R (&nuy)[3], const R (&nuz)[3]) {
  R acc = R(0);
#pragma unroll
  for (int i = 0; i <= MX; ++i)
#pragma unroll
    for (int j = 0; j <= MY; ++j)
#pragma unroll
      for (int k = 0; k <= MZ; ++k) {
        if (SKIP_SELF && i == MX && j == MY && k == MZ) continue;
        acc += R(t15::binom(MX, i) * t15::binom(MY, j) * t15::binom(MZ, k)) * nux[MX - i] * nuy[MY - j] *
               nuz[MZ - k] * r[t15::alias(i, j, k)];
      }
  return acc;
}
// rb += (row (MX, MY, MZ) of S, the self term left out when SKIP_SELF)^T v
template <class R, int MX, int MY, int MZ, bool SKIP_SELF>
__device__ __forceinline__ void shift_T(R (&rb)[kQ15], R v, const R (&nux)[3], const R (&nuy)[3],
                                        const R (&nuz)[3]) {
#pragma unroll
  for (int i = 0; i <= MX; ++i)
#pragma unroll
    for (int j = 0; j <= MY; ++j)
#pragma unroll
      for (int k = 0; k <= MZ; ++k) {
        if (SKIP_SELF && i == MX && j == MY && k == MZ) continue;
        rb[t15::alias(i, j, k)] += R(t15::binom(MX, i) * t15::binom(MY, j) * t15::binom(MZ, k)) * nux[MX - i] *
                                   nuy[MY - j] * nuz[MZ - k] * v;
      }
}
}  // namespace q15

#define FPC_Q15_SET(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#define FPC_Q15_SET_DESC(X) X(14) X(13) X(12) X(11) X(10) X(9) X(8) X(7) X(6) X(5) X(4) X(3) X(2) X(1)
#define FPC_Q15_M(K) t15::kM[K][0], t15::kM[K][1], t15::kM[K][2]

// Thermal attractors of the paper's D3Q15 lattice above second order
// (120, 012, 201, 111, 220), from the post-collision moments up to second
// order and T: option A, option B, MCM (as in fpc_collide.h).
template <class R, bool STD>
__device__ __forceinline__ void thermal15_attractors(const CollParams<R>& c, R T, const R* et, R (&mv)[5]) {
  const R cT = c.cs2T;
  if (mcm<STD>(c)) {
    mv[0] = mv[1] = mv[2] = mv[3] = R(0);
    mv[4] = cT * cT * T;
  } else if (option_b<STD>(c)) {
    const R f = R(2) / (R(3) * T);
    mv[0] = f * (et[8] * et[1] + R(2) * et[4] * et[2]);
    mv[1] = f * (et[9] * et[2] + R(2) * et[6] * et[3]);
    mv[2] = f * (et[7] * et[3] + R(2) * et[5] * et[1]);
    mv[3] = f * (et[4] * et[3] + et[5] * et[2] + et[6] * et[1]);
    mv[4] = (et[7] * et[8] + R(2) * et[4] * et[4]) / T;
  } else {
    mv[0] = R(2) / R(3) * cT * et[1];
    mv[1] = R(2) / R(3) * cT * et[2];
    mv[2] = R(2) / R(3) * cT * et[3];
    mv[3] = R(0);
    mv[4] = R(0.5) * cT * (et[7] + et[8]);
  }
}

// Thermal attractors of the paper's D2Q9 lattice above second order
// (Eq. Mvcmattractor2D_g): option A (c^_s^2 I at every order), option B
// (post-collision second order over T), MCM (T prod c(m_d)); et holds the
// post-collision moments up to second order (work layout of MS<2>).
template <class R, bool STD>
__device__ __forceinline__ void thermal9_attractors(const CollParams<R>& c, R T, const R (&et)[9], R& m21, R& m12,
                                                    R& m22) {
  using M = MS<2>;
  constexpr int i10 = M::at(1, 0, 0), i01 = M::at(0, 1, 0), i20 = M::at(2, 0, 0), i02 = M::at(0, 2, 0),
                i11 = M::at(1, 1, 0);
  const R cT = c.cs2T;
  if (mcm<STD>(c)) {
    m21 = R(0);
    m12 = R(0);
    m22 = cT * cT * T;
  } else if (option_b<STD>(c)) {
    const R iT = R(1) / T;
    m21 = R(2) / R(3) * iT * (et[i20] * et[i01] + R(2) * et[i11] * et[i10]);
    m12 = R(2) / R(3) * iT * (et[i02] * et[i10] + R(2) * et[i11] * et[i01]);
    m22 = iT * (et[i20] * et[i02] + R(2) * et[i11] * et[i11]);
  } else {
    m21 = R(2) / R(3) * cT * et[i01];
    m12 = R(2) / R(3) * cT * et[i10];
    m22 = R(0.5) * cT * (et[i20] + et[i02]);
  }
}

// Thermal moment layout (D2Q5 / D3Q7): e[0] = eta_0, e[1+ax] = eta_{e_ax},
// e[1+D+ax] = eta_{2 e_ax}.  Populations: g[0] rest, g[1+2ax] = +ax link,
// g[2+2ax] = -ax link (this is the D3Q7 order; for D2Q5 the paper order
// 0, +x, +y, -x, -y is mapped by tlink()).
template <int D>
__device__ constexpr int tlink(int ax, int sgn) {
  return D == 2 ? (sgn > 0 ? 1 + ax : 3 + ax) : (sgn > 0 ? 1 + 2 * ax : 2 + 2 * ax);
}

template <class R, int D, int UP, bool STD = false, int QG = 2 * D + 1>
__device__ __forceinline__ void forward(const R* f, const R* g, const CollParams<R>& c, Tape<R, D, QG>& t) {
  using M = MS<D>;
  constexpr int NM = M::NM;
  constexpr R cs2 = R(1) / R(3);
  // (each sum starts from its first term: an explicit 0 + x, or 0 * x below,
  // would cost an IEEE operation that cannot be dropped)
  R rho = f[M::pop(0)], j[3] = {R(0), R(0), R(0)};
  bool hj[3] = {false, false, false};
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    const R v = f[M::pop(i)];
    if (i > 0) rho += v;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      const int m = M::m(i, ax);
      if (m == 1) continue;
      j[ax] = hj[ax] ? (m == 2 ? j[ax] + v : j[ax] - v) : (m == 2 ? v : -v);
      hj[ax] = true;
    }
  }
  R T = g[0];
#pragma unroll
  for (int q = 1; q < QG; ++q) T += g[q];
  const R Fb = c.gbeta * (T - c.T0);
  const R ir = R(1) / rho;
  t.rho = rho;
  t.ir = ir;
  t.T = T;
  t.Fb = Fb;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) t.u[ax] = ax < D ? (j[ax] + (ax == UP ? R(0.5) * Fb : R(0))) * ir : R(0);
#pragma unroll
  for (int i = 0; i < NM; ++i) t.k[i] = f[M::pop(i)];
  apply<R, D, 0>(t.k, t.u);
  // relaxation, order by order
  const R* om = c.om;
  const R Fr = Fb * ir;
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    const int s = M::order(i);
    if (s == 0) t.kt[i] = rho;
    if (s == 1) {
      const int ax = M::ma(i) ? 0 : (M::mb(i) ? 1 : 2);
      const R Fa = ax == UP ? Fb : R(0);
      if (unit_f<D, STD>(M::slot(i))) {
        t.kt[i] = R(0.5) * Fa;
      } else {
        const R w = om[M::slot(i)];
        t.kt[i] = t.k[i] - w * t.k[i];
        if (ax == UP) t.kt[i] += (R(1) - R(0.5) * w) * Fa;
      }
    }
    if (s == 2 && (M::ma(i) == 1 || M::mb(i) == 1 || M::mc(i) == 1))
      t.kt[i] = unit_f<D, STD>(M::slot(i)) ? R(0) : (R(1) - om[M::slot(i)]) * t.k[i];
  }
  // diagonal second order as combinations (trace / deviators in 3D, 2s / 2d in 2D)
  if (D == 2) {
    const int a = M::at(2, 0, 0), b = M::at(0, 2, 0);
    const R s2 = t.k[a] + t.k[b], d2 = t.k[a] - t.k[b];
    const R ts = unit_f<D, STD>(3) ? R(2) * cs2 * rho : s2 + om[3] * (R(2) * cs2 * rho - s2);
    const R td = unit_f<D, STD>(4) ? R(0) : d2 - om[4] * d2;
    t.kt[a] = R(0.5) * (ts + td);
    t.kt[b] = R(0.5) * (ts - td);
  } else {
    const int a = M::at(2, 0, 0), b = M::at(0, 2, 0), cc = M::at(0, 0, 2);
    const R tr = t.k[a] + t.k[b] + t.k[cc], d1 = t.k[a] - t.k[b], d2 = t.k[a] - t.k[cc];
    const R ttr = unit_f<D, STD>(7) ? R(3) * cs2 * rho : tr + om[7] * (R(3) * cs2 * rho - tr);
    const R t1 = unit_f<D, STD>(8) ? R(0) : d1 - om[8] * d1;
    const R t2 = unit_f<D, STD>(9) ? R(0) : d2 - om[9] * d2;
    const R t200 = (ttr + t1 + t2) * (R(1) / R(3));
    t.kt[a] = t200;
    t.kt[b] = t200 - t1;
    t.kt[cc] = t200 - t2;
  }
  // orders >= 3
#pragma unroll
  for (int s = 3; s <= 2 * D; ++s) {
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      if (M::order(i) != s) continue;
      R mv = R(0);
      if (mcm<STD>(c)) {
        mv = R(maxwell_cm<D>(i)) * rho;
      } else {
#pragma unroll
        for (int p = 0; p < Terms<D>::npairs; ++p)
          if (Terms<D>::valid(i, p)) mv += R(Terms<D>::coef(i, p)) * t.kt[Terms<D>::A(p)] * t.kt[Terms<D>::B(i, p)];
        mv = mv * (ir * (R(1) / R(s)));
      }
      R sig = R(0);
      const int mu = M::m(i, UP);
      if (mu > 0 && M::order(M::down(i, UP)) >= 2) sig = R(mu) * Fr * t.k[M::down(i, UP)];
      if (unit_f<D, STD>(M::slot(i))) {
        t.kt[i] = mv + R(0.5) * sig;
      } else {
        const R w = om[M::slot(i)];
        t.kt[i] = t.k[i] + w * (mv - t.k[i]) + (R(1) - R(0.5) * w) * sig;
      }
    }
  }
  if constexpr (QG == kQ15) {
    // thermal D3Q15: raw moments, central moments by the aliased binomial
    // shift, relaxation of App. C Step 3; the post-collision raw moments
    // (inverse of the shift) give kappa~_210 for the reverse
    static_assert(D == 3, "D3Q15 is a 3D lattice");
    R r[kQ15];
#pragma unroll
    for (int mm = 0; mm < kQ15; ++mm) {
      R v = R(0);
#pragma unroll
      for (int q = 0; q < kQ15; ++q)
        if (q15::Tables::H.a[mm][q] != 0.0) v += R(q15::Tables::H.a[mm][q]) * g[q];
      r[mm] = v;
    }
    const R nux[3] = {R(1), -t.u[0], t.u[0] * t.u[0]}, nuy[3] = {R(1), -t.u[1], t.u[1] * t.u[1]},
            nuz[3] = {R(1), -t.u[2], t.u[2] * t.u[2]};
    t.e[0] = T;
#define FPC_E15(K) t.e[K] = q15::shift<R, FPC_Q15_M(K), false>(r, nux, nuy, nuz);
    FPC_Q15_SET(FPC_E15)
#undef FPC_E15
    t.e[kQ15] = q15::shift<R, 2, 1, 0, false>(r, nux, nuy, nuz);
    auto og = [&](int k) -> R { return rate_g<3, STD>(c, k); };
    const R cT = c.cs2T;
    t.et[0] = T;
#pragma unroll
    for (int k = 1; k <= 6; ++k) t.et[k] = (R(1) - og(k)) * t.e[k];
#pragma unroll
    for (int k = 7; k <= 9; ++k) t.et[k] = t.e[k] + og(k) * (cT * T - t.e[k]);
    R mv[5];
    thermal15_attractors<R, STD>(c, T, t.et, mv);
#pragma unroll
    for (int k = 10; k <= 14; ++k) t.et[k] = t.e[k] + og(k) * (mv[k - 10] - t.e[k]);
    R rt[kQ15];
    rt[0] = t.et[0];
#define FPC_R15(K) rt[K] = t.et[K] - q15::shift<R, FPC_Q15_M(K), true>(rt, nux, nuy, nuz);
    FPC_Q15_SET(FPC_R15)
#undef FPC_R15
    t.et[kQ15] = q15::shift<R, 2, 1, 0, false>(rt, nux, nuy, nuz);
    return;
  } else if constexpr (QG != 2 * D + 1) {
    // thermal D2Q9: the same tensor-product shifts as the fluid, then the
    // relaxation of the paper's D2Q9 thermal collision (App. B Step 3)
    static_assert(D == 2 && QG == kQ2, "thermal D2Q9 only");
    constexpr int i00 = M::at(0, 0, 0), i10 = M::at(1, 0, 0), i01 = M::at(0, 1, 0), i20 = M::at(2, 0, 0),
                  i02 = M::at(0, 2, 0), i11 = M::at(1, 1, 0), i21 = M::at(2, 1, 0), i12 = M::at(1, 2, 0),
                  i22 = M::at(2, 2, 0);
#pragma unroll
    for (int i = 0; i < QG; ++i) t.e[i] = g[M::pop(i)];
    apply<R, 2, 0>(t.e, t.u);
    auto og = [&](int k) -> R { return rate_g<2, STD>(c, k); };
    const R cT = c.cs2T;
    t.et[i00] = T;
    t.et[i10] = (R(1) - og(1)) * t.e[i10];
    t.et[i01] = (R(1) - og(2)) * t.e[i01];
    const R s2 = t.e[i20] + t.e[i02], d2 = t.e[i20] - t.e[i02];
    const R ts = s2 + og(3) * (R(2) * cT * T - s2), td = (R(1) - og(4)) * d2;
    t.et[i20] = R(0.5) * (ts + td);
    t.et[i02] = R(0.5) * (ts - td);
    t.et[i11] = (R(1) - og(5)) * t.e[i11];
    R m21, m12, m22;
    thermal9_attractors<R, STD>(c, T, t.et, m21, m12, m22);
    t.et[i21] = t.e[i21] + og(6) * (m21 - t.e[i21]);
    t.et[i12] = t.e[i12] + og(7) * (m12 - t.e[i12]);
    t.et[i22] = t.e[i22] + og(8) * (m22 - t.e[i22]);
    return;
  } else {
  // thermal: raw -> central
  R n[2 * D + 1];
  n[0] = T;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    const R gp = g[tlink<D>(ax, 1)], gm = g[tlink<D>(ax, -1)];
    n[1 + ax] = gp - gm;
    n[1 + D + ax] = gp + gm;
  }
  t.e[0] = T;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    t.e[1 + ax] = n[1 + ax] - t.u[ax] * T;
    t.e[1 + D + ax] = n[1 + D + ax] - R(2) * t.u[ax] * n[1 + ax] + t.u[ax] * t.u[ax] * T;
  }
  const R* og = c.omg;
  t.et[0] = T;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) t.et[1 + ax] = (R(1) - og[1 + ax]) * t.e[1 + ax];
  if (D == 2) {
    const R s2 = t.e[3] + t.e[4], d2 = t.e[3] - t.e[4];
    const R ts = unit_g<D, STD>(3) ? R(2) * c.cs2T * T : s2 + og[3] * (R(2) * c.cs2T * T - s2);
    const R td = unit_g<D, STD>(4) ? R(0) : d2 - og[4] * d2;
    t.et[3] = R(0.5) * (ts + td);
    t.et[4] = R(0.5) * (ts - td);
  } else {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
      t.et[4 + ax] = unit_g<D, STD>(4 + ax) ? c.cs2T * T : t.e[4 + ax] + og[4 + ax] * (c.cs2T * T - t.e[4 + ax]);
  }
  }
}

// Reverse of forward(): given fb (= f~bar) and gb (= g~bar) on the post-collision
// populations, overwrite them with the adjoints of the pre-collision ones.
template <class R, int D, int UP, bool STD = false, int QG = 2 * D + 1>
__device__ __forceinline__ void reverse(const Tape<R, D, QG>& t, const CollParams<R>& c, R* fb, R* gb) {
  using M = MS<D>;
  constexpr int NM = M::NM;
  constexpr R cs2 = R(1) / R(3);
  R ub[3] = {R(0), R(0), R(0)};
  R rhob = R(0), Fbb = R(0), Tb = R(0);
  const R* og = c.omg;

  // ---- thermal: g~ = P_g^-1 F_g(u)^-1 eta~ ----
  if constexpr (QG == kQ15) {
    // thermal D3Q15: g~ = H^-1 S(u)^-1 eta~, eta = S(u) H g
    auto og = [&](int k) -> R { return rate_g<3, STD>(c, k); };
    const R cT = c.cs2T;
    const R nux[3] = {R(1), -t.u[0], t.u[0] * t.u[0]}, nuy[3] = {R(1), -t.u[1], t.u[1] * t.u[1]},
            nuz[3] = {R(1), -t.u[2], t.u[2] * t.u[2]};
    R tb[kQ15];  // H^-T g~bar, then S^-T of it: the adjoint of eta~
#pragma unroll
    for (int mm = 0; mm < kQ15; ++mm) {
      R v = R(0);
#pragma unroll
      for (int q = 0; q < kQ15; ++q)
        if (q15::Tables::Hi.a[q][mm] != 0.0) v += R(q15::Tables::Hi.a[q][mm]) * gb[q];
      tb[mm] = v;
    }
#define FPC_TB15(K) q15::shift_T<R, FPC_Q15_M(K), true>(tb, -tb[K], nux, nuy, nuz);
    FPC_Q15_SET_DESC(FPC_TB15)
#undef FPC_TB15
#pragma unroll
    for (int k = 1; k < kQ15; ++k)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        if (q15::m(k, ax) > 0) ub[ax] += tb[k] * R(q15::m(k, ax)) * t.et[q15::down(k, ax)];
    // relaxation, highest orders first
    R eb[kQ15];
    R mb[5];
#pragma unroll
    for (int k = 10; k <= 14; ++k) {
      eb[k] = (R(1) - og(k)) * tb[k];
      mb[k - 10] = og(k) * tb[k];
    }
    const R* et = t.et;
    if (mcm<STD>(c)) {
      Tb += cT * cT * mb[4];
    } else if (option_b<STD>(c)) {
      const R iT = R(1) / t.T, f = R(2) / R(3) * iT;
      R mv[5];
      thermal15_attractors<R, STD>(c, t.T, t.et, mv);
      // m120 = f (et8 et1 + 2 et4 et2)
      tb[8] += f * et[1] * mb[0];
      tb[1] += f * et[8] * mb[0];
      tb[4] += R(2) * f * et[2] * mb[0];
      tb[2] += R(2) * f * et[4] * mb[0];
      // m012 = f (et9 et2 + 2 et6 et3)
      tb[9] += f * et[2] * mb[1];
      tb[2] += f * et[9] * mb[1];
      tb[6] += R(2) * f * et[3] * mb[1];
      tb[3] += R(2) * f * et[6] * mb[1];
      // m201 = f (et7 et3 + 2 et5 et1)
      tb[7] += f * et[3] * mb[2];
      tb[3] += f * et[7] * mb[2];
      tb[5] += R(2) * f * et[1] * mb[2];
      tb[1] += R(2) * f * et[5] * mb[2];
      // m111 = f (et4 et3 + et5 et2 + et6 et1)
      tb[4] += f * et[3] * mb[3];
      tb[3] += f * et[4] * mb[3];
      tb[5] += f * et[2] * mb[3];
      tb[2] += f * et[5] * mb[3];
      tb[6] += f * et[1] * mb[3];
      tb[1] += f * et[6] * mb[3];
      // m220 = (et7 et8 + 2 et4^2) / T
      tb[7] += iT * et[8] * mb[4];
      tb[8] += iT * et[7] * mb[4];
      tb[4] += R(4) * iT * et[4] * mb[4];
      Tb -= iT * (mv[0] * mb[0] + mv[1] * mb[1] + mv[2] * mb[2] + mv[3] * mb[3] + mv[4] * mb[4]);
    } else {
      tb[1] += R(2) / R(3) * cT * mb[0];
      tb[2] += R(2) / R(3) * cT * mb[1];
      tb[3] += R(2) / R(3) * cT * mb[2];
      tb[7] += R(0.5) * cT * mb[4];
      tb[8] += R(0.5) * cT * mb[4];
    }
#pragma unroll
    for (int k = 7; k <= 9; ++k) {
      eb[k] = (R(1) - og(k)) * tb[k];
      Tb += og(k) * cT * tb[k];
    }
#pragma unroll
    for (int k = 1; k <= 6; ++k) eb[k] = (R(1) - og(k)) * tb[k];
    Tb += tb[0];
    eb[0] = R(0);
    // eta = S(u) r: ubar -= sum eb_m m_d eta_{m - e_d}; rbar = S^T eb; gbar = H^T rbar
#pragma unroll
    for (int k = 1; k < kQ15; ++k)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        if (q15::m(k, ax) > 0) ub[ax] -= eb[k] * R(q15::m(k, ax)) * t.e[q15::down(k, ax)];
    R rb[kQ15];
#pragma unroll
    for (int k = 0; k < kQ15; ++k) rb[k] = R(0);
#define FPC_RB15(K) q15::shift_T<R, FPC_Q15_M(K), false>(rb, eb[K], nux, nuy, nuz);
    FPC_Q15_SET(FPC_RB15)
#undef FPC_RB15
#pragma unroll
    for (int q = 0; q < kQ15; ++q) {
      R v = R(0);
#pragma unroll
      for (int mm = 0; mm < kQ15; ++mm)
        if (q15::Tables::H.a[mm][q] != 0.0) v += R(q15::Tables::H.a[mm][q]) * rb[mm];
      gb[q] = v;
    }
  } else if constexpr (QG != 2 * D + 1) {
    // thermal D2Q9: g~ = C(u)^-1 eta~, eta = C(u) g (tensor-product shifts)
    constexpr int i00 = M::at(0, 0, 0), i10 = M::at(1, 0, 0), i01 = M::at(0, 1, 0), i20 = M::at(2, 0, 0),
                  i02 = M::at(0, 2, 0), i11 = M::at(1, 1, 0), i21 = M::at(2, 1, 0), i12 = M::at(1, 2, 0),
                  i22 = M::at(2, 2, 0);
    auto og = [&](int k) -> R { return rate_g<2, STD>(c, k); };
    const R cT = c.cs2T;
    R tb[QG];  // adjoint of the post-collision thermal moments
#pragma unroll
    for (int i = 0; i < QG; ++i) tb[i] = gb[M::pop(i)];
    apply<R, 2, 3>(tb, t.u);
#pragma unroll
    for (int i = 0; i < QG; ++i)
#pragma unroll
      for (int ax = 0; ax < 2; ++ax)
        if (M::m(i, ax) > 0) ub[ax] += tb[i] * R(M::m(i, ax)) * t.et[M::down(i, ax)];
    // orders 3-4: eta~_m = (1 - w) eta_m + w m_m, attractors from eta~ up to second order and T
    R eb[QG];
    eb[i22] = (R(1) - og(8)) * tb[i22];
    eb[i21] = (R(1) - og(6)) * tb[i21];
    eb[i12] = (R(1) - og(7)) * tb[i12];
    const R m22b = og(8) * tb[i22], m21b = og(6) * tb[i21], m12b = og(7) * tb[i12];
    if (mcm<STD>(c)) {
      Tb += cT * cT * m22b;
    } else if (option_b<STD>(c)) {
      const R iT = R(1) / t.T, f = R(2) / R(3) * iT;
      R m21, m12, m22;
      thermal9_attractors<R, STD>(c, t.T, t.et, m21, m12, m22);
      tb[i20] += iT * t.et[i02] * m22b + f * t.et[i01] * m21b;
      tb[i02] += iT * t.et[i20] * m22b + f * t.et[i10] * m12b;
      tb[i11] += R(4) * iT * t.et[i11] * m22b + R(2) * f * (t.et[i10] * m21b + t.et[i01] * m12b);
      tb[i01] += f * t.et[i20] * m21b + R(2) * f * t.et[i11] * m12b;
      tb[i10] += f * t.et[i02] * m12b + R(2) * f * t.et[i11] * m21b;
      Tb -= iT * (m22 * m22b + m21 * m21b + m12 * m12b);
    } else {
      tb[i20] += R(0.5) * cT * m22b;
      tb[i02] += R(0.5) * cT * m22b;
      tb[i01] += R(2) / R(3) * cT * m21b;
      tb[i10] += R(2) / R(3) * cT * m12b;
    }
    // second order: 11 toward 0; 2s toward 2 c^2 T; 2d toward 0
    eb[i11] = (R(1) - og(5)) * tb[i11];
    const R tsb = R(0.5) * (tb[i20] + tb[i02]), tdb = R(0.5) * (tb[i20] - tb[i02]);
    const R s2b = (R(1) - og(3)) * tsb, d2b = (R(1) - og(4)) * tdb;
    Tb += og(3) * R(2) * cT * tsb;
    eb[i20] = s2b + d2b;
    eb[i02] = s2b - d2b;
    // first order toward 0; eta~_0 = T
    eb[i10] = (R(1) - og(1)) * tb[i10];
    eb[i01] = (R(1) - og(2)) * tb[i01];
    Tb += tb[i00];
    eb[i00] = R(0);
    // eta = C(u) g: ubar_i -= sum_m etabar_m m_i eta_{m - e_i}; gbar = C^T etabar
#pragma unroll
    for (int i = 0; i < QG; ++i)
#pragma unroll
      for (int ax = 0; ax < 2; ++ax)
        if (M::m(i, ax) > 0) ub[ax] -= eb[i] * R(M::m(i, ax)) * t.e[M::down(i, ax)];
    apply<R, 2, 2>(eb, t.u);
#pragma unroll
    for (int i = 0; i < QG; ++i) gb[M::pop(i)] = eb[i];
  } else {
    R mb[2 * D + 1];  // adjoint of the post-collision raw moments
    R etb[2 * D + 1];
    // g~_0 = m0 - sum_ax m_{2ax};  g~_{+-ax} = (m_{2ax} +- m_{ax}) / 2
    mb[0] = gb[0];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      const R gp = gb[tlink<D>(ax, 1)], gm = gb[tlink<D>(ax, -1)];
      mb[1 + ax] = R(0.5) * (gp - gm);
      mb[1 + D + ax] = R(0.5) * (gp + gm) - gb[0];
    }
    // m_ax = et_ax + u_ax T ; m_2ax = et_2ax + 2 u_ax et_ax + u_ax^2 T ; m_0 = T
    etb[0] = mb[0];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      const R ua = t.u[ax];
      etb[1 + D + ax] = mb[1 + D + ax];
      etb[1 + ax] = mb[1 + ax] + R(2) * ua * mb[1 + D + ax];
      etb[0] += ua * mb[1 + ax] + ua * ua * mb[1 + D + ax];
      ub[ax] += t.T * mb[1 + ax] + (R(2) * t.et[1 + ax] + R(2) * ua * t.T) * mb[1 + D + ax];
    }
    // relaxation: et_0 = T; et_ax = (1 - w) e_ax; second order toward c^2 T
    R eb[2 * D + 1];
    Tb += etb[0];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) eb[1 + ax] = (R(1) - og[1 + ax]) * etb[1 + ax];
    if (D == 2) {
      const R tsb = R(0.5) * (etb[3] + etb[4]), tdb = R(0.5) * (etb[3] - etb[4]);
      const R s2b = unit_g<D, STD>(3) ? R(0) : (R(1) - og[3]) * tsb;
      const R d2b = unit_g<D, STD>(4) ? R(0) : (R(1) - og[4]) * tdb;
      Tb += (unit_g<D, STD>(3) ? R(2) * c.cs2T : og[3] * R(2) * c.cs2T) * tsb;
      eb[3] = s2b + d2b;
      eb[4] = s2b - d2b;
    } else {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        if (unit_g<D, STD>(4 + ax)) {
          eb[4 + ax] = R(0);
          Tb += c.cs2T * etb[4 + ax];
        } else {
          eb[4 + ax] = (R(1) - og[4 + ax]) * etb[4 + ax];
          Tb += og[4 + ax] * c.cs2T * etb[4 + ax];
        }
      }
    }
    // e_ax = n_ax - u_ax T ; e_2ax = n_2ax - 2 u_ax n_ax + u_ax^2 T ; e_0 = T
    R nb[2 * D + 1];
    nb[0] = R(0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      const R ua = t.u[ax];
      const R nax = t.e[1 + ax] + ua * t.T;  // n_ax
      nb[1 + D + ax] = eb[1 + D + ax];
      nb[1 + ax] = eb[1 + ax] - R(2) * ua * eb[1 + D + ax];
      Tb += -ua * eb[1 + ax] + ua * ua * eb[1 + D + ax];
      ub[ax] += -t.T * eb[1 + ax] + (R(-2) * nax + R(2) * ua * t.T) * eb[1 + D + ax];
    }
    // n_ax = g+ - g- ; n_2ax = g+ + g- ; T = sum g
    gb[0] = R(0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      gb[tlink<D>(ax, 1)] = nb[1 + ax] + nb[1 + D + ax];
      gb[tlink<D>(ax, -1)] = -nb[1 + ax] + nb[1 + D + ax];
    }
  }

  // ---- fluid: f~ = C(u)^-1 kappa~ ----
  R kb[NM];
#pragma unroll
  for (int i = 0; i < NM; ++i) kb[i] = fb[M::pop(i)];
  apply<R, D, 3>(kb, t.u);  // kappa~bar
#pragma unroll
  for (int i = 0; i < NM; ++i)
#pragma unroll
    for (int ax = 0; ax < D; ++ax)
      if (M::m(i, ax) > 0) ub[ax] += kb[i] * R(M::m(i, ax)) * t.kt[M::down(i, ax)];
  // relaxation reverse, highest order first; kb holds kappa~bar, kp the
  // adjoint of the pre-collision moments.  kappa = C(u) f adds
  // ubar_i -= kp_m m_i kappa_{m - e_i} once kp_m is final, i.e. right after
  // its order is done (sources only feed kp one order down), so the
  // pre-collision moments of each order die as soon as the next order up is
  // through.  Orders 0 and 1 of kappa are fixed by the macros: kappa_0 = rho,
  // kappa_{e_ax} = j_ax - rho u_ax = -F_ax / 2.
  R kp[NM];
#pragma unroll
  for (int i = 0; i < NM; ++i) kp[i] = R(0);
  const R* om = c.om;
  const R Fr = t.Fb * t.ir;
  auto kpre = [&](int j) -> R {
    const int s = M::order(j);
    if (s == 0) return t.rho;
    if (s == 1) return (M::m(j, UP) == 1) ? R(-0.5) * t.Fb : R(0);
    return t.k[j];
  };
  auto ub_from_kp = [&](int s) {
#pragma unroll
    for (int i = 0; i < NM; ++i)
      if (M::order(i) == s)
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
          if (M::m(i, ax) == 0) continue;
          const int dn = M::down(i, ax);
          if (M::order(dn) == 1 && M::m(dn, UP) != 1) continue;  // kappa_{e_ax} = 0 off the up axis
          ub[ax] -= kp[i] * R(M::m(i, ax)) * kpre(dn);
        }
  };
#pragma unroll
  for (int s = 2 * D; s >= 3; --s) {
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      if (M::order(i) != s) continue;
      const bool unit = unit_f<D, STD>(M::slot(i));
      const R w = unit ? R(1) : om[M::slot(i)];
      const R ktb = kb[i];
      if (!unit) kp[i] += (R(1) - w) * ktb;
      // attractor
      const R mvb = unit ? ktb : w * ktb;
      if (mcm<STD>(c)) {
        if (maxwell_cm<D>(i) != 0.0) rhob += mvb * R(maxwell_cm<D>(i));
      } else {
        const R irs = t.ir * (R(1) / R(s));
        R mv = R(0);
#pragma unroll
        for (int p = 0; p < Terms<D>::npairs; ++p)
          if (Terms<D>::valid(i, p)) {
            const int A = Terms<D>::A(p), B = Terms<D>::B(i, p);
            const R cf = R(Terms<D>::coef(i, p)) * irs;
            mv += cf * t.kt[A] * t.kt[B];
            kb[A] += mvb * cf * t.kt[B];
            kb[B] += mvb * cf * t.kt[A];
          }
        rhob -= mvb * mv * t.ir;
      }
      // source
      const int mu = M::m(i, UP);
      if (mu > 0 && M::order(M::down(i, UP)) >= 2) {
        const R sb = unit ? R(0.5) * ktb : (R(1) - R(0.5) * w) * ktb;
        const int p = M::down(i, UP);
        const R sig = R(mu) * Fr * t.k[p];
        Fbb += sb * R(mu) * t.k[p] * t.ir;
        kp[p] += sb * R(mu) * Fr;
        rhob -= sb * sig * t.ir;
      }
    }
    ub_from_kp(s);
  }
  // second order: off-diagonal
#pragma unroll
  for (int i = 0; i < NM; ++i)
    if (M::order(i) == 2 && (M::ma(i) == 1 || M::mb(i) == 1 || M::mc(i) == 1) && !unit_f<D, STD>(M::slot(i)))
      kp[i] += (R(1) - om[M::slot(i)]) * kb[i];
  // second order: diagonal combinations
  if (D == 2) {
    const int a = M::at(2, 0, 0), b = M::at(0, 2, 0);
    const R tsb = R(0.5) * (kb[a] + kb[b]), tdb = R(0.5) * (kb[a] - kb[b]);
    const R s2b = unit_f<D, STD>(3) ? R(0) : (R(1) - om[3]) * tsb;
    const R d2b = unit_f<D, STD>(4) ? R(0) : (R(1) - om[4]) * tdb;
    rhob += (unit_f<D, STD>(3) ? R(2) * cs2 : om[3] * R(2) * cs2) * tsb;
    kp[a] += s2b + d2b;
    kp[b] += s2b - d2b;
  } else {
    const int a = M::at(2, 0, 0), b = M::at(0, 2, 0), cc = M::at(0, 0, 2);
    const R third = R(1) / R(3);
    const R ttrb = (kb[a] + kb[b] + kb[cc]) * third;
    const R t1b = (kb[a] - R(2) * kb[b] + kb[cc]) * third;
    const R t2b = (kb[a] + kb[b] - R(2) * kb[cc]) * third;
    const R trb = unit_f<D, STD>(7) ? R(0) : (R(1) - om[7]) * ttrb;
    const R d1b = unit_f<D, STD>(8) ? R(0) : (R(1) - om[8]) * t1b;
    const R d2b = unit_f<D, STD>(9) ? R(0) : (R(1) - om[9]) * t2b;
    rhob += (unit_f<D, STD>(7) ? R(3) * cs2 : om[7] * R(3) * cs2) * ttrb;
    kp[a] += trb + d1b + d2b;
    kp[b] += trb - d1b;
    kp[cc] += trb - d2b;
  }
  ub_from_kp(2);
  // first order: kt = (1 - w) k + (1 - w/2) F
#pragma unroll
  for (int i = 0; i < NM; ++i)
    if (M::order(i) == 1) {
      const int ax = M::ma(i) ? 0 : (M::mb(i) ? 1 : 2);
      if (unit_f<D, STD>(M::slot(i))) {
        if (ax == UP) Fbb += R(0.5) * kb[i];
      } else {
        const R w = om[M::slot(i)];
        kp[i] += (R(1) - w) * kb[i];
        if (ax == UP) Fbb += (R(1) - R(0.5) * w) * kb[i];
      }
    }
  ub_from_kp(1);
  // zeroth order: kt_0 = rho
  rhob += kb[M::at(0, 0, 0)];
  apply<R, D, 2>(kp, t.u);  // C^T kappabar -> fbar (in work layout)
  // u = (j + F/2) / rho
  R jb[3];
  R udotub = R(0);
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    jb[ax] = ub[ax] * t.ir;
    udotub += t.u[ax] * ub[ax];
  }
  Fbb += ub[UP] * (R(0.5) * t.ir);
  rhob -= udotub * t.ir;
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    R v = kp[i] + rhob;
#pragma unroll
    for (int ax = 0; ax < D; ++ax)
      if (M::m(i, ax) != 1) v += R(M::m(i, ax) - 1) * jb[ax];
    fb[M::pop(i)] = v;
  }
  // T enters through the buoyancy force
  Tb += c.gbeta * Fbb;
#pragma unroll
  for (int q = 0; q < QG; ++q) gb[q] += Tb;
}

}  // namespace adj
}  // namespace fpc
