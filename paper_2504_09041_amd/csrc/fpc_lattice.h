// Lattice tables of the GPU path (compile-time constants).
//
// Population order follows the paper: D2Q9 as in Eqs. (ex), (ey) of Sec. 4.2,
// D3Q27 as in Sec. 5.2, D3Q15 as in Sec. 5.4.  The thermal lattices D2Q5 /
// D3Q7 are the first five / seven vectors of D2Q9 / D3Q27 (rest, then the
// axis links); the paper's own thermal lattices are D2Q9 and D3Q15.
//
// Weights are those of the rest state (central moments equal to their
// attractors at rho = 1 or T = 1, u = 0): the product of the 1D weights
// {2/3, 1/6, 1/6} for D2Q9 / D3Q27; for the thermal lattices, with c the
// runtime diffusion parameter c^_s^2,
//   D2Q5 / D3Q7: {1 - d c, c / 2},
//   D2Q9:        product of the 1D weights {1 - c, c / 2, c / 2},
//   D3Q15:       rest 1 - 3c + 2c^2, axis (c - c^2) / 2, corner c^2 / 8.
#pragma once

namespace fpc {

// D2Q9 in the paper's order: rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1).
constexpr int kQ2 = 9;
constexpr int D2_EX[kQ2] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int D2_EY[kQ2] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int D2_OPP[kQ2] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// index of the D2Q9 link with components (ex, ey), ex/ey in {-1,0,1}
constexpr int d2_index(int ex, int ey) {
  for (int a = 0; a < kQ2; ++a)
    if (D2_EX[a] == ex && D2_EY[a] == ey) return a;
  return -1;
}
constexpr int kQ2T = 5;  // D2Q5: first five D2Q9 links

// D3Q27 in the paper's order.
constexpr int kQ3 = 27;
constexpr int D3_EX[kQ3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int D3_EY[kQ3] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int D3_EZ[kQ3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
constexpr int d3_index(int ex, int ey, int ez) {
  for (int a = 0; a < kQ3; ++a)
    if (D3_EX[a] == ex && D3_EY[a] == ey && D3_EZ[a] == ez) return a;
  return -1;
}
constexpr int d3_opp(int a) { return d3_index(-D3_EX[a], -D3_EY[a], -D3_EZ[a]); }
constexpr int kQ3T = 7;  // D3Q7: first seven D3Q27 links

// D3Q15 in the paper's order: rest, +-x, +-y, +-z, then the eight corners
// (x sign fastest, then y, then z from +1 to -1).
constexpr int kQ15 = 15;
constexpr int T15_EX[kQ15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int T15_EY[kQ15] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int T15_EZ[kQ15] = {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
constexpr int t15_index(int ex, int ey, int ez) {
  for (int a = 0; a < kQ15; ++a)
    if (T15_EX[a] == ex && T15_EY[a] == ey && T15_EZ[a] == ez) return a;
  return -1;
}
constexpr int t15_opp(int a) { return t15_index(-T15_EX[a], -T15_EY[a], -T15_EZ[a]); }

// 1D weight of a link component e in {-1, 0, 1} (c_s^2 = 1/3).
constexpr double w1d(int e) { return e == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
constexpr double w2(int a) { return w1d(D2_EX[a]) * w1d(D2_EY[a]); }
constexpr double w3(int a) { return w1d(D3_EX[a]) * w1d(D3_EY[a]) * w1d(D3_EZ[a]); }

// Moment slots of the D3Q27 central-moment vector in the paper's order
// (000, 100, 010, 001, 110, 101, 011, 200, 020, 002, 120, 102, 210, 012,
//  201, 021, 111, 220, 202, 022, 211, 121, 112, 122, 212, 221, 222).
enum M3 : int {
  m000 = 0, m100, m010, m001, m110, m101, m011, m200, m020, m002,
  m120, m102, m210, m012, m201, m021, m111,
  m220, m202, m022, m211, m121, m112, m122, m212, m221, m222
};

}  // namespace fpc
