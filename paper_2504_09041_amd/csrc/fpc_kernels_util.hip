// Node-level utilities on a stored state: macros, FP64 export / import, and
// the FP64 diagnostics reductions (wall Nusselt number, kinetic energy,
// sum of T, max |u|, non-finite count).
//
// Macros of the time level are recovered from the post-collision state S_n:
// rho = sum f, T = sum g and rho u = sum f e - F/2 (the collision leaves
// rho and T unchanged and sets the first central moment to F/2, App. A
// Step 3 with Eq. sourceCM2D), F = g beta (T - T0) along the up axis
// (Boussinesq force, Sec. 6.1).
//
// Reductions are two-stage with a fixed tree in each block and a single-block
// final pass, so results are bit-reproducible for a given grid.
#include "fpc_kernels.h"

namespace fpc {
namespace {

constexpr int kBlock = 256;

// lattice pair codes: 1 D2Q9+D2Q5, 2 D3Q27+D3Q7, 3 D2Q9+D2Q9, 4 D3Q27+D3Q15
__device__ __forceinline__ bool is2d(int lattice) { return lattice == 1 || lattice == 3; }
__device__ __forceinline__ int qf_of(int lattice) { return is2d(lattice) ? kQ2 : kQ3; }
__device__ __forceinline__ int qg_of(int lattice) {
  return lattice == 1 ? kQ2T : (lattice == 2 ? kQ3T : (lattice == 3 ? kQ2 : kQ15));
}

__device__ __forceinline__ double wfluid(int lattice, int q) { return is2d(lattice) ? w2(q) : w3(q); }

// thermal rest weight of link q (c = c^_s^2)
__device__ __forceinline__ double wtherm(int lattice, double c, int q) {
  if (lattice == 1) return q == 0 ? 1.0 - 2.0 * c : 0.5 * c;
  if (lattice == 2) return q == 0 ? 1.0 - 3.0 * c : 0.5 * c;
  if (lattice == 3) {
    const double w0 = 1.0 - c, w1 = 0.5 * c;
    return (D2_EX[q] == 0 ? w0 : w1) * (D2_EY[q] == 0 ? w0 : w1);
  }
  return q == 0 ? 1.0 - 3.0 * c + 2.0 * c * c : (q <= 6 ? 0.5 * (c - c * c) : 0.125 * c * c);
}

__device__ __forceinline__ int ex_of(int lattice, int q) { return is2d(lattice) ? D2_EX[q] : D3_EX[q]; }
__device__ __forceinline__ int ey_of(int lattice, int q) { return is2d(lattice) ? D2_EY[q] : D3_EY[q]; }
__device__ __forceinline__ int ez_of(int lattice, int q) { return is2d(lattice) ? 0 : D3_EZ[q]; }

// thermal storage reference at a node
__device__ __forceinline__ double tref_node(const StateDesc& d, size_t node) {
  const size_t x = node % d.nx, y = (node / d.nx) % d.ny, z = node / ((size_t)d.nx * d.ny);
  return d.T_o + (d.Tg[0] * (double)x + d.Tg[1] * (double)y + d.Tg[2] * (double)z);
}

// Element of population q of (unpadded) node `node` in the storage layout:
// rows padded to nxp nodes, tiles of 64 padded nodes each holding its Q
// populations as runs of 64 values.
__device__ __forceinline__ size_t slot(const StateDesc& d, int q, size_t node) {
  const size_t x = node % d.nx, row = node / d.nx;  // row = z ny + y
  const size_t n = row * (size_t)d.nxp + x;
  const size_t Q = (size_t)(qf_of(d.lattice) + qg_of(d.lattice));
  return ((n >> 6) * Q + (size_t)q) * 64 + (n & 63);
}

template <class R>
__device__ __forceinline__ double ld(const StateDesc& d, int q, size_t node) {
  return (double)static_cast<const R*>(d.src)[slot(d, q, node)];
}

// Compile-time lattice pair (code LAT as in StateDesc::lattice).
template <int LAT>
struct Pair {
  static constexpr bool k2d = LAT == 1 || LAT == 3;
  static constexpr int QF = k2d ? kQ2 : kQ3;
  static constexpr int QG = LAT == 1 ? kQ2T : (LAT == 2 ? kQ3T : (LAT == 3 ? kQ2 : kQ15));
  static constexpr int Q = QF + QG;
  static constexpr int ex(int q) { return k2d ? D2_EX[q] : D3_EX[q]; }
  static constexpr int ey(int q) { return k2d ? D2_EY[q] : D3_EY[q]; }
  static constexpr int ez(int q) { return k2d ? 0 : D3_EZ[q]; }
};

// Padded node n of the storage layout: its coordinates and unpadded index
// (z ny + y) nx + x; false for a padding node (x >= nx).
__device__ __forceinline__ bool tile_node(const StateDesc& d, size_t n, int& x, int& y, int& z, size_t& node) {
  const size_t row = n / (size_t)d.nxp;  // z ny + y
  x = (int)(n - row * (size_t)d.nxp);
  if (x >= d.nx) return false;
  y = (int)(row % (size_t)d.ny);
  z = (int)(row / (size_t)d.ny);
  node = row * (size_t)d.nx + (size_t)x;
  return true;
}

// First element of padded node n's populations (population q at q * 64).
template <class R, int LAT>
__device__ __forceinline__ size_t tile_base(size_t n) {
  return (n >> 6) * (size_t)Pair<LAT>::Q * 64 + (n & 63);
}

// FP64 macros of one node (rho, u[3], T) from its stored populations p[q * 64]:
// rho = rho_r + sum f, T = Tr(x) + sum g, rho u = sum f e - F/2.
template <class R, int LAT>
__device__ __forceinline__ void node_macros(const StateDesc& d, const R* p, int x, int y, int z, double& rho,
                                            double u[3], double& T) {
  using P = Pair<LAT>;
  double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int q = 0; q < P::QF; ++q) {
    const double v = (double)p[(size_t)q * 64];
    s += v;
    jx += P::ex(q) * v;
    jy += P::ey(q) * v;
    jz += P::ez(q) * v;
  }
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < P::QG; ++q) t += (double)p[(size_t)(P::QF + q) * 64];
  rho = d.rho_r + s;
  T = (d.T_o + (d.Tg[0] * (double)x + d.Tg[1] * (double)y + d.Tg[2] * (double)z)) + t;
  const double Fb = d.gbeta * (T - d.T0);
  const double ir = 1.0 / rho;
  u[0] = (jx - (d.up == 0 ? 0.5 * Fb : 0.0)) * ir;
  u[1] = (jy - (d.up == 1 ? 0.5 * Fb : 0.0)) * ir;
  u[2] = (jz - (d.up == 2 ? 0.5 * Fb : 0.0)) * ir;
}

// One thread per padded node of the storage layout (consecutive lanes read
// and write consecutive elements of a tile's runs).
template <class R, int LAT>
__global__ void __launch_bounds__(kBlock) macros_kernel(StateDesc d, double* rho, double* u, double* T) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t N = (size_t)d.nx * d.ny * d.nz;
  int x, y, z;
  size_t node;
  if (n >= (size_t)d.nxp * d.ny * d.nz || !tile_node(d, n, x, y, z, node)) return;
  double r, uu[3], t;
  node_macros<R, LAT>(d, static_cast<const R*>(d.src) + tile_base<R, LAT>(n), x, y, z, r, uu, t);
  if (rho) rho[node] = r;
  if (T) T[node] = t;
  if (u) {
    constexpr int dim = Pair<LAT>::k2d ? 2 : 3;
#pragma unroll
    for (int i = 0; i < dim; ++i) u[i * N + node] = uu[i];
  }
}

template <class R, int LAT>
__global__ void __launch_bounds__(kBlock) export_kernel(StateDesc d, double* dst) {
  using P = Pair<LAT>;
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t N = (size_t)d.nx * d.ny * d.nz;
  int x, y, z;
  size_t node;
  if (n >= (size_t)d.nxp * d.ny * d.nz || !tile_node(d, n, x, y, z, node)) return;
  const R* p = static_cast<const R*>(d.src) + tile_base<R, LAT>(n);
#pragma unroll
  for (int q = 0; q < P::QF; ++q) dst[q * N + node] = (double)p[(size_t)q * 64] + wfluid(LAT, q) * d.rho_r;
  const double tr = d.T_o + (d.Tg[0] * (double)x + d.Tg[1] * (double)y + d.Tg[2] * (double)z);
#pragma unroll
  for (int q = 0; q < P::QG; ++q)
    dst[(P::QF + q) * N + node] = (double)p[(size_t)(P::QF + q) * 64] + wtherm(LAT, d.cs2T, q) * tr;
}

template <class R, int LAT>
__global__ void __launch_bounds__(kBlock) import_kernel(StateDesc d, R* out, const double* src) {
  using P = Pair<LAT>;
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t N = (size_t)d.nx * d.ny * d.nz;
  int x, y, z;
  size_t node;
  if (n >= (size_t)d.nxp * d.ny * d.nz || !tile_node(d, n, x, y, z, node)) return;
  R* p = out + tile_base<R, LAT>(n);
#pragma unroll
  for (int q = 0; q < P::QF; ++q) p[(size_t)q * 64] = (R)(src[q * N + node] - wfluid(LAT, q) * d.rho_r);
  const double tr = d.T_o + (d.Tg[0] * (double)x + d.Tg[1] * (double)y + d.Tg[2] * (double)z);
#pragma unroll
  for (int q = 0; q < P::QG; ++q)
    p[(size_t)(P::QF + q) * 64] = (R)(src[(P::QF + q) * N + node] - wtherm(LAT, d.cs2T, q) * tr);
}

// Deterministic block reduction: sum (op 0) or max (op 1) over kBlock values.
__device__ double block_reduce(double v, double* sh, int op) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = op == 0 ? sh[t] + sh[t + s] : fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Stage 1 over nodes: partials[b * 4 + (KE, sumT, umax, nonfinite)].  A
// fixed number of blocks (a function of N only) strides over the storage
// tiles, one wavefront per 64-node tile (its loads are the tile's runs), so
// the partials fit a fixed scratch size for every grid and the summation
// order is the same on every call.  LAT: the lattice pair code (compile-time
// link vectors and population counts).
template <class R, int LAT>
__global__ void __launch_bounds__(kBlock) diag_nodes_kernel(StateDesc d, double* partials) {
  constexpr int Q = Pair<LAT>::Q;
  constexpr int kWaves = kBlock / 64;
  __shared__ double sh[kBlock];
  const int lane = (int)(threadIdx.x & 63);
  const size_t tiles_x = (size_t)d.nxp / 64;
  const size_t ntiles = tiles_x * d.ny * d.nz;
  const size_t wstride = (size_t)gridDim.x * kWaves;
  const R* src = static_cast<const R*>(d.src);
  double ke = 0.0, st = 0.0, um = 0.0, bad = 0.0;
  for (size_t t = (size_t)blockIdx.x * kWaves + (threadIdx.x >> 6); t < ntiles; t += wstride) {
    const size_t row = t / tiles_x;  // z ny + y
    const int x = (int)(t - row * tiles_x) * 64 + lane;
    if (x >= d.nx) continue;  // padding node
    const int y = (int)(row % (size_t)d.ny), z = (int)(row / (size_t)d.ny);
    double r, uu[3], T;
    node_macros<R, LAT>(d, src + t * (size_t)Q * 64 + lane, x, y, z, r, uu, T);
    const double ux = uu[0], uy = uu[1], uz = uu[2];
    const double u2 = ux * ux + uy * uy + uz * uz;
    if (!isfinite(r) || !isfinite(T) || !isfinite(u2)) {
      bad += 1.0;
    } else {
      ke += 0.5 * r * u2;
      st += T;
      um = fmax(um, sqrt(u2));
    }
  }
  ke = block_reduce(ke, sh, 0);
  st = block_reduce(st, sh, 0);
  um = block_reduce(um, sh, 1);
  bad = block_reduce(bad, sh, 0);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = ke;
    partials[blockIdx.x * 4 + 1] = st;
    partials[blockIdx.x * 4 + 2] = um;
    partials[blockIdx.x * 4 + 3] = bad;
  }
}

template <class R>
void launch_diag_nodes(const StateDesc& d, unsigned nb, double* partials, hipStream_t s) {
  switch (d.lattice) {
    case 1: diag_nodes_kernel<R, 1><<<nb, kBlock, 0, s>>>(d, partials); break;
    case 2: diag_nodes_kernel<R, 2><<<nb, kBlock, 0, s>>>(d, partials); break;
    case 3: diag_nodes_kernel<R, 3><<<nb, kBlock, 0, s>>>(d, partials); break;
    default: diag_nodes_kernel<R, 4><<<nb, kBlock, 0, s>>>(d, partials); break;
  }
}

// Stage 1 over the per-tile partials of a step with fused diagnostics: the
// same four quantities, a fixed number of blocks striding over the tiles.
__global__ void __launch_bounds__(kBlock) diag_tiles_kernel(const double* part, size_t ntiles, double* partials) {
  __shared__ double sh[kBlock];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  double ke = 0.0, st = 0.0, um = 0.0, bad = 0.0;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += stride) {
    ke += part[t * 4 + 0];
    st += part[t * 4 + 1];
    um = fmax(um, part[t * 4 + 2]);
    bad += part[t * 4 + 3];
  }
  ke = block_reduce(ke, sh, 0);
  st = block_reduce(st, sh, 0);
  um = block_reduce(um, sh, 1);
  bad = block_reduce(bad, sh, 0);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = ke;
    partials[blockIdx.x * 4 + 1] = st;
    partials[blockIdx.x * 4 + 2] = um;
    partials[blockIdx.x * 4 + 3] = bad;
  }
}

__device__ __forceinline__ size_t face_nodes_dev(const StateDesc& d, int face) {
  const int k = face >> 1;
  const size_t n[3] = {(size_t)d.nx, (size_t)d.ny, (size_t)d.nz};
  return n[(k + 1) % 3] * n[(k + 2) % 3];
}

// Local Nusselt number at wall node i of `face` (i in the profile layout:
// faster tangential axis first): the one-sided stencil of Sec. 6.1,
// dT/dn = -8/3 T_w + 3 T(1/2) - 1/3 T(3/2) along the inward normal,
// Nu = -(L / dT_ref) dT/dn with L the nodes along the normal.
template <class R>
__device__ double local_nusselt(const StateDesc& d, int face, const FaceDev& fd, double dT_ref, size_t i) {
  const int k = face >> 1;
  const int n[3] = {d.nx, d.ny, d.nz};
  const int t1 = k == 0 ? 1 : 0;  // faster tangential axis
  const int t2 = k == 2 ? 1 : 2;  // slower tangential axis
  const int L = n[k];
  const int Qf = qf_of(d.lattice);
  const int Qg = qg_of(d.lattice);
  int c[3];
  c[t1] = (int)(i % n[t1]);
  c[t2] = (int)(i / n[t1]);
  double Tl[2];
  for (int layer = 0; layer < 2; ++layer) {
    c[k] = (face & 1) ? L - 1 - layer : layer;
    const size_t node = ((size_t)c[2] * d.ny + c[1]) * d.nx + c[0];
    double t = 0.0;
    for (int q = 0; q < Qg; ++q) t += ld<R>(d, Qf + q, node);
    Tl[layer] = tref_node(d, node) + t;
  }
  const double Tw = fd.Tprof ? fd.Tprof[i] : fd.Tw;
  const double dTdn = -8.0 / 3.0 * Tw + 3.0 * Tl[0] - Tl[1] / 3.0;
  return -((double)L / dT_ref) * dTdn;
}

// Stage 1 over the nodes of one face: sums of the local Nusselt numbers
// (fixed number of blocks striding over the face).
template <class R>
__global__ void __launch_bounds__(kBlock) diag_face_kernel(StateDesc d, int face, FaceDev fd, double dT_ref,
                                                           double* partials) {
  __shared__ double sh[kBlock];
  const size_t M = face_nodes_dev(d, face);
  double nu = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (size_t)gridDim.x * blockDim.x)
    nu += local_nusselt<R>(d, face, fd, dT_ref, i);
  nu = block_reduce(nu, sh, 0);
  if (threadIdx.x == 0) partials[blockIdx.x] = nu;
}

// Local Nusselt number of every node of a face (profile layout).
template <class R>
__global__ void __launch_bounds__(kBlock) nu_local_kernel(StateDesc d, int face, FaceDev fd, double dT_ref,
                                                          double* out) {
  const size_t M = face_nodes_dev(d, face);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (size_t)gridDim.x * blockDim.x)
    out[i] = local_nusselt<R>(d, face, fd, dT_ref, i);
}

// Final stage (one block): out = (mean Nu over the face or 0, KE, sum T,
// max |u|, number of non-finite nodes).
__global__ void __launch_bounds__(kBlock) diag_final_kernel(const double* pn, int nb, const double* pf, int nf,
                                                            double inv_face_nodes, double* out) {
  __shared__ double sh[kBlock];
  double ke = 0.0, st = 0.0, um = 0.0, bad = 0.0, nu = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    ke += pn[b * 4 + 0];
    st += pn[b * 4 + 1];
    um = fmax(um, pn[b * 4 + 2]);
    bad += pn[b * 4 + 3];
  }
  for (int b = threadIdx.x; b < nf; b += kBlock) nu += pf[b];
  nu = block_reduce(nu, sh, 0);
  ke = block_reduce(ke, sh, 0);
  st = block_reduce(st, sh, 0);
  um = block_reduce(um, sh, 1);
  bad = block_reduce(bad, sh, 0);
  if (threadIdx.x == 0) {
    out[0] = nu * inv_face_nodes;
    out[1] = ke;
    out[2] = st;
    out[3] = um;
    out[4] = bad;
  }
}

// Stage 1 of the wall-Nusselt slot reduction: each block sums its slots
// (grid-stride, fixed order) into partials[blockIdx.x] and resets them to 0.
__global__ void __launch_bounds__(kBlock) nu_slots_partial_kernel(double* slot, size_t count, double* partials) {
  __shared__ double sh[kBlock];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  double v = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    v += slot[i];
    slot[i] = 0.0;
  }
  v = block_reduce(v, sh, 0);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// Stage 2: acc[0] += the sum of the nb partials (fixed order).
__global__ void __launch_bounds__(kBlock) nu_slots_final_kernel(const double* partials, int nb, double* acc) {
  __shared__ double sh[kBlock];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) v += partials[b];
  v = block_reduce(v, sh, 0);
  if (threadIdx.x == 0) acc[0] += v;
}

__global__ void __launch_bounds__(kBlock) fill_zero_kernel(double* p, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Adjoint seeds of J = weight <Nu>_face with
// <Nu> = (1/M) sum_wall -(L / dT_ref) (-8/3 T_w + 3 T(1/2) - 1/3 T(3/2)):
// dJ/dT = 3 s on the first layer, -s/3 on the second, 0 elsewhere, and
// dJ/dT_w = -8/3 s, with s = -(L / dT_ref) weight / M.
__global__ void __launch_bounds__(kBlock) nu_seed_kernel(int nx, int ny, int nz, int face, double s, double* dJdT) {
  const size_t N = (size_t)nx * ny * nz;
  const int k = face >> 1;
  const int n = k == 0 ? nx : (k == 1 ? ny : nz);
  for (size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x; node < N;
       node += (size_t)gridDim.x * blockDim.x) {
    const int c = k == 0 ? (int)(node % nx) : (k == 1 ? (int)((node / nx) % ny) : (int)(node / ((size_t)nx * ny)));
    const int layer = (face & 1) ? n - 1 - c : c;
    dJdT[node] = layer == 0 ? 3.0 * s : (layer == 1 ? -s / 3.0 : 0.0);
  }
}

__global__ void __launch_bounds__(kBlock) nu_seed_wall_kernel(size_t M, double s, double* dJdTw) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (size_t)gridDim.x * blockDim.x)
    dJdTw[i] = -8.0 / 3.0 * s;
}

unsigned grid_for(size_t count) {
  const size_t b = (count + kBlock - 1) / kBlock;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Blocks of the two stage-1 kernels: one per kBlock nodes, capped.
unsigned diag_node_blocks(const StateDesc& d) {
  const size_t N = (size_t)d.nx * d.ny * d.nz;
  const size_t b = (N + kBlock - 1) / kBlock;
  return (unsigned)(b < kDiagNodeBlocks ? b : kDiagNodeBlocks);
}

size_t face_nodes(const StateDesc& d, int face) {
  const int k = face >> 1;
  const size_t n[3] = {(size_t)d.nx, (size_t)d.ny, (size_t)d.nz};
  return n[(k + 1) % 3] * n[(k + 2) % 3];
}

unsigned diag_face_blocks(const StateDesc& d, int face) {
  const size_t b = (face_nodes(d, face) + kBlock - 1) / kBlock;
  return (unsigned)(b < kDiagFaceBlocks ? b : kDiagFaceBlocks);
}

}  // namespace

namespace {
// blocks of kBlock threads over the padded nodes of the storage layout
unsigned padded_blocks(const StateDesc& d) {
  return (unsigned)(((size_t)d.nxp * d.ny * d.nz + kBlock - 1) / kBlock);
}
}  // namespace

#define FPC_BY_LATTICE(KERNEL, R, ...)                                                          \
  switch (d.lattice) {                                                                          \
    case 1: KERNEL<R, 1><<<padded_blocks(d), kBlock, 0, s>>>(__VA_ARGS__); break;              \
    case 2: KERNEL<R, 2><<<padded_blocks(d), kBlock, 0, s>>>(__VA_ARGS__); break;              \
    case 3: KERNEL<R, 3><<<padded_blocks(d), kBlock, 0, s>>>(__VA_ARGS__); break;              \
    default: KERNEL<R, 4><<<padded_blocks(d), kBlock, 0, s>>>(__VA_ARGS__); break;             \
  }

hipError_t launch_macros(const StateDesc& d, double* rho, double* u, double* T, hipStream_t s) {
  if (d.precision == 0) {
    FPC_BY_LATTICE(macros_kernel, double, d, rho, u, T)
  } else {
    FPC_BY_LATTICE(macros_kernel, float, d, rho, u, T)
  }
  return hipGetLastError();
}

hipError_t launch_export(const StateDesc& d, double* dst, hipStream_t s) {
  if (d.precision == 0) {
    FPC_BY_LATTICE(export_kernel, double, d, dst)
  } else {
    FPC_BY_LATTICE(export_kernel, float, d, dst)
  }
  return hipGetLastError();
}

hipError_t launch_import(const StateDesc& d, void* dst, const double* src, hipStream_t s) {
  if (d.precision == 0) {
    FPC_BY_LATTICE(import_kernel, double, d, static_cast<double*>(dst), src)
  } else {
    FPC_BY_LATTICE(import_kernel, float, d, static_cast<float*>(dst), src)
  }
  return hipGetLastError();
}
#undef FPC_BY_LATTICE

hipError_t launch_diagnostics(const StateDesc& d, int face, const FaceDev& fd, double dT_ref, double* scratch,
                              double* out, hipStream_t s) {
  const unsigned nb = diag_node_blocks(d);
  double* pf = scratch + (size_t)kDiagNodeBlocks * 4;
  unsigned nf = 0;
  double inv_m = 0.0;
  if (d.precision == 0)
    launch_diag_nodes<double>(d, nb, scratch, s);
  else
    launch_diag_nodes<float>(d, nb, scratch, s);
  if (face >= 0) {
    nf = diag_face_blocks(d, face);
    inv_m = 1.0 / (double)face_nodes(d, face);
    if (d.precision == 0)
      diag_face_kernel<double><<<nf, kBlock, 0, s>>>(d, face, fd, dT_ref, pf);
    else
      diag_face_kernel<float><<<nf, kBlock, 0, s>>>(d, face, fd, dT_ref, pf);
  }
  diag_final_kernel<<<1, kBlock, 0, s>>>(scratch, (int)nb, pf, (int)nf, inv_m, out);
  return hipGetLastError();
}

size_t nu_slot_count(int nx, int ny, int nz, int nxp, int face) {
  const size_t nxt = (size_t)nxp / 64;
  const int k = face >> 1;
  if (k == 0) return 2 * (size_t)ny * nz;
  if (k == 1) return 2 * (size_t)nz * nxt;
  return 2 * (size_t)ny * nxt;
}

namespace {
unsigned nu_slot_blocks(size_t count) {
  const size_t b = (count + kBlock - 1) / kBlock;
  return (unsigned)(b == 0 ? 1 : (b < kDiagFaceBlocks ? b : kDiagFaceBlocks));
}
}  // namespace

hipError_t launch_diag_tiles(const double* part, size_t ntiles, double* slot, size_t nslots, double* scratch,
                             double* out, hipStream_t s) {
  size_t nb = (ntiles + kBlock - 1) / kBlock;
  if (nb > kDiagNodeBlocks) nb = kDiagNodeBlocks;
  if (nb == 0) nb = 1;
  diag_tiles_kernel<<<(unsigned)nb, kBlock, 0, s>>>(part, ntiles, scratch);
  double* pf = scratch + (size_t)kDiagNodeBlocks * 4;
  unsigned nf = 0;
  if (slot != nullptr) {
    nf = nu_slot_blocks(nslots);
    nu_slots_partial_kernel<<<nf, kBlock, 0, s>>>(slot, nslots, pf);
  }
  // the slots already carry the 1 / (nodes on the face) of the mean
  diag_final_kernel<<<1, kBlock, 0, s>>>(scratch, (int)nb, pf, (int)nf, 1.0, out);
  return hipGetLastError();
}

hipError_t launch_nu_slots_reduce(double* slot, size_t count, double* scratch, double* acc, hipStream_t s) {
  double* pf = scratch + (size_t)kDiagNodeBlocks * 4;
  const unsigned nf = nu_slot_blocks(count);
  nu_slots_partial_kernel<<<nf, kBlock, 0, s>>>(slot, count, pf);
  nu_slots_final_kernel<<<1, kBlock, 0, s>>>(pf, (int)nf, acc);
  return hipGetLastError();
}

hipError_t launch_nu_local(const StateDesc& d, int face, const FaceDev& fd, double dT_ref, double* out,
                           hipStream_t s) {
  const unsigned nb = grid_for(face_nodes(d, face));
  if (d.precision == 0)
    nu_local_kernel<double><<<nb, kBlock, 0, s>>>(d, face, fd, dT_ref, out);
  else
    nu_local_kernel<float><<<nb, kBlock, 0, s>>>(d, face, fd, dT_ref, out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, size_t count, hipStream_t s) {
  fill_zero_kernel<<<grid_for(count), kBlock, 0, s>>>(p, count);
  return hipGetLastError();
}

hipError_t launch_nu_seed(const StateDesc& d, int face, double dT_ref, double weight, double* dJdT, double* dJdTw,
                          hipStream_t s) {
  const size_t N = (size_t)d.nx * d.ny * d.nz;
  const size_t M = face_nodes(d, face);
  const int n[3] = {d.nx, d.ny, d.nz};
  const double sc = -((double)n[face >> 1] / dT_ref) * weight / (double)M;
  nu_seed_kernel<<<grid_for(N), kBlock, 0, s>>>(d.nx, d.ny, d.nz, face, sc, dJdT);
  if (dJdTw) nu_seed_wall_kernel<<<grid_for(M), kBlock, 0, s>>>(M, sc, dJdTw);
  return hipGetLastError();
}

}  // namespace fpc
