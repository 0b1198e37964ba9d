// Fused pull-stream + collide kernel (D2Q9 + D2Q5 and D3Q27 + D3Q7).
//
// One thread per node.  Each thread gathers its incoming populations
// f_a(x) = f~_a(x - e_a) from S_{n-1} (Eq. LBMsteps-stream, LBMsteps-streamg);
// where x - e_a lies outside a wall face it applies the halfway wall rule at
// its own node (Sec. 6.1):
//   no-slip      f_a = f~_abar
//   moving wall  f_a = f~_abar + 2 w_a rho_w (e_a . u_w) / c_s^2
//   adiabatic    g_a = g~_abar
//   Dirichlet    g_a = -g~_abar + 2 w^T_a T_w
// then collides in registers (fpc_collide.h) and stores its own values to S_n.
//
// Layout: SoA planes, plane q holds the N node values [z][y][x]; a wavefront
// covers 64 consecutive x of one row, so every load is a contiguous run of one
// plane (shifted by at most one element) and every store is fully coalesced.
//
// Boundary handling is resolved per wavefront: a ballot tells whether any lane
// of the wave sits on an x, y or z edge of the box, and the gather is
// instantiated with range checks only on those axes.  Interior wavefronts (the
// vast majority) load every population from a wave-uniform plane base with a
// 32-bit lane offset and no checks at all; x-edge wavefronts check only the
// links that move along x.  Checked links stay branch-free: a wall redirects
// the single load of the link to the node's own opposite slot.
//
// Stores are non-temporal when the state is too large to stay in the
// last-level cache (it then streams through HBM anyway); smaller states keep
// ordinary stores so that the next step reads them from the cache.
#include "fpc_kernels.h"


namespace fpc {
namespace {

struct Lat2 {
  static constexpr int D = 2, Qf = kQ2, Qg = kQ2T;
  static constexpr int ex(int a) { return D2_EX[a]; }
  static constexpr int ey(int a) { return D2_EY[a]; }
  static constexpr int ez(int) { return 0; }
  static constexpr int opp(int a) { return D2_OPP[a]; }
  static constexpr double w(int a) { return w2(a); }
};

struct Lat3 {
  static constexpr int D = 3, Qf = kQ3, Qg = kQ3T;
  static constexpr int ex(int a) { return D3_EX[a]; }
  static constexpr int ey(int a) { return D3_EY[a]; }
  static constexpr int ez(int a) { return D3_EZ[a]; }
  static constexpr int opp(int a) { return d3_opp(a); }
  static constexpr double w(int a) { return w3(a); }
};

// ---------------------------------------------------------------------------
// State addressing.  Two policies with the same interface:
//   load(q, shift, idx)   plane q at lane index idx - shift (shift wave-uniform)
//   load_sel(w, qw, iw, q, shift, idx)  per lane: plane qw at iw if w, else as load
//   store<NT>(q, idx, v)
// Buf32: the whole buffer through one raw buffer descriptor; the lane supplies
//   a 32-bit byte offset and the plane offset is a wave-uniform scalar
//   (usable while the buffer is below 4 GiB).  Keeps the address arithmetic
//   off the vector ALU and the scalar register file small.
// Glob64: 64-bit plane base pointers plus a 32-bit lane offset (any size).
// ---------------------------------------------------------------------------
constexpr int kBufDword3 = 0x00020000;  // raw (untyped) buffer, gfx9 family
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

template <class R>
struct Buf32 {
  const StepArgs<R>& a;
  unsigned nbytes;  // buffer size (bytes)
  static constexpr unsigned S = sizeof(R);

  __device__ __forceinline__ Buf32(const StepArgs<R>& a_, unsigned total_bytes) : a(a_), nbytes(total_bytes) {}

  // descriptors built at each use from the kernel arguments (wave-uniform,
  // so they stay in scalar registers and are shared by CSE)
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_src() const {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<R*>(a.src), 0, (int)nbytes, kBufDword3);
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_dst() const {
    return __builtin_amdgcn_make_buffer_rsrc(a.dst, 0, (int)nbytes, kBufDword3);
  }
  __device__ __forceinline__ unsigned pb() const { return (unsigned)a.plane * S; }

  __device__ __forceinline__ R raw(unsigned voff, unsigned soff) const {
    if constexpr (sizeof(R) == 4)
      return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rsrc_src(), (int)voff, (int)soff, 0));
    else
      return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rsrc_src(), (int)voff, (int)soff, 0));
  }
  // byte offset of plane q minus the streaming shift (non-negative for q >= 1
  // or shift == 0, as every plane is longer than any shift)
  __device__ __forceinline__ unsigned base(int q, long long shift) const {
    return (unsigned)q * pb() - (unsigned)(shift * (long long)S);
  }
  __device__ __forceinline__ R load(int q, long long shift, unsigned idx) const {
    return raw(idx * S, base(q, shift));
  }
  __device__ __forceinline__ R load_sel(bool w, int qw, unsigned iw, int q, long long shift, unsigned idx) const {
    const unsigned vs = idx * S + base(q, shift);
    const unsigned vw = iw * S + (unsigned)qw * pb();
    return raw(w ? vw : vs, 0u);
  }
  template <bool NT>
  __device__ __forceinline__ void store(int q, unsigned idx, R v) const {
    constexpr int aux = NT ? 2 : 0;  // cache policy: non-temporal
    // plane offset on the lane side: one add per store, no scalar register
    // per plane held across the collision
    const int vo = (int)(idx * S + (unsigned)q * pb());
    if constexpr (sizeof(R) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rsrc_dst(), vo, 0, aux);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rsrc_dst(), vo, 0, aux);
  }
};

template <class R>
struct Glob64 {
  const R* src;
  R* dst;
  size_t plane;

  __device__ __forceinline__ Glob64(const StepArgs<R>& a, unsigned) : src(a.src), dst(a.dst), plane(a.plane) {}

  // base[idx] with a 32-bit byte offset (uniform base + lane offset)
  static __device__ __forceinline__ R ld(const R* base, unsigned idx) {
    return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(R));
  }
  __device__ __forceinline__ R load(int q, long long shift, unsigned idx) const {
    return ld(src + (size_t)q * plane - shift, idx);
  }
  __device__ __forceinline__ R load_sel(bool w, int qw, unsigned iw, int q, long long shift, unsigned idx) const {
    const R* pw = src + (size_t)qw * plane;
    const R* ps = src + (size_t)q * plane - shift;
    return ld(w ? pw : ps, w ? iw : idx);
  }
  template <bool NT>
  __device__ __forceinline__ void store(int q, unsigned idx, R v) const {
    R* p = reinterpret_cast<R*>(reinterpret_cast<char*>(dst + (size_t)q * plane) + idx * (unsigned)sizeof(R));
    if constexpr (NT)
      __builtin_nontemporal_store(v, p);
    else
      *p = v;
  }
};

template <class L, class R, class M, bool CX, bool CY, bool CZ, bool PX>
struct Gather {
  const StepArgs<R>& a;
  const M& m;
  int x, y, z;
  unsigned node;
  R Tr;  // thermal storage reference of this node
  // Lane on the low / high edge of a checked axis.  A link with e_k = +1
  // crossing the low edge (or e_k = -1 crossing the high edge) either wraps
  // (periodic axis: the source index moves by +-n_k times the axis stride) or
  // meets a wall.  PX: x is known to be periodic.
  bool xlo = false, xhi = false, ylo = false, yhi = false, zlo = false, zhi = false;
  unsigned nxm = 0, nxp = 0;  // node index with the x wrap of an e_x = -1 / +1 link applied

  __device__ __forceinline__ Gather(const StepArgs<R>& a_, const M& m_, int x_, int y_, int z_, unsigned node_,
                                    R Tr_)
      : a(a_), m(m_), x(x_), y(y_), z(z_), node(node_), Tr(Tr_) {
    if (CX) {
      xlo = x == 0;
      xhi = x == a.nx - 1;
      nxp = node + (xlo ? (unsigned)a.nx : 0u);
      nxm = node - (xhi ? (unsigned)a.nx : 0u);
    }
    if (CY) {
      ylo = y == 0;
      yhi = y == a.ny - 1;
    }
    if (CZ) {
      zlo = z == 0;
      zhi = z == a.nz - 1;
    }
  }

  // Incoming population of link A of one distribution whose planes start at
  // QBASE (fluid: 0, thermal: Qf).  Returns the pulled or bounced value and
  // reports per axis whether the link met a wall there.
  template <int A, int QBASE>
  __device__ __forceinline__ R pull(bool& wx, bool& wy, bool& wz) const {
    constexpr int ex = L::ex(A), ey = L::ey(A), ez = L::ez(A);
    const long long shift = (long long)ex + (long long)ey * a.nx + (long long)ez * a.nx * a.ny;
    constexpr bool cx = CX && ex != 0, cy = CY && ey != 0, cz = CZ && ez != 0;
    if (!cx && !cy && !cz) return m.load(QBASE + A, shift, node);
    const bool ox = cx && (ex > 0 ? xlo : xhi);
    const bool oy = cy && (ey > 0 ? ylo : yhi);
    const bool oz = cz && (ez > 0 ? zlo : zhi);
    unsigned idx = cx ? (ex > 0 ? nxp : nxm) : node;
    if (cy) idx += oy ? (unsigned)(ey * a.ny) * (unsigned)a.nx : 0u;
    if (cz) idx += oz ? (unsigned)(ez * a.nz) * (unsigned)a.nx * (unsigned)a.ny : 0u;
    wx = ox && !PX && !a.per[0];
    wy = oy && !a.per[1];
    wz = oz && !a.per[2];
    if (PX && !cy && !cz) return m.load(QBASE + A, shift, idx);  // periodic x only: never a wall
    const bool wall = wx || wy || wz;
    return m.load_sel(wall, QBASE + L::opp(A), node, QBASE + A, shift, idx);
  }

  template <int F>
  __device__ __forceinline__ R lid_term(int A_ex, int A_ey, int A_ez, double w) const {
    if (!a.face[F].lid) return R(0);
    const double eu = A_ex * a.face[F].uw[0] + A_ey * a.face[F].uw[1] + A_ez * a.face[F].uw[2];
    return R(2.0 * 3.0 * w) * a.rho_w * R(eu);
  }

  template <int A>
  __device__ __forceinline__ R f() const {
    bool wx = false, wy = false, wz = false;
    R v = pull<A, 0>(wx, wy, wz);
    constexpr int ex = L::ex(A), ey = L::ey(A), ez = L::ez(A);
    constexpr bool checked = (CX && ex != 0) || (CY && ey != 0) || (CZ && ez != 0);
    if (checked) {
      // moving wall: only when exactly one face is crossed
      constexpr int FX = ex > 0 ? 0 : 1, FY = ey > 0 ? 2 : 3, FZ = ez > 0 ? 4 : 5;
      const int nc = (int)wx + (int)wy + (int)wz;
      R add = R(0);
      if (ex != 0) add = (nc == 1 && wx) ? lid_term<FX>(ex, ey, ez, L::w(A)) : add;
      if (ey != 0) add = (nc == 1 && wy) ? lid_term<FY>(ex, ey, ez, L::w(A)) : add;
      if (ez != 0) add = (nc == 1 && wz) ? lid_term<FZ>(ex, ey, ez, L::w(A)) : add;
      v += add;
    }
    return v;
  }

  // Thermal link A (axis links: at most one face can be crossed).
  template <int A>
  __device__ __forceinline__ R g() const {
    bool wx = false, wy = false, wz = false;
    R v = pull<A, L::Qf>(wx, wy, wz);
    if (A == 0) return v;
    constexpr int ex = L::ex(A), ey = L::ey(A), ez = L::ez(A);
    constexpr bool checked = (CX && ex != 0) || (CY && ey != 0) || (CZ && ez != 0);
    constexpr int F = ex > 0 ? 0 : (ex < 0 ? 1 : (ey > 0 ? 2 : (ey < 0 ? 3 : (ez > 0 ? 4 : 5))));
    constexpr int k = F >> 1;
    constexpr int e = ex + ey + ez;  // axis link: the one non-zero component
    const bool wall = checked && (wx || wy || wz);
    if (wall) {
      if (a.face[F].dirichlet) {
        double Tw = a.face[F].Tw;
        if (a.face[F].Tprof) {
          const size_t t = k == 0 ? (size_t)z * a.ny + y : (k == 1 ? (size_t)z * a.nx + x : (size_t)y * a.nx + x);
          Tw = a.face[F].Tprof[t];
        }
        v = -v + a.c.cs2T * (R(Tw) - Tr);  // 2 w^T_a = c^_s^2 on axis links
      }
    } else if constexpr (kDeviations<R>) {
      // the value was stored against the source node's reference Tr(x - e_A)
      v -= R(0.5) * a.c.cs2T * (R(e) * a.Tg[k]);
    }
    return v;
  }
};

template <class L, class R, class M, bool CX, bool CY, bool CZ, bool PX = false>
__device__ __forceinline__ void gather(const StepArgs<R>& a, const M& m, int x, int y, int z, unsigned node, R Tr,
                                       R (&f)[L::Qf], R (&g)[L::Qg]) {
  const Gather<L, R, M, CX, CY, CZ, PX> p(a, m, x, y, z, node, Tr);
  if constexpr (L::D == 2) {
    f[0] = p.template f<0>(); f[1] = p.template f<1>(); f[2] = p.template f<2>();
    f[3] = p.template f<3>(); f[4] = p.template f<4>(); f[5] = p.template f<5>();
    f[6] = p.template f<6>(); f[7] = p.template f<7>(); f[8] = p.template f<8>();
    g[0] = p.template g<0>(); g[1] = p.template g<1>(); g[2] = p.template g<2>();
    g[3] = p.template g<3>(); g[4] = p.template g<4>();
  } else {
#define FPC_F(A) f[A] = p.template f<A>();
    FPC_F(0) FPC_F(1) FPC_F(2) FPC_F(3) FPC_F(4) FPC_F(5) FPC_F(6) FPC_F(7) FPC_F(8)
    FPC_F(9) FPC_F(10) FPC_F(11) FPC_F(12) FPC_F(13) FPC_F(14) FPC_F(15) FPC_F(16) FPC_F(17)
    FPC_F(18) FPC_F(19) FPC_F(20) FPC_F(21) FPC_F(22) FPC_F(23) FPC_F(24) FPC_F(25) FPC_F(26)
#undef FPC_F
    g[0] = p.template g<0>(); g[1] = p.template g<1>(); g[2] = p.template g<2>();
    g[3] = p.template g<3>(); g[4] = p.template g<4>(); g[5] = p.template g<5>();
    g[6] = p.template g<6>();
  }
}

template <class L, class R, class M, int UP, bool NT, bool STD>
__device__ __forceinline__ void collide_store(const StepArgs<R>& a, const M& m, unsigned node, R Tr, R (&f)[L::Qf],
                                              R (&g)[L::Qg]) {
  if constexpr (L::D == 2)
    collide2d<R, UP, STD>(f, g, a.c, Tr, (Macros<R>*)nullptr);
  else
    collide3d<R, UP, STD>(f, g, a.c, Tr, (Macros<R>*)nullptr);
#pragma unroll
  for (int q = 0; q < L::Qf; ++q) m.template store<NT>(q, node, f[q]);
#pragma unroll
  for (int q = 0; q < L::Qg; ++q) m.template store<NT>(L::Qf + q, node, g[q]);
}

__device__ __forceinline__ unsigned node_of(int x, int y, int z, int nx, int ny) {
  return ((unsigned)z * (unsigned)ny + (unsigned)y) * (unsigned)nx + (unsigned)x;
}

// M: addressing policy (Buf32 when the buffer is below 4 GiB, else Glob64).
// STD: the standard rate set (see rate_f / rate_g).
template <class L, class R, class M, int UP, bool NT, bool STD>
__global__ void __launch_bounds__(256) step_kernel(StepArgs<R> a, unsigned total_bytes) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const M m(a, total_bytes);
  const unsigned node = node_of(x, y, z, a.nx, a.ny);
  const R Tr = tref(a, x, y, z);
  R f[L::Qf], g[L::Qg];
  // which axes have an edge node in this wavefront (wave-uniform)
  const bool needx = __any(x == 0 || x == a.nx - 1);
  const bool needy = __any(y == 0 || y == a.ny - 1);
  const bool needz = L::D == 3 && __any(z == 0 || z == a.nz - 1);
  if (!needy && !needz) {
    if (!needx)
      gather<L, R, M, false, false, false>(a, m, x, y, z, node, Tr, f, g);
    else if (a.per[0])
      gather<L, R, M, true, false, false, true>(a, m, x, y, z, node, Tr, f, g);
    else
      gather<L, R, M, true, false, false>(a, m, x, y, z, node, Tr, f, g);
  } else {
    gather<L, R, M, true, true, L::D == 3>(a, m, x, y, z, node, Tr, f, g);
  }
  collide_store<L, R, M, UP, NT, STD>(a, m, node, Tr, f, g);
}

// Initial state: the collision of f = w rho0, g = w^T T_init at every node.
template <class L, class R, int UP>
__global__ void __launch_bounds__(256) init_kernel(StepArgs<R> a, const double* __restrict__ T_init) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const Glob64<R> m(a, 0u);
  const unsigned node = node_of(x, y, z, a.nx, a.ny);
  R f[L::Qf], g[L::Qg];
  const R drw = a.rho_w - a.c.rho_r;
#pragma unroll
  for (int q = 0; q < L::Qf; ++q) f[q] = R(L::w(q)) * drw;
  const R Tr = tref(a, x, y, z);
  const R dT = R(T_init[node]) - Tr;
  g[0] = (R(1) - R(L::D) * a.c.cs2T) * dT;
#pragma unroll
  for (int q = 1; q < L::Qg; ++q) g[q] = R(0.5) * a.c.cs2T * dT;
  collide_store<L, R, Glob64<R>, UP, false, false>(a, m, node, Tr, f, g);
}

// Whether the rates form the standard set of rate_f / rate_g: the viscous
// slots share one rate, the thermal first-order slots share one rate, and
// every other slot in use relaxes at exactly 1.
template <class R>
bool standard_rates(const StepArgs<R>& a, int D) {
  const int Qf = D == 2 ? kQ2 : kQ3;
  for (int k = 1; k < Qf; ++k) {
    const bool nu = D == 2 ? (k == 4 || k == 5) : (k == 4 || k == 5 || k == 6 || k == 8 || k == 9);
    if (nu ? a.c.om[k] != a.c.om[4] : a.c.om[k] != R(1)) return false;
  }
  const int Qg = D == 2 ? kQ2T : kQ3T;
  for (int k = 1; k < Qg; ++k) {
    const bool first = k <= D;
    if (first ? a.c.omg[k] != a.c.omg[1] : a.c.omg[k] != R(1)) return false;
  }
  return true;
}

template <class L, class R, int UP>
hipError_t launch_up(const StepArgs<R>& a, const double* T_init, int mode, hipStream_t s) {
  const int bx = a.nx >= 256 ? 256 : (a.nx >= 128 ? 128 : 64);
  const int by = 256 / bx;
  const dim3 block(bx, by, 1);
  const dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
  if (mode == 1) {
    init_kernel<L, R, UP><<<grid, block, 0, s>>>(a, T_init);
    return hipGetLastError();
  }
  const double state_bytes = (double)a.plane * (L::Qf + L::Qg) * sizeof(R);
  const bool nt = state_bytes > 128.0 * 1024 * 1024;
  const bool std_rates = standard_rates(a, L::D);
  if (state_bytes < 4294967296.0) {
    const unsigned tb = (unsigned)state_bytes;
    if (nt) {
      if (std_rates)
        step_kernel<L, R, Buf32<R>, UP, true, true><<<grid, block, 0, s>>>(a, tb);
      else
        step_kernel<L, R, Buf32<R>, UP, true, false><<<grid, block, 0, s>>>(a, tb);
    } else {
      if (std_rates)
        step_kernel<L, R, Buf32<R>, UP, false, true><<<grid, block, 0, s>>>(a, tb);
      else
        step_kernel<L, R, Buf32<R>, UP, false, false><<<grid, block, 0, s>>>(a, tb);
    }
  } else {
    if (std_rates)
      step_kernel<L, R, Glob64<R>, UP, true, true><<<grid, block, 0, s>>>(a, 0u);
    else
      step_kernel<L, R, Glob64<R>, UP, true, false><<<grid, block, 0, s>>>(a, 0u);
  }
  return hipGetLastError();
}

}  // namespace

template <class R>
hipError_t launch_step2d(const StepArgs<R>& a, int up, const double* T_init, int mode, hipStream_t s) {
  return up == 0 ? launch_up<Lat2, R, 0>(a, T_init, mode, s) : launch_up<Lat2, R, 1>(a, T_init, mode, s);
}

template <class R>
hipError_t launch_step3d(const StepArgs<R>& a, int up, const double* T_init, int mode, hipStream_t s) {
  switch (up) {
    case 0: return launch_up<Lat3, R, 0>(a, T_init, mode, s);
    case 1: return launch_up<Lat3, R, 1>(a, T_init, mode, s);
    default: return launch_up<Lat3, R, 2>(a, T_init, mode, s);
  }
}

template hipError_t launch_step2d<double>(const StepArgs<double>&, int, const double*, int, hipStream_t);
template hipError_t launch_step2d<float>(const StepArgs<float>&, int, const double*, int, hipStream_t);
template hipError_t launch_step3d<double>(const StepArgs<double>&, int, const double*, int, hipStream_t);
template hipError_t launch_step3d<float>(const StepArgs<float>&, int, const double*, int, hipStream_t);

}  // namespace fpc
