// Streaming access shared by the forward step and the adjoint step.
//
// Forward (gather): each node pulls f_a(x) = f~_a(x - e_a) from the previous
// state (Eq. LBMsteps-stream, LBMsteps-streamg); where x - e_a lies beyond a
// wall face it applies the halfway wall rule at its own node (Sec. 6.1):
//   no-slip      f_a = f~_abar
//   moving wall  f_a = f~_abar + 2 w_a rho_w (e_a . u_w) / c_s^2
//   adiabatic    g_a = g~_abar
//   Dirichlet    g_a = -g~_abar + 2 w^T_a T_w
// Adjoint: the transpose of that selection, taken as a pull in the opposite
// direction (Rev below): the adjoint of stored slot (x, a) is that of the
// incoming link it feeds, (x + e_a, a), or across a wall face the node's own
// (x, abar), with the factor -1 of the Dirichlet rule.
//
// Layout: tiles of 64 nodes (below); a wavefront owns one tile, so every
// access is a contiguous run of 64 values of one population of one tile
// (shifted by at most one element into the neighbouring tile).
//
// Boundary handling is resolved per wavefront by the caller (a ballot over
// the edge tests) and compiled in: CX / CY / CZ enable the range checks of an
// axis; PX states that x is periodic (x-edge waves then only wrap).  Checked
// links stay branch-free: a wall redirects the single access of the link to
// the node's own opposite slot.
#pragma once

#include "fpc_kernels.h"

namespace fpc {
namespace stream {

// Lattice pairs: fluid links (ex, ey, ez, opp, w) and thermal links (tex,
// tey, tez, topp, wT with the runtime diffusion parameter c = c^_s^2).
struct Lat2 {  // D2Q9 + D2Q5
  static constexpr int D = 2, Qf = kQ2, Qg = kQ2T;
  static constexpr int ex(int a) { return D2_EX[a]; }
  static constexpr int ey(int a) { return D2_EY[a]; }
  static constexpr int ez(int) { return 0; }
  static constexpr int opp(int a) { return D2_OPP[a]; }
  static constexpr double w(int a) { return w2(a); }
  static constexpr int tex(int a) { return D2_EX[a]; }
  static constexpr int tey(int a) { return D2_EY[a]; }
  static constexpr int tez(int) { return 0; }
  static constexpr int topp(int a) { return D2_OPP[a]; }
  template <class R>
  static __device__ __forceinline__ R wT(int a, R c) { return a == 0 ? R(1) - R(2) * c : R(0.5) * c; }
};

struct Lat2T9 : Lat2 {  // D2Q9 + D2Q9
  static constexpr int Qg = kQ2;
  template <class R>
  static __device__ __forceinline__ R wT(int a, R c) {
    const R w0 = R(1) - c, w1 = R(0.5) * c;
    return (D2_EX[a] == 0 ? w0 : w1) * (D2_EY[a] == 0 ? w0 : w1);
  }
};

struct Lat3 {  // D3Q27 + D3Q7
  static constexpr int D = 3, Qf = kQ3, Qg = kQ3T;
  static constexpr int ex(int a) { return D3_EX[a]; }
  static constexpr int ey(int a) { return D3_EY[a]; }
  static constexpr int ez(int a) { return D3_EZ[a]; }
  static constexpr int opp(int a) { return d3_opp(a); }
  static constexpr double w(int a) { return w3(a); }
  static constexpr int tex(int a) { return D3_EX[a]; }
  static constexpr int tey(int a) { return D3_EY[a]; }
  static constexpr int tez(int a) { return D3_EZ[a]; }
  static constexpr int topp(int a) { return d3_opp(a); }
  template <class R>
  static __device__ __forceinline__ R wT(int a, R c) { return a == 0 ? R(1) - R(3) * c : R(0.5) * c; }
};

struct Lat3T15 : Lat3 {  // D3Q27 + D3Q15
  static constexpr int Qg = kQ15;
  static constexpr int tex(int a) { return T15_EX[a]; }
  static constexpr int tey(int a) { return T15_EY[a]; }
  static constexpr int tez(int a) { return T15_EZ[a]; }
  static constexpr int topp(int a) { return t15_opp(a); }
  template <class R>
  static __device__ __forceinline__ R wT(int a, R c) {
    return a == 0 ? R(1) - R(3) * c + R(2) * c * c : (a <= 6 ? R(0.5) * (c - c * c) : R(0.125) * c * c);
  }
};

// The same lattice pair with every link reversed (e -> -e; slots, opposite
// slots and weights unchanged).  A pull on Rev<L> reads x + e_a, and a link
// whose x + e_a lies beyond a wall face takes the node's own opposite slot:
// the transpose of the selection made by the pull on L.
template <class L>
struct Rev : L {
  static constexpr int ex(int a) { return -L::ex(a); }
  static constexpr int ey(int a) { return -L::ey(a); }
  static constexpr int ez(int a) { return -L::ez(a); }
  static constexpr int tex(int a) { return -L::tex(a); }
  static constexpr int tey(int a) { return -L::tey(a); }
  static constexpr int tez(int a) { return -L::tez(a); }
};

// link components of the fluid (TH = false) or thermal (TH = true) lattice
template <class L, bool TH>
constexpr int lex(int a) { return TH ? L::tex(a) : L::ex(a); }
template <class L, bool TH>
constexpr int ley(int a) { return TH ? L::tey(a) : L::ey(a); }
template <class L, bool TH>
constexpr int lez(int a) { return TH ? L::tez(a) : L::ez(a); }
template <class L, bool TH>
constexpr int lopp(int a) { return TH ? L::topp(a) : L::opp(a); }

// Padded node index: rows hold nxp = nx rounded up to 64 nodes.
__device__ __forceinline__ unsigned node_of(int x, int y, int z, int nxp, int ny) {
  return ((unsigned)z * (unsigned)ny + (unsigned)y) * (unsigned)nxp + (unsigned)x;
}

// ---------------------------------------------------------------------------
// Storage layout of a state buffer (and of an adjoint state): nodes are
// grouped in tiles of 64 consecutive padded node indices (64 consecutive x of
// one row; rows are padded to whole tiles).  A tile stores its Q = Qf + Qg
// populations one after the other, each as a run of 64 values, so population
// q of node n is element
//     elem(q, n) = (tile(n) Q + q) 64 + lane(n),  tile = n / 64, lane = n % 64.
// A wavefront owns exactly one tile: its stores fill Q * 64 contiguous values,
// and each pulled population is a run of 64 values of one source tile
// (straddling two tiles by one element for e_x != 0).
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ unsigned elem(int q, unsigned n) {
  return ((n >> 6) * (unsigned)Q + (unsigned)q) * 64u + (n & 63u);
}
template <int Q>
__device__ __forceinline__ size_t elem64(int q, unsigned n) {
  return ((size_t)(n >> 6) * (unsigned)Q + (unsigned)q) * 64u + (n & 63u);
}

// Interior fast path of a pull along e = (ex, ey, ez): the source of lane l
// lies in tile t - dt (dt = ey nxp/64 + ez ny nxp/64, wave-uniform) at lane
// l - ex, or across the tile border for the first / last lane.  Relative to a
// base tile that is wave-uniform, the lane's element offset is a per-lane
// constant, precomputed once:
//   ex =  0: base t - dt,     lane offset l
//   ex = +1: base t - dt - 1, lane offset 63 (l = 0) or Q 64 + l - 1
//   ex = -1: base t - dt,     lane offset Q 64 (l = 63) or l + 1
// (all non-negative; used only for waves with no x-edge lane, so the border
// tiles exist in the same row).
template <int Q>
struct TileLanes {
  unsigned t;       // tile of the wave (wave-uniform)
  unsigned o0, op, om;  // lane element offsets for ex = 0, +1, -1
  __device__ __forceinline__ explicit TileLanes(unsigned node) {
    t = __builtin_amdgcn_readfirstlane(node >> 6);
    const unsigned l = node & 63u;
    o0 = l;
    op = l == 0 ? 63u : (unsigned)Q * 64u + l - 1u;
    om = l == 63 ? (unsigned)Q * 64u : l + 1u;
  }
  template <int EX>
  __device__ __forceinline__ unsigned base(int dt) const { return t - (unsigned)dt - (EX > 0 ? 1u : 0u); }
  template <int EX>
  __device__ __forceinline__ unsigned lane() const { return EX == 0 ? o0 : (EX > 0 ? op : om); }
};

// ---------------------------------------------------------------------------
// Addressing of a pair of buffers in the storage layout (read side `src`,
// write side `dst`).  Two policies with the same interface:
//   load(q, shift, idx)               population q of padded node idx - shift
//   load_sel(w, qw, iw, q, shift, idx)  per lane: (qw, iw) if w, else as load
//   load_tile(q, tb, lane)            interior fast path (TileLanes)
//   cursor(n) / store_next<NT>(cur, v)  the Q populations of node n in order
//   store_at(q, shift, idx, v), store_sel(...), store_tile(q, tb, lane, v)
// Buf32: each buffer through one raw buffer descriptor (below 4 GiB); the
//   interior path passes the lane offset in a vector register and the tile
//   offset as a wave-uniform scalar, so it costs no vector ALU.
// Glob64: 64-bit element offsets (any size).
// ---------------------------------------------------------------------------
constexpr int kBufDword3 = 0x00020000;  // raw (untyped) buffer, gfx9 family
// Cache-policy bits of the ordinary (not non-temporal) state stores, per
// element type (launch tuning, measured): FP64 states store with sc1 (2D FP64
// step -2.3%, 3D FP64 64^3 step -10%), FP32 states with the default policy
// (sc1 measured 1-5% slower there).
#ifndef FPC_STORE_AUX_F64
#define FPC_STORE_AUX_F64 16  // sc1
#endif
#ifndef FPC_STORE_AUX_F32
#define FPC_STORE_AUX_F32 0
#endif
// Non-temporal stores (states above the last-level cache) carry sc1 as well
// (-0.2% to -0.8% on every such state, same-box A/B).  Loads keep the default
// policy (nt loads measured 3-24% slower, sc1 loads no faster).
#ifndef FPC_STORE_AUX_NT
#define FPC_STORE_AUX_NT 18  // nt | sc1
#endif
#ifndef FPC_LOAD_AUX
#define FPC_LOAD_AUX 0
#endif
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// LAUX: cache policy of the loads (the multi-step kernel reads the previous
// step with device-scope loads, which miss the per-CU L1: another CU of the
// same XCD may have written the line since).
template <class R, int Q, int LAUX = FPC_LOAD_AUX>
struct Buf32 {
  __amdgpu_buffer_rsrc_t rsrc_s, rsrc_d;
  static constexpr unsigned S = sizeof(R);

  __device__ __forceinline__ Buf32(const R* s, R* d, unsigned total_bytes)
      : rsrc_s(__builtin_amdgcn_make_buffer_rsrc(const_cast<R*>(s), 0, (int)total_bytes, kBufDword3)),
        rsrc_d(__builtin_amdgcn_make_buffer_rsrc(d, 0, (int)total_bytes, kBufDword3)) {}

  __device__ __forceinline__ R raw(unsigned voff, unsigned soff) const {
    if constexpr (sizeof(R) == 4)
      return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rsrc_s, (int)voff, (int)soff, LAUX));
    else
      return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rsrc_s, (int)voff, (int)soff, LAUX));
  }
  template <bool NT>
  __device__ __forceinline__ void raw_store(unsigned voff, unsigned soff, R v) const {
    // cache policy: non-temporal, else the element type's ordinary policy
    constexpr int aux = NT ? FPC_STORE_AUX_NT : (sizeof(R) == 8 ? FPC_STORE_AUX_F64 : FPC_STORE_AUX_F32);
    if constexpr (sizeof(R) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rsrc_d, (int)voff, (int)soff, aux);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rsrc_d, (int)voff, (int)soff, aux);
  }
  __device__ __forceinline__ R load(int q, long long shift, unsigned idx) const {
    return raw(elem<Q>(q, idx - (unsigned)shift) * S, 0u);
  }
  __device__ __forceinline__ R load_sel(bool w, int qw, unsigned iw, int q, long long shift, unsigned idx) const {
    return raw((w ? elem<Q>(qw, iw) : elem<Q>(q, idx - (unsigned)shift)) * S, 0u);
  }
  __device__ __forceinline__ R load_tile(int q, unsigned tb, unsigned lane) const {
    return raw(lane * S, (tb * (unsigned)Q + (unsigned)q) * 64u * S);
  }
  __device__ __forceinline__ unsigned cursor(unsigned n) const { return elem<Q>(0, n) * S; }
  template <bool NT>
  __device__ __forceinline__ void store_next(unsigned& cur, R v) const {
    raw_store<NT>(cur, 0u, v);
    cur += 64u * S;
  }
  __device__ __forceinline__ void store_at(int q, long long shift, unsigned idx, R v) const {
    raw_store<false>(elem<Q>(q, idx - (unsigned)shift) * S, 0u, v);
  }
  __device__ __forceinline__ void store_sel(bool w, int qw, unsigned iw, int q, long long shift, unsigned idx,
                                            R v) const {
    raw_store<false>((w ? elem<Q>(qw, iw) : elem<Q>(q, idx - (unsigned)shift)) * S, 0u, v);
  }
  __device__ __forceinline__ void store_tile(int q, unsigned tb, unsigned lane, R v) const {
    raw_store<false>(lane * S, (tb * (unsigned)Q + (unsigned)q) * 64u * S, v);
  }
};

template <class R, int Q>
struct Glob64 {
  const R* src;
  R* dst;

  __device__ __forceinline__ Glob64(const R* s, R* d, unsigned) : src(s), dst(d) {}

  __device__ __forceinline__ R load(int q, long long shift, unsigned idx) const {
    return src[elem64<Q>(q, idx - (unsigned)shift)];
  }
  __device__ __forceinline__ R load_sel(bool w, int qw, unsigned iw, int q, long long shift, unsigned idx) const {
    return src[w ? elem64<Q>(qw, iw) : elem64<Q>(q, idx - (unsigned)shift)];
  }
  __device__ __forceinline__ R load_tile(int q, unsigned tb, unsigned lane) const {
    return src[((size_t)tb * (unsigned)Q + (unsigned)q) * 64u + lane];
  }
  __device__ __forceinline__ R* cursor(unsigned n) const { return dst + elem64<Q>(0, n); }
  template <bool NT>
  __device__ __forceinline__ void store_next(R*& cur, R v) const {
    if constexpr (NT)
      __builtin_nontemporal_store(v, cur);
    else
      *cur = v;
    cur += 64;
  }
  __device__ __forceinline__ void store_at(int q, long long shift, unsigned idx, R v) const {
    dst[elem64<Q>(q, idx - (unsigned)shift)] = v;
  }
  __device__ __forceinline__ void store_sel(bool w, int qw, unsigned iw, int q, long long shift, unsigned idx,
                                            R v) const {
    dst[w ? elem64<Q>(qw, iw) : elem64<Q>(q, idx - (unsigned)shift)] = v;
  }
  __device__ __forceinline__ void store_tile(int q, unsigned tb, unsigned lane, R v) const {
    dst[((size_t)tb * (unsigned)Q + (unsigned)q) * 64u + lane] = v;
  }
};

// ---------------------------------------------------------------------------
// Per-lane edge state of one node and the source slot of each link.
// ---------------------------------------------------------------------------
template <class L, class R, bool CX, bool CY, bool CZ, bool PX>
struct Edges {
  const StepArgs<R>& a;
  unsigned node;
  // Lane on the low / high edge of a checked axis.  A link with e_k = +1
  // crossing the low edge (or e_k = -1 crossing the high edge) either wraps
  // (periodic axis: the source index moves by +-n_k times the axis stride) or
  // meets a wall.  PX: x is known to be periodic.
  bool xlo = false, xhi = false, ylo = false, yhi = false, zlo = false, zhi = false;
  unsigned wxm = 0, wxp = 0;  // node index with the x wrap of an e_x = -1 / +1 link applied
  TileLanes<L::Qf + L::Qg> tl;  // interior fast path

  __device__ __forceinline__ Edges(const StepArgs<R>& a_, int x, int y, int z, unsigned node_)
      : a(a_), node(node_), tl(node_) {
    if (CX) {
      xlo = x == 0;
      xhi = x == a.nx - 1;
      wxp = node + (xlo ? (unsigned)a.nx : 0u);
      wxm = node - (xhi ? (unsigned)a.nx : 0u);
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

  template <int A, bool TH>
  static constexpr bool checked() {
    return (CX && lex<L, TH>(A) != 0) || (CY && ley<L, TH>(A) != 0) || (CZ && lez<L, TH>(A) != 0);
  }
  // padded-index offset of the source of link A (strides 1, nxp, nxp ny)
  template <int A, bool TH>
  __device__ __forceinline__ long long shift() const {
    return (long long)lex<L, TH>(A) + (long long)ley<L, TH>(A) * a.nxp + (long long)lez<L, TH>(A) * a.nxp * a.ny;
  }
  // the same in whole tiles, without the x component (wave-uniform)
  template <int A, bool TH>
  __device__ __forceinline__ int dtile() const {
    const int rt = a.nxp >> 6;  // tiles per row
    return ley<L, TH>(A) * rt + lez<L, TH>(A) * rt * a.ny;
  }
  // Checked link A: the wrapped source index (used with shift()) and the
  // axes on which the link meets a wall.
  template <int A, bool TH>
  __device__ __forceinline__ unsigned source(bool& wx, bool& wy, bool& wz) const {
    constexpr int ex = lex<L, TH>(A), ey = ley<L, TH>(A), ez = lez<L, TH>(A);
    constexpr bool cx = CX && ex != 0, cy = CY && ey != 0, cz = CZ && ez != 0;
    const bool ox = cx && (ex > 0 ? xlo : xhi);
    const bool oy = cy && (ey > 0 ? ylo : yhi);
    const bool oz = cz && (ez > 0 ? zlo : zhi);
    unsigned idx = cx ? (ex > 0 ? wxp : wxm) : node;
    if (cy) idx += oy ? (unsigned)(ey * a.ny) * (unsigned)a.nxp : 0u;
    if (cz) idx += oz ? (unsigned)(ez * a.nz) * (unsigned)a.nxp * (unsigned)a.ny : 0u;
    wx = ox && !PX && !a.per[0];
    wy = oy && !a.per[1];
    wz = oz && !a.per[2];
    return idx;
  }
  // only periodic wraps are possible on this link (no wall test needed)
  template <int A, bool TH>
  static constexpr bool wrap_only() {
    return PX && !(CY && ley<L, TH>(A) != 0) && !(CZ && lez<L, TH>(A) != 0);
  }
};

// ---------------------------------------------------------------------------
// Gather: the incoming (pre-collision) populations of one node, in storage
// form relative to this node's references.
// ---------------------------------------------------------------------------
// e . t for a compile-time link e, summing only its non-zero components
// (a zero component times t would still cost an IEEE multiply-add).
template <int EX, int EY, int EZ, class R>
__device__ __forceinline__ R edot(const R (&t)[3]) {
  R d = R(0);  // the rest link (never used for it)
  bool any = false;
  if constexpr (EX != 0) {
    d = R(EX) * t[0];
    any = true;
  }
  if constexpr (EY != 0) {
    d = any ? d + R(EY) * t[1] : R(EY) * t[1];
    any = true;
  }
  if constexpr (EZ != 0) d = any ? d + R(EZ) * t[2] : R(EZ) * t[2];
  return d;
}

template <class L, class R, class M, bool CX, bool CY, bool CZ, bool PX>
struct Gather {
  using E = Edges<L, R, CX, CY, CZ, PX>;
  const StepArgs<R>& a;
  const M& m;
  E e;
  int x, y, z;
  R Tr;  // thermal storage reference of this node

  __device__ __forceinline__ Gather(const StepArgs<R>& a_, const M& m_, int x_, int y_, int z_, unsigned node_, R Tr_)
      : a(a_), m(m_), e(a_, x_, y_, z_, node_), x(x_), y(y_), z(z_), Tr(Tr_) {}

  // Incoming population of link A of the fluid (TH = false, populations from
  // 0) or thermal (TH = true, from Qf) distribution, pulled or bounced;
  // reports per axis whether the link met a wall there.
  template <int A, bool TH>
  __device__ __forceinline__ R pull(bool& wx, bool& wy, bool& wz) const {
    constexpr int QBASE = TH ? L::Qf : 0;
    constexpr int ex = lex<L, TH>(A);
    if (!E::template checked<A, TH>())
      return m.load_tile(QBASE + A, e.tl.template base<ex>(e.template dtile<A, TH>()), e.tl.template lane<ex>());
    const long long sh = e.template shift<A, TH>();
    const unsigned idx = e.template source<A, TH>(wx, wy, wz);
    if (E::template wrap_only<A, TH>()) return m.load(QBASE + A, sh, idx);
    const bool wall = wx || wy || wz;
    return m.load_sel(wall, QBASE + lopp<L, TH>(A), e.node, QBASE + A, sh, idx);
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
    R v = pull<A, false>(wx, wy, wz);
    constexpr int ex = L::ex(A), ey = L::ey(A), ez = L::ez(A);
    if (E::template checked<A, false>()) {
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

  // Dirichlet temperature of face F at this node (uniform or per-node profile)
  template <int F>
  __device__ __forceinline__ double wall_T() const {
    constexpr int k = F >> 1;
    double Tw = a.face[F].Tw;
    if (a.face[F].Tprof) {
      const size_t t = k == 0 ? (size_t)z * a.ny + y : (k == 1 ? (size_t)z * a.nx + x : (size_t)y * a.nx + x);
      Tw = a.face[F].Tprof[t];
    }
    return Tw;
  }

  // Thermal link A.  A wall link is bounced back; if any face it crosses is a
  // Dirichlet face it is anti-bounced toward the mean of those faces'
  // temperatures (axis links cross one face; diagonal links of D2Q9 / D3Q15
  // can cross two or three at edges and corners).
  template <int A>
  __device__ __forceinline__ R g() const {
    bool wx = false, wy = false, wz = false;
    R v = pull<A, true>(wx, wy, wz);
    if (A == 0) return v;
    constexpr int ex = L::tex(A), ey = L::tey(A), ez = L::tez(A);
    constexpr int FX = ex > 0 ? 0 : 1, FY = ey > 0 ? 2 : 3, FZ = ez > 0 ? 4 : 5;
    constexpr int nax = (ex != 0) + (ey != 0) + (ez != 0);
    const R wa = L::template wT<R>(A, a.c.cs2T);
    const bool wall = E::template checked<A, true>() && (wx || wy || wz);
    if (wall) {
      double tsum = 0.0;
      int nd = 0;
      if (ex != 0 && wx && a.face[FX].dirichlet) {
        tsum += wall_T<FX>();
        ++nd;
      }
      if (ey != 0 && wy && a.face[FY].dirichlet) {
        tsum += wall_T<FY>();
        ++nd;
      }
      if (ez != 0 && wz && a.face[FZ].dirichlet) {
        tsum += wall_T<FZ>();
        ++nd;
      }
      if (nd > 0) {
        const double Tw = nax == 1 ? tsum : tsum / nd;
        v = -v + R(2) * wa * (R(Tw) - Tr);  // 2 w^T_a T_w, in storage form
      }
    } else if constexpr (kDeviations<R>) {
      // the value was stored against the source node's reference Tr(x - e_A)
      v -= wa * edot<ex, ey, ez>(a.Tg);
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
  } else {
#define FPC_F(A) f[A] = p.template f<A>();
    FPC_F(0) FPC_F(1) FPC_F(2) FPC_F(3) FPC_F(4) FPC_F(5) FPC_F(6) FPC_F(7) FPC_F(8)
    FPC_F(9) FPC_F(10) FPC_F(11) FPC_F(12) FPC_F(13) FPC_F(14) FPC_F(15) FPC_F(16) FPC_F(17)
    FPC_F(18) FPC_F(19) FPC_F(20) FPC_F(21) FPC_F(22) FPC_F(23) FPC_F(24) FPC_F(25) FPC_F(26)
#undef FPC_F
  }
#define FPC_G(A) if constexpr (A < L::Qg) g[A] = p.template g<A>();
  FPC_G(0) FPC_G(1) FPC_G(2) FPC_G(3) FPC_G(4) FPC_G(5) FPC_G(6) FPC_G(7)
  FPC_G(8) FPC_G(9) FPC_G(10) FPC_G(11) FPC_G(12) FPC_G(13) FPC_G(14)
#undef FPC_G
}

}  // namespace stream
}  // namespace fpc
