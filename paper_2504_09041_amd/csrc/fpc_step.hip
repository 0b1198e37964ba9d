// Fused pull-stream + collide kernel (D2Q9 + D2Q5 and D3Q27 + D3Q7).
//
// One thread per node.  Each thread gathers its incoming populations from
// S_{n-1} with the wall rules applied at its own node (fpc_gather.h), collides
// in registers (fpc_collide.h) and stores its own values to S_n.
//
// A wavefront owns one 64-node tile of the storage layout (blocks are whole
// multiples of 64 along x, rows are padded to whole tiles).  Boundary handling
// is resolved per wavefront: a ballot tells whether any lane of the wave sits
// on an x, y or z edge of the box, and the gather is instantiated with range
// checks only on those axes.  Interior wavefronts (the vast majority) load
// every population from a wave-uniform tile offset plus a per-lane constant
// and no checks at all; x-edge wavefronts of a periodic x axis only wrap.
//
// Stores are non-temporal when the state is too large to stay in the
// last-level cache (it then streams through HBM anyway); smaller states keep
// ordinary stores so that the next step reads them from the cache.
#include "fpc_gather.h"



// Launch tuning (compile-time): widest block along x, state size above which
// stores are non-temporal, optional extra kernel attributes.
#ifndef FPC_BLOCK_2D
#define FPC_BLOCK_2D 256  // threads per block of the 2D kernels
#endif
#ifndef FPC_BLOCK_3D
#define FPC_BLOCK_3D 256  // threads per block of the 3D FP64 step kernels
#endif
#ifndef FPC_BLOCK_3DF
#define FPC_BLOCK_3DF 128  // threads per block of the 3D FP32 step kernels (128^3: -0.7% against 256)
#endif

#ifndef FPC_BLOCK_X_MAX
#define FPC_BLOCK_X_MAX 256
#endif
#ifndef FPC_NT_MIB
#define FPC_NT_MIB 128
#endif
#ifndef FPC_STEP_ATTR
#define FPC_STEP_ATTR
#endif

static_assert(FPC_BLOCK_X_MAX % 64 == 0, "a wavefront must cover one whole 64-node tile");
static_assert(FPC_BLOCK_2D % 64 == 0 && FPC_BLOCK_2D >= 64 && FPC_BLOCK_2D <= 1024, "2D block size");
static_assert(FPC_BLOCK_3D % 64 == 0 && FPC_BLOCK_3D >= 64 && FPC_BLOCK_3D <= 1024, "3D block size");
static_assert(FPC_BLOCK_3DF % 64 == 0 && FPC_BLOCK_3DF >= 64 && FPC_BLOCK_3DF <= 1024, "3D FP32 block size");

namespace fpc {
namespace {

using namespace stream;

// Lane l's value of a double (any lane, active or not).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Fused wall-Nusselt accumulation (StepArgs::obj): a node in the layer next
// to the face (the stencil's T(1/2)) adds scale (3 T - 8/3 T_w), a node in the
// second layer (T(3/2)) adds scale (-T / 3), with T the time-level
// temperature of the stored post-collision populations (Sec. 6.1 stencil,
// Nu = -(L / dT) dT/dn).  The wavefront sums its lanes in a fixed order and
// adds the sum to the slot of its tile.
template <class L, class R>
__device__ __forceinline__ void nu_accumulate(const StepArgs<R>& a, int x, int y, int z, double t) {
  // (axis lengths come from NuAcc: a select between fields of the kernel
  // argument would make the compiler keep a private copy of it)
  const NuAcc& o = a.obj;
  const int k = o.face >> 1;
  const int c = k == 0 ? x : (k == 1 ? y : z);
  const int layer = (o.face & 1) ? o.nk - 1 - c : c;
  const bool in = layer <= 1;
  if (!__any(in)) return;
  double v = 0.0;
  if (in) {
    const double T = (o.T_o + (o.Tg[0] * (double)x + o.Tg[1] * (double)y + o.Tg[2] * (double)z)) + t;
    if (layer == 0) {
      const size_t i = (size_t)(k == 2 ? y : z) * o.nt + (k == 0 ? y : x);
      const double Tw = o.Tprof ? o.Tprof[i] : o.Tw;
      v = o.scale * (3.0 * T - (8.0 / 3.0) * Tw);
    } else {
      v = o.scale * (-T / 3.0);
    }
  }
  // sum over the wavefront in a fixed order: a butterfly when every lane is
  // active, else lane by lane over the active lanes (a ragged last tile)
  const unsigned long long act = __ballot(1);
  double sum = v;
  if (act == ~0ull) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  } else {
    sum = 0.0;
    for (int l = 0; l < 64; ++l)
      if ((act >> l) & 1ull) sum += readlane_f64(v, l);
  }
  // slot of this wavefront's tile (x >> 6, y, z and, on y / z faces, the
  // layer are uniform over a wavefront)
  const int xt = x >> 6;
  const int nxt = a.nxp >> 6;
  size_t idx;
  if (k == 0) {
    const int xlo = (o.face & 1) ? o.nk - 2 : 0;
    idx = ((size_t)z * o.nt + y) * 2 + (size_t)(xt - (xlo >> 6));
  } else if (k == 1) {
    idx = ((size_t)z * 2 + layer) * nxt + xt;
  } else {
    idx = ((size_t)layer * o.ns + y) * nxt + xt;
  }
  // one add per slot and launch (the launches of a run are ordered on the
  // stream, so the per-slot sum has a fixed order); an atomic add needs no
  // return value, so the wavefront does not wait for the slot's old value
  if (__lane_id() == (unsigned)(__ffsll((long long)act) - 1)) atomicAdd(&o.slot[idx], sum);
}

// Sum (op 0) or max (op 1) of a double over the active lanes of the
// wavefront in a fixed order: a butterfly when every lane is active, else lane
// by lane over the active lanes (a ragged last tile).
__device__ __forceinline__ double wave_reduce(double v, int op) {
  const unsigned long long act = __ballot(1);
  if (act == ~0ull) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v, off);
      v = op == 0 ? v + o : fmax(v, o);
    }
    return v;
  }
  double r = op == 0 ? 0.0 : readlane_f64(v, __ffsll((long long)act) - 1);
  for (int l = 0; l < 64; ++l)
    if ((act >> l) & 1ull) r = op == 0 ? r + readlane_f64(v, l) : fmax(r, readlane_f64(v, l));
  return r;
}

// Fused diagnostics (StepArgs::dg): the per-node values fpc_diagnostics forms
// from the stored state (rho = rho_r + sum f, T = Tr + sum g, rho u = sum f e
// - F/2, in FP64 and in the same order), reduced over the wavefront's tile
// and written to the tile's four partials.
template <class L, class R, int UP>
__device__ __forceinline__ void diag_accumulate(const StepArgs<R>& a, int x, int y, int z, unsigned node,
                                                const R (&f)[L::Qf], const R (&g)[L::Qg]) {
  const DiagAcc& d = a.dg;
  double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int q = 0; q < L::Qf; ++q) {
    const double v = (double)f[q];
    s += v;
    jx += L::ex(q) * v;
    jy += L::ey(q) * v;
    jz += L::ez(q) * v;
  }
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < L::Qg; ++q) t += (double)g[q];
  const double rho = d.rho_r + s;
  const double T = (d.T_o + (d.Tg[0] * (double)x + d.Tg[1] * (double)y + d.Tg[2] * (double)z)) + t;
  const double Fb = d.gbeta * (T - d.T0);
  const double ir = 1.0 / rho;
  double u[3];
  u[0] = (jx - (UP == 0 ? 0.5 * Fb : 0.0)) * ir;
  u[1] = (jy - (UP == 1 ? 0.5 * Fb : 0.0)) * ir;
  u[2] = (jz - (UP == 2 ? 0.5 * Fb : 0.0)) * ir;
  const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double ke = 0.0, st = 0.0, um = 0.0, bad = 0.0;
  if (!isfinite(rho) || !isfinite(T) || !isfinite(u2)) {
    bad = 1.0;
  } else {
    ke = 0.5 * rho * u2;
    st = T;
    um = sqrt(u2);
  }
  ke = wave_reduce(ke, 0);
  st = wave_reduce(st, 0);
  um = wave_reduce(um, 1);
  bad = wave_reduce(bad, 0);
  if (__lane_id() == (unsigned)(__ffsll((long long)__ballot(1)) - 1)) {
    double* p = d.part + (size_t)(node >> 6) * 4;
    p[0] = ke;
    p[1] = st;
    p[2] = um;
    p[3] = bad;
  }
}

// HOOKS: the optional fused wall-Nusselt and diagnostics hooks (absent from
// the multi-step kernel, which never takes them)
template <class L, class R, class M, int UP, bool NT, bool STD, bool HOOKS = true>
__device__ __forceinline__ void collide_store(const StepArgs<R>& a, const M& m, int x, int y, int z, unsigned node,
                                              R Tr, R (&f)[L::Qf], R (&g)[L::Qg]) {
  if constexpr (L::D == 2)
    collide2d<R, UP, STD, L::Qg>(f, g, a.c, Tr, (Macros<R>*)nullptr);
  else
    collide3d<R, UP, STD, L::Qg>(f, g, a.c, Tr, (Macros<R>*)nullptr);
  auto cur = m.cursor(node);
#pragma unroll
  for (int q = 0; q < L::Qf; ++q) m.template store_next<NT>(cur, f[q]);
#pragma unroll
  for (int q = 0; q < L::Qg; ++q) m.template store_next<NT>(cur, g[q]);
  // the fused wall-Nusselt accumulation needs only the sum of the stored
  // thermal values; it is formed after the stores, so that its branch does
  // not split the collision (and its scheduling) in two
  if constexpr (HOOKS) {
    if (a.obj.slot != nullptr) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < L::Qg; ++q) t += (double)g[q];
      nu_accumulate<L, R>(a, x, y, z, t);
    }
    if (a.dg.part != nullptr) diag_accumulate<L, R, UP>(a, x, y, z, node, f, g);
  }
}


// One node's update: pull S_{n-1} (m's source), collide, store S_n (m's
// destination).  Lanes outside the box must not call it (the edge ballots
// count the calling lanes only).
template <class L, class R, class M, int UP, bool NT, bool STD, bool HOOKS = true>
__device__ __forceinline__ void step_node(const StepArgs<R>& a, const M& m, int x, int y, int z) {
  const unsigned node = node_of(x, y, z, a.nxp, a.ny);
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
  collide_store<L, R, M, UP, NT, STD, HOOKS>(a, m, x, y, z, node, Tr, f, g);
}

// M: addressing policy (Buf32 when the buffer is below 4 GiB, else Glob64).
// STD: the standard rate set (see rate_f / rate_g).
template <class L, class R, class M, int UP, bool NT, bool STD>
__global__ void __launch_bounds__(L::D == 2 ? FPC_BLOCK_2D : (sizeof(R) == 4 ? FPC_BLOCK_3DF : FPC_BLOCK_3D)) FPC_STEP_ATTR
    step_kernel(StepArgs<R> a, unsigned total_bytes) {
  // XCD-aware block order: contiguous ranges of rows per XCD in 2D; in 3D
  // FP32, contiguous ranges of rows per XCD within each z plane (3D FP64
  // measured 2% slower with it, and 3D with whole z slabs per XCD 1-3%)
  const dim3 bi = block_order<L::D, sizeof(R)>();
  const int x = bi.x * blockDim.x + threadIdx.x;
  const int y = bi.y * blockDim.y + threadIdx.y;
  const int z = bi.z;
  if (x >= a.nx || y >= a.ny) return;
  const M m(a.src, a.dst, total_bytes);
  step_node<L, R, M, UP, NT, STD>(a, m, x, y, z);
}

// ---------------------------------------------------------------------------
// Several steps in one cooperative launch (small grids).
//
// On a grid of a few thousand nodes a step is a few microseconds of work, and
// a launch per step costs about as much again (ramp-up, drain and the cache
// maintenance between dependent launches).  This kernel runs nsteps steps in
// one launch: every working block updates the same nodes each step, ping-
// ponging between the two state buffers, and a grid-wide barrier separates
// the steps.  Only every kXcds-th block of the launch works: with workgroups
// dispatched round-robin over the XCDs, the working blocks then share one XCD
// and its L2.
//
// Two ways to separate the steps.  The full barrier brackets the arrival
// with agent-scope release / acquire fences (an L2 writeback and invalidate),
// which is correct wherever the blocks run.  The light one (multi_sync_light)
// only waits for the neighbour blocks, whose stores it reads, and reads the
// next step with device-scope loads, which miss the per-CU L1; that is enough
// when every working block runs on one XCD, whose L2 is then the point of
// coherence.  Each launch checks the placement: before a first, full barrier
// every working block ORs the bit of its XCD (hardware register XCC_ID) into
// a word of this launch, and after it every block reads the word; one bit
// set means one XCD and the light form for the rest of the launch, else the
// full barrier throughout.
//
// The full barrier's word is self-resetting: each arrival adds 1, except the
// first block, which adds 2^31 - (nwork - 1), so the top bit flips exactly
// when the last block arrives and the low bits return to zero.  The light
// form numbers its rounds (gen: unique per launch and step, increasing), so
// its words need no reset.  The placement words alternate between launches,
// and each launch clears the next one's.  A waiter gives up after spin_limit
// polls (co-residency is what the cooperative launch guarantees, so this only
// fires on a fault elsewhere): it sets *err and leaves, and every later wait
// and launch sees *err and leaves at once.  The host reports the flag at the
// next synchronising call.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 0xfu;  // hwreg(HW_REG_XCC_ID, 0, 4)
}

// Full barrier (any placement): agent-scope fences around one atomic
// arrival word.
__device__ __forceinline__ bool multi_barrier_full(const MultiCtl& c, unsigned lb) {
  __shared__ int ok;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const unsigned inc = lb == 0 ? 0x80000000u - (c.nwork - 1u) : 1u;
    const unsigned old = __hip_atomic_fetch_add(c.bar, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    unsigned spins = 0;
    while (((__hip_atomic_load(c.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ^ old) & 0x80000000u) == 0u) {
      if (++spins > c.spin_limit || __hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(c.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    ok = good;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok != 0;
}

// Light synchronisation (every working block on one XCD).  A step of a block
// reads only the nodes of the blocks around it (one node across each face,
// edge and corner, with the periodic wraps), and overwrites the buffer those
// blocks read in the previous step; so before step s + 1 a block waits only
// for its neighbour blocks to have finished step s.  Each block waits for its
// stores to reach the L2 and writes its own arrival word (the step's number,
// gen); the first wave then polls the arrival words of the neighbours, one
// lane each (dep: this lane's neighbour block, or -1), until each shows gen
// or later (a neighbour can be at most one step ahead).  The next step is
// read with device-scope loads, which miss the per-CU L1.
__device__ __forceinline__ bool multi_sync_light(const MultiCtl& c, unsigned lb, unsigned gen, int dep) {
  __shared__ int ok;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const unsigned tid = threadIdx.y * blockDim.x + threadIdx.x;
  if (tid == 0) __hip_atomic_store(c.arrive + lb, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (tid < 64) {  // the first wave
    int good = 1;
    unsigned spins = 0;
    for (;;) {
      bool here = true;
      if (dep >= 0) here = (int)(__hip_atomic_load(c.arrive + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - gen) >= 0;
      if (__all(here)) break;
      if (++spins > c.spin_limit || __hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (tid == 0) {
      if (!good) __hip_atomic_store(c.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ok = good;
    }
  }
  __syncthreads();
  return ok != 0;
}

// The neighbour block that lane `lane` (0..26: offsets -1..1 per axis) of the
// first wave watches, or -1 (itself, outside a walled axis, or lane >= 27).
__device__ __forceinline__ int multi_neighbour(unsigned lane, int bx, int by, int bz, int gx, int gy, int gz,
                                               const int (&per)[3]) {
  if (lane >= 27) return -1;
  const int d[3] = {(int)(lane % 3) - 1, (int)((lane / 3) % 3) - 1, (int)(lane / 9) - 1};
  if (d[0] == 0 && d[1] == 0 && d[2] == 0) return -1;
  int b[3] = {bx + d[0], by + d[1], bz + d[2]};
  const int g[3] = {gx, gy, gz};
  for (int k = 0; k < 3; ++k) {
    if (b[k] < 0 || b[k] >= g[k]) {
      if (!per[k]) return -1;
      b[k] = (b[k] + g[k]) % g[k];
    }
  }
  return (b[2] * gy + b[1]) * gx + b[0];
}

template <class L, class R, int UP, bool STD>
__global__ void __launch_bounds__(256) step_multi_kernel(StepArgs<R> a, unsigned total_bytes, MultiCtl c) {
  if (blockIdx.x % kXcds != 0) return;
  const unsigned lb = blockIdx.x / kXcds;  // logical block of the per-step grid
  const unsigned gx = (a.nx + blockDim.x - 1) / blockDim.x, gy = (a.ny + blockDim.y - 1) / blockDim.y;
  const int x = (int)((lb % gx) * blockDim.x + threadIdx.x);
  const int y = (int)(((lb / gx) % gy) * blockDim.y + threadIdx.y);
  const int z = (int)(lb / (gx * gy));
  const bool live = x < a.nx && y < a.ny;
  // device-scope loads: the previous step may have been written by another CU
  using M = Buf32<R, L::Qf + L::Qg, 16>;
  if (__hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  __shared__ int light;
  const bool t0 = threadIdx.x == 0 && threadIdx.y == 0;
  unsigned* const place = c.place + (c.seq & 1);
  if (t0) {
    if (lb == 0) __hip_atomic_store(c.place + ((c.seq + 1) & 1), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_or(place, 1u << xcc_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!multi_barrier_full(c, lb)) return;
  if (t0) {
    const unsigned mask = __hip_atomic_load(place, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    light = (mask & (mask - 1u)) == 0u;
  }
  __syncthreads();
  const bool one_xcd = light != 0;
  const unsigned tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int dep = multi_neighbour(tid, (int)(lb % gx), (int)((lb / gx) % gy), z, (int)gx, (int)gy, a.nz, a.per);
  for (int s = 0; s < c.nsteps; ++s) {
    if (live) {
      // the node's coordinates pass through an empty asm so that what the
      // step derives from them is recomputed every step instead of being
      // hoisted out of the loop and held in registers across it
      int xs = x, ys = y;
      asm volatile("" : "+v"(xs), "+v"(ys));
      const bool odd = s & 1;
      const M m(odd ? a.dst : a.src, odd ? const_cast<R*>(a.src) : a.dst, total_bytes);
      step_node<L, R, M, UP, false, STD, false>(a, m, xs, ys, z);
    }
    if (s + 1 < c.nsteps && !(one_xcd ? multi_sync_light(c, lb, c.gen + (unsigned)s, dep)
                                      : multi_barrier_full(c, lb)))
      return;
  }
}

// Initial state: the collision of f = w rho0, g = w^T T_init at every node.
template <class L, class R, int UP>
__global__ void __launch_bounds__(256) init_kernel(StepArgs<R> a, const double* __restrict__ T_init) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  using M = Glob64<R, L::Qf + L::Qg>;
  const M m(a.src, a.dst, 0u);
  const unsigned node = node_of(x, y, z, a.nxp, a.ny);
  R f[L::Qf], g[L::Qg];
  const R drw = a.rho_w - a.c.rho_r;
#pragma unroll
  for (int q = 0; q < L::Qf; ++q) f[q] = R(L::w(q)) * drw;
  const R Tr = tref(a, x, y, z);
  const R dT = R(T_init[((size_t)z * a.ny + y) * a.nx + x]) - Tr;
#pragma unroll
  for (int q = 0; q < L::Qg; ++q) g[q] = L::template wT<R>(q, a.c.cs2T) * dT;
  collide_store<L, R, M, UP, false, false>(a, m, x, y, z, node, Tr, f, g);
}

template <class L, class R, int UP>
hipError_t launch_up(const StepArgs<R>& a, const double* T_init, int mode, hipStream_t s) {
  const int threads =
      mode == 0 ? (L::D == 2 ? FPC_BLOCK_2D : (sizeof(R) == 4 ? FPC_BLOCK_3DF : FPC_BLOCK_3D)) : 256;
  int bx = a.nx >= FPC_BLOCK_X_MAX ? FPC_BLOCK_X_MAX : (a.nx >= 128 ? 128 : 64);
  if (bx > threads) bx = threads;
  const int by = threads / bx;  // >= 1: threads and bx are multiples of 64, bx <= threads
  const dim3 block(bx, by, 1);
  const dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
  if (mode == 1) {
    init_kernel<L, R, UP><<<grid, block, 0, s>>>(a, T_init);
    return hipGetLastError();
  }
  const double state_bytes = (double)a.nxp * a.ny * a.nz * (L::Qf + L::Qg) * sizeof(R);
  using B32 = Buf32<R, L::Qf + L::Qg>;
  using G64 = Glob64<R, L::Qf + L::Qg>;
  const bool nt = state_bytes > FPC_NT_MIB * 1024.0 * 1024.0;
  const bool std_rates = standard_rates(a, L::D, L::Qg);
  if (state_bytes < 4294967296.0) {
    const unsigned tb = (unsigned)state_bytes;
    if (nt) {
      if (std_rates)
        step_kernel<L, R, B32, UP, true, true><<<grid, block, 0, s>>>(a, tb);
      else
        step_kernel<L, R, B32, UP, true, false><<<grid, block, 0, s>>>(a, tb);
    } else {
      if (std_rates)
        step_kernel<L, R, B32, UP, false, true><<<grid, block, 0, s>>>(a, tb);
      else
        step_kernel<L, R, B32, UP, false, false><<<grid, block, 0, s>>>(a, tb);
    }
  } else {
    if (std_rates)
      step_kernel<L, R, G64, UP, true, true><<<grid, block, 0, s>>>(a, 0u);
    else
      step_kernel<L, R, G64, UP, true, false><<<grid, block, 0, s>>>(a, 0u);
  }
  return hipGetLastError();
}

template <class L, class R, int UP>
hipError_t launch_multi_up(const StepArgs<R>& a, const MultiCtl& c0, hipStream_t s) {
  const int bx = a.nx >= 256 ? 256 : (a.nx >= 128 ? 128 : 64);
  const int by = 256 / bx;
  MultiCtl c = c0;
  c.nwork = multi_work_blocks(a.nx, a.ny, a.nz);
  StepArgs<R> args = a;
  unsigned tb = (unsigned)((double)a.nxp * a.ny * a.nz * (L::Qf + L::Qg) * sizeof(R));
  void* kargs[] = {(void*)&args, (void*)&tb, (void*)&c};
  const dim3 grid(c.nwork * kXcds, 1, 1), block(bx, by, 1);
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&step_multi_kernel<L, R, UP, true>), grid, block,
                                    kargs, 0, s);
}

}  // namespace

// tk: thermal lattice, 0 = D2Q5 / D3Q7, 1 = the paper's D2Q9 / D3Q15
template <class R>
hipError_t launch_step2d(const StepArgs<R>& a, int up, int tk, const double* T_init, int mode, hipStream_t s) {
  if (tk == 0)
    return up == 0 ? launch_up<Lat2, R, 0>(a, T_init, mode, s) : launch_up<Lat2, R, 1>(a, T_init, mode, s);
  return up == 0 ? launch_up<Lat2T9, R, 0>(a, T_init, mode, s) : launch_up<Lat2T9, R, 1>(a, T_init, mode, s);
}

template <class R>
hipError_t launch_step3d(const StepArgs<R>& a, int up, int tk, const double* T_init, int mode, hipStream_t s) {
  if (tk == 0) {
    switch (up) {
      case 0: return launch_up<Lat3, R, 0>(a, T_init, mode, s);
      case 1: return launch_up<Lat3, R, 1>(a, T_init, mode, s);
      default: return launch_up<Lat3, R, 2>(a, T_init, mode, s);
    }
  }
  switch (up) {
    case 0: return launch_up<Lat3T15, R, 0>(a, T_init, mode, s);
    case 1: return launch_up<Lat3T15, R, 1>(a, T_init, mode, s);
    default: return launch_up<Lat3T15, R, 2>(a, T_init, mode, s);
  }
}

// 2D in either precision and 3D FP32 (the 3D FP64 step would hold more than
// 256 registers per lane inside the step loop; it keeps per-step launches).
template <class R>
hipError_t launch_step_multi(const StepArgs<R>& a, int dim, int up, int tk, const MultiCtl& c, hipStream_t s) {
  if (dim == 2) {
    if (tk == 1) return up == 0 ? launch_multi_up<Lat2T9, R, 0>(a, c, s) : launch_multi_up<Lat2T9, R, 1>(a, c, s);
    return up == 0 ? launch_multi_up<Lat2, R, 0>(a, c, s) : launch_multi_up<Lat2, R, 1>(a, c, s);
  }
  if constexpr (sizeof(R) == 8) {
    return hipErrorNotSupported;
  } else {
    if (tk == 1) {
      switch (up) {
        case 0: return launch_multi_up<Lat3T15, R, 0>(a, c, s);
        case 1: return launch_multi_up<Lat3T15, R, 1>(a, c, s);
        default: return launch_multi_up<Lat3T15, R, 2>(a, c, s);
      }
    }
    switch (up) {
      case 0: return launch_multi_up<Lat3, R, 0>(a, c, s);
      case 1: return launch_multi_up<Lat3, R, 1>(a, c, s);
      default: return launch_multi_up<Lat3, R, 2>(a, c, s);
    }
  }
}

template hipError_t launch_step2d<double>(const StepArgs<double>&, int, int, const double*, int, hipStream_t);
template hipError_t launch_step2d<float>(const StepArgs<float>&, int, int, const double*, int, hipStream_t);
template hipError_t launch_step3d<double>(const StepArgs<double>&, int, int, const double*, int, hipStream_t);
template hipError_t launch_step3d<float>(const StepArgs<float>&, int, int, const double*, int, hipStream_t);

template hipError_t launch_step_multi<double>(const StepArgs<double>&, int, int, int, const MultiCtl&, hipStream_t);
template hipError_t launch_step_multi<float>(const StepArgs<float>&, int, int, int, const MultiCtl&, hipStream_t);

}  // namespace fpc
