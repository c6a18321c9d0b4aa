// C ABI of the batched PSR solver: mechanism packing, kernels, schedulers.
//
// Kernels (one workgroup of kBS threads per reactor):
//   k_residual     psr_residual: F(x) and the scaled residual (Eqs. 2-9)
//   k_jacobian     psr_jacobian: analytic dF/dx
//   k_lu_factor    psr_lu_factor_batch (FP64, or float factors)
//   k_lu_solve     psr_lu_solve_batch
//   k_round        plain scheduler: one controller round per launch, the
//                  reactor's vectors and matrices kept in HBM between rounds
//   k_persistent   persistent scheduler: workgroups pull reactors from a
//                  device work queue and run each to completion in LDS
#include <hip/hip_runtime.h>

#include <math.h>

#include <cmath>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/psr.h"
#include "psr_lu_wave.hpp"
#include "psr_solver.hpp"
#include "psr_wave_solver.hpp"

using namespace psr;

namespace {

constexpr int kBS = 256;
thread_local std::string g_err;

psr_status fail(psr_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(PSR_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
  } while (0)

int lds_limit_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v;
}

}  // namespace

struct psr_mech {
  int E, N, I, nnz;
  double soot_vol = 0.0;  // cm^3 of soot per carbon atom (m_C / rho_s); 0: no soot
  MechDev dev;
  void *blob;  // one device allocation holding every table
};

// ------------------------------------------------------------------ kernels

// Reactor of a one-workgroup-per-reactor launch.  Workgroups are dealt to
// the 8 XCDs round-robin (workgroup i to XCD i mod 8); numbering the reactors
// so that the workgroups of one XCD take consecutive reactors keeps the
// [var][reactor] lines that neighbouring reactors share in one XCD's L2.
// A bijection of [0, G).
__device__ inline int64_t xcd_reactor(int64_t blk, int64_t G) {
  constexpr int64_t kX = 8;
  const int64_t x = blk % kX, j = blk / kX, q = G / kX, r = G % kX;
  return x * q + (x < r ? x : r) + j;
}

__device__ inline Ctx make_ctx(const MechDev &m, const Layout &L, int energy, double P, double tau,
                               double Tin, double *base) {
  Ctx c;
  c.m = m;
  c.N = m.N;
  c.n = n_unknowns(m, energy);
  c.energy = energy;
  c.P = P;
  c.tau = tau;
  c.Tin = Tin;
  c.base = base;
  c.mat = nullptr;
  c.L = L;
  return c;
}

__global__ void __launch_bounds__(kBS) k_residual(MechDev m, int energy, int64_t B, const double *P,
                                                  const double *tau, const double *Tin,
                                                  const double *Yin, const double *x, double *F,
                                                  double *scaled) {
  extern __shared__ double lds[];
  const int64_t b = xcd_reactor(blockIdx.x, gridDim.x);
  Layout L;
  L.make(m.N, m.I, n_unknowns(m, energy), false, kBS, true, true);  // a residual alone
  Ctx c = make_ctx(m, L, energy, P[b], tau[b], Tin[b], lds);
  load_inlet<kBS>(c, Yin, B, b);
  double *xl = c.p(L.x), *G = c.p(L.G);
  for (int i = threadIdx.x; i < c.n; i += kBS) xl[i] = x[(int64_t)i * B + b];
  __syncthreads();
  const double sr = residual<kBS>(c, xl, G, scaled != nullptr);
  for (int i = threadIdx.x; i < c.n; i += kBS) F[(int64_t)i * B + b] = G[i];
  if (scaled && threadIdx.x == 0) scaled[b] = sr;
}

__global__ void __launch_bounds__(kBS) k_jacobian(MechDev m, int energy, int64_t B, const double *P,
                                                  const double *tau, const double *Tin,
                                                  const double *Yin, const double *x, double *J) {
  extern __shared__ double lds[];
  const int64_t b = xcd_reactor(blockIdx.x, gridDim.x);
  Layout L;
  L.make(m.N, m.I, n_unknowns(m, energy), false, kBS, true);  // the matrix is the output
  Ctx c = make_ctx(m, L, energy, P[b], tau[b], Tin[b], lds);
  load_inlet<kBS>(c, Yin, B, b);
  double *xl = c.p(L.x), *G = c.p(L.G);
  const int n = c.n;
  for (int i = threadIdx.x; i < n; i += kBS) xl[i] = x[(int64_t)i * B + b];
  __syncthreads();
  residual<kBS>(c, xl, G, false);
  jacobian<kBS>(c, xl, J + (int64_t)b * n * n, n);
}

template <typename T>
__global__ void __launch_bounds__(kBS) k_lu_factor(int n, double *A, int *piv, int *info) {
  extern __shared__ double lds[];
  const int64_t b = blockIdx.x;
  const int lda = (n % 2 == 0) ? n + 1 : n;
  T *M = reinterpret_cast<T *>(lds);
  double *red = lds + (n * lda * sizeof(T) + 7) / 8;
  int *pv = reinterpret_cast<int *>(red + kBS + 8);
  double *g = A + b * (int64_t)n * n;
  for (int e = threadIdx.x; e < n * n; e += kBS) M[(e / n) * lda + e % n] = (T)g[e];
  __syncthreads();
  const int r = lu_factor<kBS, T>(M, n, lda, pv, red);
  for (int e = threadIdx.x; e < n * n; e += kBS) g[e] = (double)M[(e / n) * lda + e % n];
  for (int k = threadIdx.x; k < n; k += kBS) piv[b * n + k] = (r == 0 || k < r) ? pv[k] : k;
  if (threadIdx.x == 0) info[b] = r;
}

// Factors of large matrices (float 64 < n <= 256, FP64 64 < n <= 128), one
// wavefront per matrix: four independent wavefronts per workgroup, each with
// its own LDS panel area and its own padded working area in HBM.
template <typename T>
__global__ void __launch_bounds__(256) k_lu_factor_wave(int n, int ld, int64_t batch, double *A, int *piv,
                                                        int *info, T *scratch) {
  extern __shared__ double lds[];
  psr::luw::WaveLds<T> *sh = reinterpret_cast<psr::luw::WaveLds<T> *>(lds);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t worker = (int64_t)blockIdx.x * psr::luw::kW + wv;
  const int64_t nworkers = (int64_t)gridDim.x * psr::luw::kW;
  T *M = scratch + worker * (int64_t)psr::luw::pad_rows(n) * ld;
  for (int64_t b = worker; b < batch; b += nworkers) {
    const int r = psr::luw::factor<T>(n, ld, A + b * (int64_t)n * n, M, piv + b * n, sh[wv], lane);
    if (lane == 0) info[b] = r;
  }
}

// Triangular solves with the factors of n <= 256 matrices, one wavefront per
// matrix: the right-hand side in registers (element i in lane i mod 64, slot
// i / 64), the interchanges applied in order, then row-oriented forward and
// back substitution -- each row of L and U read once, coalesced, the next
// row's loads issued before the current row's wavefront sum.
__global__ void __launch_bounds__(256) k_lu_solve_wave(int n, int64_t batch, const double *LU, const int *piv,
                                                       double *rhs) {
  constexpr int NS = 4;
  const int lane = threadIdx.x & 63;
  const int64_t worker = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nworkers = (int64_t)gridDim.x * 4;
  for (int64_t b = worker; b < batch; b += nworkers) {
    const double *A = LU + b * (int64_t)n * n;
    const int *pv = piv + b * n;
    double *r = rhs + b * n;
    double z[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
      const int i = lane + 64 * s;
      z[s] = i < n ? r[i] : 0.0;
    }
    for (int k = 0; k < n; k++) {
      const int p = pv[k];
      if (p == k) continue;
      double zk = 0.0, zp = 0.0;
#pragma unroll
      for (int s = 0; s < NS; s++) {
        if (s == (k >> 6)) zk = lane_read(z[s], k & 63);
        if (s == (p >> 6)) zp = lane_read(z[s], p & 63);
      }
#pragma unroll
      for (int s = 0; s < NS; s++) {
        const int i = lane + 64 * s;
        z[s] = i == k ? zp : (i == p ? zk : z[s]);
      }
    }
    // forward: z_i -= sum_{k < i} L_ik z_k (unit diagonal)
    double cur[NS], nxt[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
      const int c = lane + 64 * s;
      cur[s] = (n > 1 && c < n) ? A[(int64_t)1 * n + c] : 0.0;
    }
    for (int i = 1; i < n; i++) {
      if (i + 1 < n) {
#pragma unroll
        for (int s = 0; s < NS; s++) {
          const int c = lane + 64 * s;
          nxt[s] = c < n ? A[(int64_t)(i + 1) * n + c] : 0.0;
        }
      }
      double d = 0.0;
#pragma unroll
      for (int s = 0; s < NS; s++) {
        const int c = lane + 64 * s;
        d = c < i ? fma(cur[s], z[s], d) : d;
      }
      d = wave_sum(d);
#pragma unroll
      for (int s = 0; s < NS; s++) z[s] = (lane + 64 * s) == i ? z[s] - d : z[s];
#pragma unroll
      for (int s = 0; s < NS; s++) cur[s] = nxt[s];
    }
    // back: z_i = (z_i - sum_{k > i} U_ik z_k) / U_ii
#pragma unroll
    for (int s = 0; s < NS; s++) {
      const int c = lane + 64 * s;
      cur[s] = c < n ? A[(int64_t)(n - 1) * n + c] : 0.0;
    }
    for (int i = n - 1; i >= 0; i--) {
      if (i > 0) {
#pragma unroll
        for (int s = 0; s < NS; s++) {
          const int c = lane + 64 * s;
          nxt[s] = c < n ? A[(int64_t)(i - 1) * n + c] : 0.0;
        }
      }
      double d = 0.0, uii = 0.0;
#pragma unroll
      for (int s = 0; s < NS; s++) {
        const int c = lane + 64 * s;
        d = (c > i && c < n) ? fma(cur[s], z[s], d) : d;
        if (s == (i >> 6)) uii = lane_read(cur[s], i & 63);
      }
      d = wave_sum(d);
#pragma unroll
      for (int s = 0; s < NS; s++) z[s] = (lane + 64 * s) == i ? (z[s] - d) / uii : z[s];
#pragma unroll
      for (int s = 0; s < NS; s++) cur[s] = nxt[s];
    }
#pragma unroll
    for (int s = 0; s < NS; s++) {
      const int i = lane + 64 * s;
      if (i < n) r[i] = z[s];
    }
  }
}

__global__ void __launch_bounds__(kBS) k_lu_solve(int n, const double *A, const int *piv, double *rhs) {
  extern __shared__ double lds[];
  const int64_t b = blockIdx.x;
  const int lda = (n % 2 == 0) ? n + 1 : n;
  double *M = lds, *z = lds + n * lda;
  int *pv = reinterpret_cast<int *>(z + n);
  const double *g = A + b * (int64_t)n * n;
  for (int e = threadIdx.x; e < n * n; e += kBS) M[(e / n) * lda + e % n] = g[e];
  for (int k = threadIdx.x; k < n; k += kBS) {
    pv[k] = piv[b * n + k];
    z[k] = rhs[b * n + k];
  }
  __syncthreads();
  lu_solve<kBS, double>(M, n, lda, pv, z);
  for (int k = threadIdx.x; k < n; k += kBS) rhs[b * n + k] = z[k];
}

// Inputs of one group as the kernels see them.
struct GroupDev {
  MechDev m;
  int energy;
  int64_t B;
  const double *P, *tau, *Tin, *Yin;
  double *x;       // [n][B]
  int *status;     // [B]
  int *nlin;       // [B] or null
  const int *order;  // persistent queue position -> reactor index, or null (batch order)
};

__device__ inline void write_result(const GroupDev &g, const Ctx &c, const RState &s, int64_t b) {
  const double *xl = c.p(c.L.x);
  for (int i = threadIdx.x; i < c.n; i += kBS) g.x[(int64_t)i * g.B + b] = xl[i];
  if (threadIdx.x == 0) {
    g.status[b] = s.status;
    if (g.nlin) g.nlin[b] = s.n_lin;
  }
}

// Plain scheduler: one round per launch.  The persistent part of each
// reactor's area lives in HBM (`area`, [B][persist]) between launches.
template <bool MIXED, bool FIRST, bool BIG>
__global__ void __launch_bounds__(kBS) k_round(GroupDev g, Opts o, RState *states, double *area,
                                               int split, int *active) {
  extern __shared__ double lds[];
  const int64_t b = blockIdx.x;
  RState s = states[b];
  if (!FIRST && s.phase == PH_DONE) return;
  Layout L;
  L.make(g.m.N, g.m.I, n_unknowns(g.m, g.energy), MIXED, kBS, split != 0);
  Ctx c = make_ctx(g.m, L, g.energy, g.P[b], g.tau[b], g.Tin[b], lds);
  const int persist = L.persist;
  double *mine = area + b * (int64_t)(L.persist + L.mat_total);
  if (split) c.mat = mine + L.persist;  // the matrices stay in HBM
  if (FIRST) {
    load_inlet<kBS>(c, g.Yin, g.B, b);
    double *xl = c.p(L.x);
    for (int i = threadIdx.x; i < c.n; i += kBS) xl[i] = g.x[(int64_t)i * g.B + b];
    __syncthreads();
    init_state<kBS>(c, o, s);
  } else {
    for (int e = threadIdx.x; e < persist; e += kBS) lds[e] = mine[e];
    __syncthreads();
    round_step<kBS, MIXED, BIG>(c, o, s);
  }
  if (s.phase == PH_DONE) {
    write_result(g, c, s, b);
  } else {
    for (int e = threadIdx.x; e < persist; e += kBS) mine[e] = lds[e];
    if (threadIdx.x == 0) atomicAdd(active, 1);
  }
  if (threadIdx.x == 0) states[b] = s;
}

// Persistent scheduler: grid sized to the resident capacity; each
// workgroup takes the next reactor index from `queue` until none is left,
// and runs it to completion with every array in LDS.
template <bool MIXED, bool BIG>
__global__ void __launch_bounds__(kBS) k_persistent(GroupDev g, Opts o, RState *states, int *queue,
                                                    double *matws) {
  extern __shared__ double lds[];
  Layout L;
  L.make(g.m.N, g.m.I, n_unknowns(g.m, g.energy), MIXED, kBS, matws != nullptr);
  int *next = reinterpret_cast<int *>(lds + L.red + kBS + 4);
  for (;;) {
    if (threadIdx.x == 0) *next = atomicAdd(queue, 1);
    __syncthreads();
    const int64_t pos = *next;
    __syncthreads();
    if (pos >= g.B) break;
    const int64_t b = g.order ? g.order[pos] : pos;
    Ctx c = make_ctx(g.m, L, g.energy, g.P[b], g.tau[b], g.Tin[b], lds);
    if (matws) c.mat = matws + (int64_t)blockIdx.x * L.mat_total;  // this workgroup's HBM matrices
    load_inlet<kBS>(c, g.Yin, g.B, b);
    double *xl = c.p(L.x);
    for (int i = threadIdx.x; i < c.n; i += kBS) xl[i] = g.x[(int64_t)i * g.B + b];
    __syncthreads();
    RState s;
    init_state<kBS>(c, o, s);
    while (s.phase != PH_DONE) round_step<kBS, MIXED, BIG>(c, o, s);
    write_result(g, c, s, b);
    if (threadIdx.x == 0) states[b] = s;
    __syncthreads();
  }
}

// Soot outputs from the moments, one reactor per thread (coalesced over b):
// f_v = M_1 v_C, N = M_0, d = (6 f_v / (pi N))^(1/3); v_C = m_C / rho_s.
__global__ void __launch_bounds__(256) k_soot_outputs(int64_t B, int N, const double *__restrict__ x,
                                                      double *__restrict__ out, double vC) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B; b += (int64_t)gridDim.x * blockDim.x) {
    const double N0 = exp(x[(int64_t)(N + 1) * B + b]);
    const double fv = exp(x[(int64_t)(N + 2) * B + b]) * vC;
    out[b] = fv;
    out[B + b] = N0;
    out[2 * B + b] = cbrt(6.0 * fv / (3.14159265358979323846 * N0));
  }
}

__global__ void k_zero_int(int *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}


// ------------------------------------------------- wavefront-per-reactor engine

namespace wk {
using namespace psr::wave;

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) / 16 * 16; }

// Doubles of one reactor's HBM area for the plain scheduler (lane-interleaved).
template <int NP, bool MIXED>
__host__ __device__ inline int plain_stride(int n) {
  return 10 * WS + NP * WS + (MIXED ? n * WArea<NP>::ldj_of(n) : 0);
}

// LDS of a wave-engine workgroup: mechanism tables, a copy of the solver
// options (read from LDS where used, so they do not occupy scalar registers
// for the whole kernel), then the per-wavefront reactor areas.
__host__ __device__ inline size_t wave_opts_off(int N, int I, int nnz) { return align16(tables_bytes(N, I, nnz)); }
__host__ __device__ inline size_t wave_area_off(int N, int I, int nnz) {
  return wave_opts_off(N, I, nnz) + align16(sizeof(Opts));
}

template <int NP, bool MIXED>
__device__ inline void make_wctx(WCtx &c, const Tables &t, const GroupDev &g, int64_t b) {
  const int lane = lane_id();
  c.t = t;
  c.N = g.m.N;
  c.n = n_unknowns(g.m, g.energy);
  c.energy = g.energy;
  c.P = g.P[b];
  c.tau = g.tau[b];
  c.Tin = g.Tin[b];
  c.Yin = lane < c.N ? g.Yin[(int64_t)lane * g.B + b] : 0.0;
  c.Hin = lane < c.N ? inlet_enthalpy(t, lane, c.Tin) : 0.0;
}

template <int NP, bool MIXED>
__device__ inline void write_result_w(const GroupDev &g, const WCtx &c, const WState<NP, MIXED> &r,
                                      RState *states, int64_t b) {
  const int lane = lane_id();
  if (lane < c.n) g.x[(int64_t)lane * g.B + b] = r.x;
  if (lane == 0) {
    g.status[b] = r.s.status;
    if (g.nlin) g.nlin[b] = r.s.n_lin;
    states[b] = r.s;
  }
}

// Persistent scheduler: each wavefront pulls reactor indices from the device
// queue and solves each reactor to completion; the workgroup's wavefronts
// share the LDS copy of the mechanism tables.
template <int NP, bool MIXED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) k_wpersist(GroupDev g, Opts og, RState *states, int *queue) {
  extern __shared__ double lds[];
  char *base = reinterpret_cast<char *>(lds);
  const Tables t = stage_tables(g.m, base, g.m.packed);
  Opts *ol = reinterpret_cast<Opts *>(base + wave_opts_off(g.m.N, g.m.I, g.m.nnz));
  if (threadIdx.x == 0) *ol = og;
  __syncthreads();
  const Opts &o = *ol;
  const int n = n_unknowns(g.m, g.energy);
  const size_t toff = wave_area_off(g.m.N, g.m.I, g.m.nnz);
  WArea<NP> A;
  A.at(reinterpret_cast<double *>(base + toff) + (size_t)wave_id() * WArea<NP>::doubles(n), n);
  const int lane = lane_id();
  for (;;) {
    int b = 0;
    if (lane == 0) b = atomicAdd(queue, 1);
    b = bcast(b, 0);
    if (b >= g.B) break;
    if (g.order) b = g.order[b];
    WCtx c;
    make_wctx<NP, MIXED>(c, t, g, b);
    WState<NP, MIXED> r;
    init_w<NP, MIXED>(c, o, r, lane < n ? g.x[(int64_t)lane * g.B + b] : 0.0);
    while (r.s.phase != PH_DONE) w_round<NP, MIXED>(c, A, o, r);
    write_result_w<NP, MIXED>(g, c, r, states, b);
  }
}

// ------------------------------------------------ fused persistent launch

// Several groups (mechanisms) of one persistent solve in one launch over one
// device queue.  Queue positions [start_g, start_g + B_g) belong to group g;
// the workgroup-engine groups come first (largest n first), at most one
// wavefront-engine group last.  A workgroup takes positions one at a time and
// solves the reactor with all its threads; once it draws a position of the
// wavefront-engine group it stages that group's tables in its LDS and from
// then on each of its four wavefronts takes positions on its own.
constexpr int kMaxFused = 4;

struct FusedGroup {
  GroupDev g;
  RState *states;
  int64_t start;  // first queue position of the group
  int wave;       // 1: wavefront engine
  int split;      // workgroup engine: matrices in HBM
};

struct FusedDev {
  FusedGroup grp[kMaxFused];
  int ng;
  int64_t total;       // positions in the queue (reactors of every group)
  double *matws;       // HBM matrices of the workgroup engine, mat_stride doubles per workgroup
  int64_t mat_stride;
  int next_off;        // LDS byte offset of the position broadcast slot
};

template <int NP, bool MIXED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_fused(FusedDev fd, Opts og, int *queue) {
  extern __shared__ double lds[];
  char *base = reinterpret_cast<char *>(lds);
  int *next = reinterpret_cast<int *>(base + fd.next_off);
  int p = 0;
  int gi = 0;
  for (;;) {
    if (threadIdx.x == 0) *next = atomicAdd(queue, 1);
    __syncthreads();
    p = *next;
    __syncthreads();
    if (p >= fd.total) return;
    gi = 0;
    while (gi + 1 < fd.ng && p >= fd.grp[gi + 1].start) gi++;
    if (fd.grp[gi].wave) break;  // the same for every thread: p is shared
    const GroupDev &g = fd.grp[gi].g;
    Layout L;
    L.make(g.m.N, g.m.I, n_unknowns(g.m, g.energy), MIXED, kBS, fd.grp[gi].split != 0);
    const int64_t pos = p - fd.grp[gi].start;
    const int64_t b = g.order ? g.order[pos] : pos;
    Ctx c = make_ctx(g.m, L, g.energy, g.P[b], g.tau[b], g.Tin[b], lds);
    if (fd.grp[gi].split) c.mat = fd.matws + (int64_t)blockIdx.x * fd.mat_stride;
    load_inlet<kBS>(c, g.Yin, g.B, b);
    double *xl = c.p(L.x);
    for (int i = threadIdx.x; i < c.n; i += kBS) xl[i] = g.x[(int64_t)i * g.B + b];
    __syncthreads();
    RState s;
    init_state<kBS>(c, og, s);
    while (s.phase != PH_DONE) round_step<kBS, MIXED, true>(c, og, s);
    write_result(g, c, s, b);
    if (threadIdx.x == 0) fd.grp[gi].states[b] = s;
    __syncthreads();
  }
  if constexpr (NP > 0) {
    const GroupDev &g = fd.grp[gi].g;
    RState *states = fd.grp[gi].states;
    const int64_t start = fd.grp[gi].start;
    const Tables t = stage_tables(g.m, base, g.m.packed);
    Opts *ol = reinterpret_cast<Opts *>(base + wave_opts_off(g.m.N, g.m.I, g.m.nnz));
    if (threadIdx.x == 0) *ol = og;
    __syncthreads();
    const Opts &o = *ol;
    const int n = n_unknowns(g.m, g.energy);
    WArea<NP> A;
    A.at(reinterpret_cast<double *>(base + wave_area_off(g.m.N, g.m.I, g.m.nnz)) +
             (size_t)wave_id() * WArea<NP>::doubles(n), n);
    const int lane = lane_id();
    int q = p;  // wavefront 0 keeps the position its workgroup drew
    if (wave_id() != 0) {
      int v = 0;
      if (lane == 0) v = atomicAdd(queue, 1);
      q = bcast(v, 0);
    }
    while (q < fd.total) {
      const int64_t pos = q - start;
      const int64_t b = g.order ? g.order[pos] : pos;
      WCtx c;
      make_wctx<NP, MIXED>(c, t, g, b);
      WState<NP, MIXED> r;
      init_w<NP, MIXED>(c, o, r, lane < n ? g.x[(int64_t)lane * g.B + b] : 0.0);
      while (r.s.phase != PH_DONE) w_round<NP, MIXED>(c, A, o, r);
      write_result_w<NP, MIXED>(g, c, r, states, b);
      int v = 0;
      if (lane == 0) v = atomicAdd(queue, 1);
      q = bcast(v, 0);
    }
  }
}

template <int NP, bool MIXED>
__device__ inline void save_w(const WCtx &c, const WArea<NP> &A, const WState<NP, MIXED> &r, double *ar) {
  const int lane = lane_id(), n = c.n;
  const double v[9] = {r.x, r.xnw, r.xev, r.d, r.t, r.M, r.rs, r.cs, r.piv};
#pragma unroll
  for (int q = 0; q < 9; q++) ar[q * WS + lane] = v[q];
  int *ints = reinterpret_cast<int *>(ar + 9 * WS);
  ints[lane] = r.perm;
  double *fac = ar + 10 * WS;
  if (r.s.phase == PH_NW_TRIAL || r.s.phase == PH_TS2) {  // factors still in use
#pragma unroll
    for (int j = 0; j < NP; j++)
      if (j < n) fac[j * WS + lane] = r.a[j];
    if (MIXED && !r.s.fb64) {  // refinement needs the FP64 matrix
      double *Jc = fac + NP * WS;
      for (int e = lane; e < n * A.ldj; e += WS) Jc[e] = A.J[e];
    }
  }
}

template <int NP, bool MIXED>
__device__ inline void load_w(const WCtx &c, const WArea<NP> &A, WState<NP, MIXED> &r, const double *ar) {
  const int lane = lane_id(), n = c.n;
  r.x = ar[lane]; r.xnw = ar[WS + lane]; r.xev = ar[2 * WS + lane]; r.d = ar[3 * WS + lane];
  r.t = ar[4 * WS + lane]; r.M = ar[5 * WS + lane]; r.rs = ar[6 * WS + lane]; r.cs = ar[7 * WS + lane];
  r.piv = ar[8 * WS + lane];
  const int *ints = reinterpret_cast<const int *>(ar + 9 * WS);
  r.perm = ints[lane];
  const double *fac = ar + 10 * WS;
#pragma unroll
  for (int j = 0; j < NP; j++) r.a[j] = 0.0;
  if (r.s.phase == PH_NW_TRIAL || r.s.phase == PH_TS2) {
#pragma unroll
    for (int j = 0; j < NP; j++)
      if (j < n) r.a[j] = fac[j * WS + lane];
    if (MIXED && !r.s.fb64) {
      const double *Jc = fac + NP * WS;
      for (int e = lane; e < n * A.ldj; e += WS) A.J[e] = Jc[e];
    }
  }
  wsync();
}

// Plain scheduler on the wavefront engine: one controller round per launch,
// each reactor's vectors (and, while a linearisation is in use, its factors)
// kept in HBM between launches.
template <int NP, bool MIXED, bool FIRST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) k_wround(GroupDev g, Opts og, RState *states, double *area,
                                                int stride, int rpw, int *active) {
  extern __shared__ double lds[];
  char *base = reinterpret_cast<char *>(lds);
  const Tables t = stage_tables(g.m, base, g.m.packed);
  Opts *ol = reinterpret_cast<Opts *>(base + wave_opts_off(g.m.N, g.m.I, g.m.nnz));
  if (threadIdx.x == 0) *ol = og;
  __syncthreads();
  const Opts &o = *ol;
  const int n = n_unknowns(g.m, g.energy);
  const int64_t b = (int64_t)blockIdx.x * rpw + wave_id();
  if (b >= g.B) return;
  RState s0 = states[b];
  if (!FIRST && s0.phase == PH_DONE) return;
  const size_t toff = wave_area_off(g.m.N, g.m.I, g.m.nnz);
  WArea<NP> A;
  A.at(reinterpret_cast<double *>(base + toff) + (size_t)wave_id() * WArea<NP>::doubles(n), n);
  const int lane = lane_id();
  WCtx c;
  make_wctx<NP, MIXED>(c, t, g, b);
  WState<NP, MIXED> r;
  double *ar = area + b * (int64_t)stride;
  if (FIRST) {
    init_w<NP, MIXED>(c, o, r, lane < n ? g.x[(int64_t)lane * g.B + b] : 0.0);
  } else {
    r.s = s0;
    load_w<NP, MIXED>(c, A, r, ar);
    w_round<NP, MIXED>(c, A, o, r);
  }
  if (r.s.phase == PH_DONE) {
    write_result_w<NP, MIXED>(g, c, r, states, b);
  } else {
    save_w<NP, MIXED>(c, A, r, ar);
    if (lane == 0) {
      states[b] = r.s;
      atomicAdd(active, 1);
    }
  }
}

// Residual of a batch (Eqs. 2-3): one wavefront per reactor, kWR
// wavefronts per workgroup sharing the LDS tables, grid-stride over reactors
// so the tables are staged once per workgroup.
constexpr int kWR = 8;

__global__ void __launch_bounds__(kWR * 64) __attribute__((amdgpu_waves_per_eu(6)))
k_wresidual(GroupDev g, double *F, double *scaled) {
  extern __shared__ double lds[];
  char *base = reinterpret_cast<char *>(lds);
  const Tables t = stage_tables(g.m, base, g.m.packed);
  __syncthreads();
  const int n = n_unknowns(g.m, g.energy);
  const size_t toff = align16(tables_bytes(g.m.N, g.m.I, g.m.nnz));
  WArea<64> A;
  A.at_species(reinterpret_cast<double *>(base + toff) + (size_t)wave_id() * WArea<64>::species_doubles());
  const int lane = lane_id();
  // each workgroup walks one contiguous range of reactors, kWR at a time:
  // the [var][reactor] lines its wavefronts read (and write) are shared by
  // neighbouring reactors, which then stay on one CU and one XCD's L2
  const int64_t per = ((g.B + gridDim.x - 1) / gridDim.x + kWR - 1) / kWR * kWR;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < g.B ? b0 + per : g.B;
  for (int64_t b = b0 + wave_id(); b < b1; b += kWR) {
    WCtx c;
    make_wctx<64, false>(c, t, g, b);
    const double x = lane < n ? g.x[(int64_t)lane * g.B + b] : 0.0;
    Eval ev;
    double Fl = 0.0;
    const double sres = w_residual<64>(c, A, x, Fl, ev, scaled != nullptr);
    if (lane < n) F[(int64_t)lane * g.B + b] = Fl;
    if (scaled && lane == 0) scaled[b] = sres;
  }
}

}  // namespace wk

// ------------------------------------------------------------ host: mechanism

extern "C" const char *psr_last_error(void) { return g_err.c_str(); }

extern "C" void psr_default_opts(psr_solve_opts *o) {
  memset(o, 0, sizeof(*o));
  o->precision = PSR_FP64;
  o->scheduler = PSR_PLAIN;
  o->rtol = 1e-10;
  o->atol_Y = 1e-20;
  o->atol_T = 1e-12;
  o->ftol = 1e-10;
  o->lambda_min = 0.0;
  o->T_min = 300.0;
  o->T_max = 4000.0;
  o->ts_rtol = 0.1;
  o->ts_atol_Y = 1e-6;
  o->ts_atol_T = 1e-3;
  o->ts_neg_tol = 1e-8;
  o->h0 = 1e-6;
  o->h_max = 1e6;
  o->h_min = 1e-30;
  o->nw_h_ratio = 0.0;
  o->nw_max_it = 30;
  o->nw_every = 10;
  o->max_lin = 1500;
  o->max_refine = 6;
  o->engine = 0;
  o->use_graph = 1;
  o->refine_tol = 1e-6;
  o->atol_lnM = 1e-10;
  o->ts_atol_lnM = 1e-3;
  o->lnM_step = 2.0;
  o->ct_ratio = 10.0;
  o->ct_tau_min = 1e-6;
  o->ct_min_step = 0.05;
  o->order = 1;
  o->mixed_max_n = 64;
}

// Lagrange basis polynomial l over the nodes 0..m-1, at p.
static double lagrange(double p, int l, int m) {
  double v = 1.0;
  for (int k = 0; k < m; k++)
    if (k != l) v *= (p - k) / (double)(l - k);
  return v;
}

// Validate a soot description and build the closure table: for each
// fractional order p of the closure (index order of kSootOrders), the
// coefficients c_j of ln mu_p = sum_j c_j ln M_j, from the Lagrange
// interpolation of ln mu_l = ln M_l - ln M_0 over l = 0..5 (p >= 0) or
// l = 0..2 (p < 0); then the four weights L_l(1/2), l = 0..3.
static psr_status soot_tables(const psr_mech_desc *d, std::vector<double> &frac) {
  const psr_soot_desc *sd = d->soot;
  const int E = d->n_elements, N = d->n_species;
  if (sd->carbon < 0 || sd->carbon >= E) return fail(PSR_EINVAL, "soot: carbon element out of range");
  for (int sp : {sd->precursor, sd->growth}) {
    if (sp < 0 || sp >= N) return fail(PSR_EINVAL, "soot: species index out of range");
    for (int e = 0; e < E; e++)
      if ((e == sd->carbon) != (d->species_elems[sp * E + e] > 0))
        return fail(PSR_EINVAL, "soot: precursor and growth species must be pure carbon");
  }
  if (sd->precursor == sd->growth) return fail(PSR_EINVAL, "soot: precursor and growth species coincide");
  const double v[] = {sd->A_nuc, sd->beta_nuc, sd->E_nuc, sd->A_grow, sd->beta_grow, sd->E_grow,
                      sd->site_density, sd->soot_density, sd->coag_scale};
  for (double a : v)
    if (!std::isfinite(a)) return fail(PSR_EINVAL, "soot: non-finite constant");
  if (sd->A_nuc < 0 || sd->A_grow < 0 || sd->site_density < 0 || !(sd->soot_density > 0) ||
      sd->coag_scale < 0)
    return fail(PSR_EINVAL, "soot: negative rate constant or non-positive density");
  frac.assign(6 * kSootOrders + 4, 0.0);
  for (int q = 0; q < kSootOrders; q++) {
    double p;
    if (q < 24) p = (q / 3) + (q % 3 == 0 ? 1.0 / 6.0 : (q % 3 == 1 ? -1.0 / 6.0 : -0.5));
    else p = (q - 24) + 2.0 / 3.0;
    const int nodes = p >= 0.0 ? 6 : 3;
    double *c = frac.data() + 6 * q;
    for (int l = 1; l < nodes; l++) {
      const double L = lagrange(p, l, nodes);
      c[l] += L;
      c[0] -= L;
    }
  }
  for (int l = 0; l < 4; l++) frac[6 * kSootOrders + l] = lagrange(0.5, l, 4);
  return PSR_OK;
}

extern "C" psr_status psr_create_mechanism(const psr_mech_desc *d, psr_mech_t *out) {
  if (!d || !out) return fail(PSR_EINVAL, "null argument");
  *out = nullptr;
  const int E = d->n_elements, N = d->n_species, I = d->n_reactions;
  if (E <= 0 || N <= 0 || I <= 0) return fail(PSR_EINVAL, "counts must be positive");
  if (!d->elem_weight || !d->species_elems || !d->nasa7 || !d->reac_idx || !d->reac_nu ||
      !d->prod_idx || !d->prod_nu || !d->A || !d->beta || !d->Ea)
    return fail(PSR_EINVAL, "null table pointer");
  if (!(d->t_low < d->t_high)) return fail(PSR_EINVAL, "t_low must be < t_high");
  std::vector<double> W(N, 0.0);
  for (int i = 0; i < N; i++) {
    for (int e = 0; e < E; e++) {
      if (d->species_elems[i * E + e] < 0)
        return fail(PSR_EINVAL, "negative atom count, species " + std::to_string(i));
      W[i] += d->species_elems[i * E + e] * d->elem_weight[e];
    }
    if (!(W[i] > 0.0)) return fail(PSR_EINVAL, "species " + std::to_string(i) + " has no weight");
  }
  std::vector<double> lnA(I), beta(I), EoR(I);
  std::vector<int> dnu(I), ridx(3 * I), rnu(3 * I), pidx(3 * I), pnu(3 * I);
  std::vector<std::vector<std::pair<int, int>>> bysp(N);
  for (int k = 0; k < I; k++) {
    if (!(d->A[k] > 0.0) || !std::isfinite(d->A[k]) || !std::isfinite(d->beta[k]) ||
        !std::isfinite(d->Ea[k]))
      return fail(PSR_EINVAL, "reaction " + std::to_string(k) + ": bad Arrhenius parameters");
    lnA[k] = log(d->A[k]);
    beta[k] = d->beta[k];
    EoR[k] = d->Ea[k] / kR;
    std::vector<long long> bal(E, 0);
    std::vector<int> net(N, 0);
    int nr = 0, np = 0, sum = 0;
    for (int s = 0; s < 3; s++) {
      const int ir = d->reac_idx[3 * k + s], ip = d->prod_idx[3 * k + s];
      ridx[3 * k + s] = ir;
      rnu[3 * k + s] = ir >= 0 ? d->reac_nu[3 * k + s] : 0;
      pidx[3 * k + s] = ip;
      pnu[3 * k + s] = ip >= 0 ? d->prod_nu[3 * k + s] : 0;
      for (int side = 0; side < 2; side++) {
        const int i = side ? ip : ir;
        const int nu = side ? d->prod_nu[3 * k + s] : d->reac_nu[3 * k + s];
        if (i < -1 || i >= N)
          return fail(PSR_EINVAL, "reaction " + std::to_string(k) + ": species index out of range");
        if (i < 0) continue;
        if (nu < 1 || nu > 8)
          return fail(PSR_EINVAL, "reaction " + std::to_string(k) + ": coefficient out of range");
        const int sg = side ? 1 : -1;
        if ((side && net[i] < 0) || (!side && net[i] > 0))
          return fail(PSR_EINVAL, "reaction " + std::to_string(k) + ": species on both sides");
        if (net[i] != 0)
          return fail(PSR_EINVAL, "reaction " + std::to_string(k) + ": repeated species slot");
        net[i] = sg * nu;
        sum += sg * nu;
        (side ? np : nr)++;
        for (int e = 0; e < E; e++) bal[e] += (long long)sg * nu * d->species_elems[i * E + e];
      }
    }
    if (nr == 0 || np == 0)
      return fail(PSR_EINVAL, "reaction " + std::to_string(k) + ": empty side");
    for (int e = 0; e < E; e++)
      if (bal[e] != 0)
        return fail(PSR_EINVAL, "reaction " + std::to_string(k) + ": not element balanced");
    dnu[k] = sum;
    for (int i = 0; i < N; i++)
      if (net[i] != 0) bysp[i].push_back({k, net[i]});
  }
  std::vector<int> ptr(N + 1, 0), rx, nu;
  for (int i = 0; i < N; i++) {
    ptr[i + 1] = ptr[i] + (int)bysp[i].size();
    for (auto &pr : bysp[i]) { rx.push_back(pr.first); nu.push_back(pr.second); }
  }
  const int nnz = ptr[N];
  // soot closure: d ln mu_p / d ln M_j of the fractional orders, then the
  // weights L_l(1/2) of the coagulation interpolation over l = 0..3
  const psr_soot_desc *sd = d->soot;
  std::vector<double> frac;
  if (sd) {
    psr_status sst = soot_tables(d, frac);
    if (sst != PSR_OK) return sst;
  }
  // one blob: doubles first, then ints
  const size_t nd = (size_t)N + 7 * N + 3 * I + frac.size();
  // packed slot words for the wavefront engine (needs N <= 254, nu <= 15)
  bool packable = N <= 254;
  std::vector<int> pk(3 * (size_t)I + nnz, 0);
  for (int k = 0; k < I && packable; k++) {
    int w0 = 0, w1 = 0, w2 = 0;
    for (int s = 0; s < 3; s++) {
      const int ir = ridx[3 * k + s], ip = pidx[3 * k + s];
      w0 |= (ir >= 0 ? ir : 0xff) << (8 * s);
      w1 |= (ip >= 0 ? ip : 0xff) << (8 * s);
      if (rnu[3 * k + s] > 15 || pnu[3 * k + s] > 15) packable = false;
      w2 |= (rnu[3 * k + s] & 0xf) << (4 * s);
      w2 |= (pnu[3 * k + s] & 0xf) << (12 + 4 * s);
    }
    if (dnu[k] < -16 || dnu[k] > 100) packable = false;
    w2 |= ((dnu[k] + 16) & 0xff) << 24;
    pk[k] = w0; pk[I + k] = w1; pk[2 * I + k] = w2;
  }
  for (int e = 0; e < nnz && packable; e++) {
    if (rx[e] >= (1 << 23) || nu[e] < -127 || nu[e] > 127) packable = false;
    pk[3 * (size_t)I + e] = (rx[e] << 8) | ((nu[e] + 128) & 0xff);
  }
  const size_t ni = (size_t)I + 12 * I + (N + 1) + 2 * std::max(nnz, 1) + pk.size();
  std::vector<char> host(nd * 8 + ni * 4);
  double *hd = reinterpret_cast<double *>(host.data());
  int *hi = reinterpret_cast<int *>(host.data() + nd * 8);
  size_t od = 0, oi = 0;
  auto putd = [&](const double *src, size_t cnt) { if (cnt) memcpy(hd + od, src, cnt * 8); od += cnt; return od - cnt; };
  auto puti = [&](const int *src, size_t cnt) { if (cnt) memcpy(hi + oi, src, cnt * 4); oi += cnt; return oi - cnt; };
  const size_t oW = putd(W.data(), N), oNasa = putd(d->nasa7, 7 * (size_t)N);
  const size_t olnA = putd(lnA.data(), I), obeta = putd(beta.data(), I), oEoR = putd(EoR.data(), I);
  const size_t ofrac = putd(frac.data(), frac.size());
  const size_t odnu = puti(dnu.data(), I), orI = puti(ridx.data(), 3 * I), orN = puti(rnu.data(), 3 * I);
  const size_t opI = puti(pidx.data(), 3 * I), opN = puti(pnu.data(), 3 * I);
  const size_t optr = puti(ptr.data(), N + 1), orx = puti(rx.data(), nnz), onu = puti(nu.data(), nnz);
  const size_t opk = puti(pk.data(), pk.size());
  for (int i = 0; i < N * 7; i++)
    if (!std::isfinite(d->nasa7[i])) return fail(PSR_EINVAL, "non-finite NASA-7 coefficient");
  void *blob = nullptr;
  HIP_OK(hipMalloc(&blob, host.size()));
  if (hipMemcpy(blob, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(blob);
    return fail(PSR_EDEVICE, "hipMemcpy of mechanism tables failed");
  }
  psr_mech *m = new psr_mech();
  m->E = E; m->N = N; m->I = I; m->nnz = nnz; m->blob = blob;
  const double *bd = reinterpret_cast<const double *>(blob);
  const int *bi = reinterpret_cast<const int *>(reinterpret_cast<const char *>(blob) + nd * 8);
  m->dev.N = N; m->dev.I = I; m->dev.nnz = nnz;
  m->dev.W = bd + oW; m->dev.nasa = bd + oNasa;
  m->dev.lnA = bd + olnA; m->dev.beta = bd + obeta; m->dev.EoR = bd + oEoR;
  m->dev.dnu = bi + odnu; m->dev.r_idx = bi + orI; m->dev.r_nu = bi + orN;
  m->dev.p_idx = bi + opI; m->dev.p_nu = bi + opN;
  m->dev.sp_ptr = bi + optr; m->dev.sp_rx = bi + orx; m->dev.sp_nu = bi + onu;
  m->dev.packed = packable ? bi + opk : nullptr;
  m->dev.soot = 0;
  if (sd) {  // the wavefront engine has no soot rows: soot mechanisms use the block engine
    const double kNA = 6.02214076e23, kB = 1.380649e-16, pi = 3.14159265358979323846;
    const double mC = d->elem_weight[sd->carbon] / kNA;  // g per carbon atom
    m->dev.packed = nullptr;
    m->dev.soot = 1;
    m->dev.sP = sd->precursor;
    m->dev.sG = sd->growth;
    m->dev.Cmin = 2.0 * d->species_elems[sd->precursor * E + sd->carbon];
    m->dev.D = d->species_elems[sd->growth * E + sd->carbon];
    m->dev.An = sd->A_nuc; m->dev.bn = sd->beta_nuc; m->dev.EnR = sd->E_nuc / kR;
    m->dev.As = sd->A_grow; m->dev.bs = sd->beta_grow; m->dev.EsR = sd->E_grow / kR;
    m->dev.KW = sd->site_density * pi * pow(6.0 * mC / (pi * sd->soot_density), 2.0 / 3.0);
    m->dev.KF0 = sd->coag_scale * 2.2 * pow(3.0 * mC / (4.0 * pi * sd->soot_density), 1.0 / 6.0) *
                 sqrt(6.0 * kB / sd->soot_density);
    m->dev.frac = bd + ofrac;
    m->soot_vol = mC / sd->soot_density;
  }
  *out = m;
  return PSR_OK;
}

extern "C" psr_status psr_destroy_mechanism(psr_mech_t m) {
  if (!m) return PSR_OK;
  hipError_t e = hipFree(m->blob);
  delete m;
  if (e != hipSuccess) return fail(PSR_EDEVICE, "hipFree failed");
  return PSR_OK;
}

extern "C" int32_t psr_num_unknowns(psr_mech_t m, int32_t energy) {
  return m ? n_unknowns(m->dev, energy) : -1;
}

// ------------------------------------------------------------ host: kernels

static psr_status check_cond(psr_mech_t m, const psr_conditions *c) {
  if (!m || !c) return fail(PSR_EINVAL, "null argument");
  if (c->n_reactors <= 0) return fail(PSR_EINVAL, "n_reactors must be positive");
  if (c->n_reactors > 0x7fffffffLL) return fail(PSR_EUNSUPPORTED, "n_reactors above 2^31-1");
  if (!c->P || !c->tau || !c->T_in || !c->Y_in) return fail(PSR_EINVAL, "null condition pointer");
  if (c->energy < 0 || c->energy > 2) return fail(PSR_EINVAL, "energy must be 0, 1 or 2");
  if (m->dev.soot && !c->energy) return fail(PSR_EINVAL, "a soot mechanism needs a temperature unknown (energy 1 or 2)");
  return PSR_OK;
}

static size_t layout_bytes(psr_mech_t m, int energy, bool mixed, bool split = false, bool lean = false) {
  Layout L;
  L.make(m->N, m->I, n_unknowns(m->dev, energy), mixed, kBS, split, lean);
  return (size_t)L.total * 8;
}

// Block-engine layout of a group: everything in LDS when it fits, else the
// matrices in HBM (split).  Returns false if even the split layout exceeds
// the LDS of one workgroup.
static bool block_layout(psr_mech_t m, int energy, bool mixed, Layout &L) {
  L.make(m->N, m->I, n_unknowns(m->dev, energy), mixed, kBS, false);
  if ((size_t)L.total * 8 <= (size_t)lds_limit_bytes()) return true;
  L.make(m->N, m->I, n_unknowns(m->dev, energy), mixed, kBS, true);
  return (size_t)L.total * 8 <= (size_t)lds_limit_bytes();
}

// Resident workgroups of the block engine's persistent kernel (at most
// per_cu_cap per compute unit when it is positive).
static int64_t block_grid(const Layout &L, bool mixed, int64_t B, int per_cu_cap) {
  const bool big = L.n > 64;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t lds = (size_t)L.total * 8;
  hipError_t e;
  if (mixed)
    e = big ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<true, true>, kBS, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<true, false>, kBS, lds);
  else
    e = big ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<false, true>, kBS, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<false, false>, kBS, lds);
  if (e != hipSuccess) return 0;
  if (per_cu_cap > 0) per_cu = std::min(per_cu, per_cu_cap);
  if (per_cu < 1) per_cu = 1;
  return std::min<int64_t>(B, (int64_t)ncu * per_cu);
}

extern "C" psr_status psr_residual(psr_mech_t m, const psr_conditions *c, const double *x, double *F,
                                   double *scaled, void *stream) {
  psr_status st = check_cond(m, c);
  if (st != PSR_OK) return st;
  if (!x || !F) return fail(PSR_EINVAL, "null x or F");
  const int n = n_unknowns(m->dev, c->energy);
  if (m->dev.packed && n <= 64 && c->energy != 2) {
    const size_t lds = wk::align16(psr::wave::tables_bytes(m->N, m->I, m->nnz)) +
                       (size_t)wk::kWR * psr::wave::WArea<64>::species_doubles() * 8;
    if (lds <= (size_t)lds_limit_bytes()) {
      GroupDev g{};
      g.m = m->dev;
      g.energy = c->energy;
      g.B = c->n_reactors;
      g.P = c->P; g.tau = c->tau; g.Tin = c->T_in; g.Yin = c->Y_in;
      g.x = const_cast<double *>(x);
      const int64_t blocks = (c->n_reactors + wk::kWR - 1) / wk::kWR;
      const unsigned grid = (unsigned)(blocks < 2048 ? blocks : 2048);
      hipLaunchKernelGGL(wk::k_wresidual, dim3(grid), dim3(wk::kWR * 64), lds, (hipStream_t)stream, g, F,
                         scaled);
      HIP_OK(hipGetLastError());
      return PSR_OK;
    }
  }
  const size_t lds = layout_bytes(m, c->energy, false, true, true);
  if (lds > (size_t)lds_limit_bytes()) return fail(PSR_EUNSUPPORTED, "mechanism too large for LDS");
  hipLaunchKernelGGL(k_residual, dim3((unsigned)c->n_reactors), dim3(kBS), lds, (hipStream_t)stream,
                     m->dev, c->energy, c->n_reactors, c->P, c->tau, c->T_in, c->Y_in, x, F,
                     scaled);
  HIP_OK(hipGetLastError());
  return PSR_OK;
}

extern "C" psr_status psr_soot_outputs(psr_mech_t m, int64_t B, const double *x, double *out, void *stream) {
  if (!m || !x || !out) return fail(PSR_EINVAL, "null argument");
  if (B < 1) return fail(PSR_EINVAL, "n_reactors must be positive");
  if (!m->dev.soot) return fail(PSR_EINVAL, "mechanism has no soot model");
  const int64_t blocks = (B + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
  hipLaunchKernelGGL(k_soot_outputs, dim3(grid), dim3(256), 0, (hipStream_t)stream, B, m->N, x, out, m->soot_vol);
  HIP_OK(hipGetLastError());
  return PSR_OK;
}

extern "C" psr_status psr_jacobian(psr_mech_t m, const psr_conditions *c, const double *x, double *J,
                                   void *stream) {
  psr_status st = check_cond(m, c);
  if (st != PSR_OK) return st;
  if (!x || !J) return fail(PSR_EINVAL, "null x or J");
  const size_t lds = layout_bytes(m, c->energy, false, true);
  if (lds > (size_t)lds_limit_bytes()) return fail(PSR_EUNSUPPORTED, "mechanism too large for LDS");
  hipLaunchKernelGGL(k_jacobian, dim3((unsigned)c->n_reactors), dim3(kBS), lds, (hipStream_t)stream,
                     m->dev, c->energy, c->n_reactors, c->P, c->tau, c->T_in, c->Y_in, x, J);
  HIP_OK(hipGetLastError());
  return PSR_OK;
}

// ------------------------------------------------------------ finite-difference Jacobian

namespace fd {

constexpr double kRel = 1.4901161193847656e-08;  // 2^-26, about the square root of FP64 epsilon
constexpr double kFloorY = 1e-10;                // smallest |x_j| the step is scaled by (species rows)
constexpr int kThreads = 256;

// Forward-difference step of unknown x_j: the representable difference
// (x_j + h) - x_j of the nominal step h = 2^-26 max(|x_j|, floor).
__device__ __forceinline__ double step(double xj, double floor_) {
  const double h = kRel * fmax(fabs(xj), floor_);
  return (xj + h) - xj;
}

// Row j of every reactor's perturbed state: x_j + step(x_j).
__global__ void __launch_bounds__(kThreads) k_perturb(const double *__restrict__ x, double *__restrict__ xp,
                                                      int64_t B, int j, double floor_) {
  const size_t row = (size_t)j * (size_t)B;
  for (int64_t b = blockIdx.x * (int64_t)kThreads + threadIdx.x; b < B; b += (int64_t)gridDim.x * kThreads) {
    const double xj = x[row + b];
    xp[row + b] = xj + step(xj, floor_);
  }
}

// Column j of every reactor's Jacobian, (F(x + h e_j) - F(x)) / h, then row j
// of the perturbed state back to x_j.  Reads of F are coalesced over reactors.
__global__ void __launch_bounds__(kThreads) k_column(const double *__restrict__ x, double *__restrict__ xp,
                                                     const double *__restrict__ F0, const double *__restrict__ Fp,
                                                     double *__restrict__ J, int64_t B, int n, int j, double floor_) {
  const size_t row = (size_t)j * (size_t)B;
  const size_t nn = (size_t)n * (size_t)n;
  for (int64_t b = blockIdx.x * (int64_t)kThreads + threadIdx.x; b < B; b += (int64_t)gridDim.x * kThreads) {
    const double xj = x[row + b];
    const double h = step(xj, floor_);
    double *Jb = J + (size_t)b * nn + j;
    for (int r = 0; r < n; r++) {
      const size_t i = (size_t)r * (size_t)B + b;
      Jb[(size_t)r * n] = (Fp[i] - F0[i]) / h;
    }
    xp[row + b] = xj;
  }
}

}  // namespace fd

extern "C" psr_status psr_jacobian_fd(psr_mech_t m, const psr_conditions *c, const double *x, double *J,
                                      double *work, void *stream) {
  psr_status st = check_cond(m, c);
  if (st != PSR_OK) return st;
  if (!x || !J || !work) return fail(PSR_EINVAL, "null x, J or work");
  const hipStream_t s = (hipStream_t)stream;
  const int n = n_unknowns(m->dev, c->energy);
  const int64_t B = c->n_reactors;
  const size_t nB = (size_t)n * (size_t)B;
  double *F0 = work, *Fp = work + nB, *xp = work + 2 * nB;
  const int64_t blocks = (B + fd::kThreads - 1) / fd::kThreads;
  const unsigned grid = (unsigned)std::min<int64_t>(blocks, 4096);
  HIP_OK(hipMemcpyAsync(xp, x, nB * sizeof(double), hipMemcpyDeviceToDevice, s));
  st = psr_residual(m, c, x, F0, nullptr, stream);
  if (st != PSR_OK) return st;
  for (int j = 0; j < n; j++) {
    const double floor_ = j < m->N ? fd::kFloorY : 1.0;
    hipLaunchKernelGGL(fd::k_perturb, dim3(grid), dim3(fd::kThreads), 0, s, x, xp, B, j, floor_);
    HIP_OK(hipGetLastError());
    st = psr_residual(m, c, xp, Fp, nullptr, stream);
    if (st != PSR_OK) return st;
    hipLaunchKernelGGL(fd::k_column, dim3(grid), dim3(fd::kThreads), 0, s, x, xp, F0, Fp, J, B, n, j, floor_);
    HIP_OK(hipGetLastError());
  }
  return PSR_OK;
}

// ------------------------------------------- allocation-free FD Jacobian

// Scratch of psr_jacobian_fd_noalloc: the three n x B work arrays of the
// finite-difference Jacobian (F(x), F at the perturbed state, the perturbed
// state) live in this file-scope device array, one copy per device, held
// until the process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kFdScratchDoubles = (size_t)4 << 20;  // 4 Mi doubles, 32 MiB per device
static __device__ __align__(256) double scratch[kFdScratchDoubles];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device, looked up once per
// device (the device current during the lookup) and kept.
static psr_status scratch_address(double **out) {
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PSR_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char msg[160];
      snprintf(msg, sizeof msg, "hipGetSymbolAddress of the FD scratch failed: %s", hipGetErrorString(e));
      return fail(PSR_EDEVICE, msg);
    }
    addr[dev] = static_cast<double *>(p);
  }
  *out = addr[dev];
  return PSR_OK;
}

extern "C" psr_status psr_jacobian_fd_noalloc(psr_mech_t m, const psr_conditions *c, const double *x,
                                              double *J, void *stream) {
  psr_status st = check_cond(m, c);
  if (st != PSR_OK) return st;
  if (!x || !J) return fail(PSR_EINVAL, "null x or J");
  const int n = n_unknowns(m->dev, c->energy);
  const size_t need = 3 * (size_t)n * (size_t)c->n_reactors;
  if (need > kFdScratchDoubles) {
    char msg[200];
    snprintf(msg, sizeof msg,
             "3 n B = %zu doubles exceeds the %zu-double scratch of psr_jacobian_fd_noalloc "
             "(use psr_jacobian_fd with a caller-owned work buffer)", need, kFdScratchDoubles);
    return fail(PSR_EINVAL, msg);
  }
  double *work = nullptr;
  st = scratch_address(&work);
  if (st != PSR_OK) return st;
  return psr_jacobian_fd(m, c, x, J, work, stream);
}

// Device scratch of the large-matrix LU entry point: one buffer per (device,
// stream), grown on demand and kept for the life of the process.  Launches on
// one stream are ordered, so a buffer is never used by two factorisations at
// once; calls on different streams or host threads get different buffers.
static psr_status lu_scratch(int dev, hipStream_t stream, size_t bytes, float **out) {
  struct Buf { int dev; hipStream_t stream; float *p; size_t bytes; };
  static std::mutex mu;
  static std::vector<Buf> bufs;
  std::lock_guard<std::mutex> lock(mu);
  Buf *b = nullptr;
  for (Buf &e : bufs)
    if (e.dev == dev && e.stream == stream) b = &e;
  if (!b) {
    bufs.push_back({dev, stream, nullptr, 0});
    b = &bufs.back();
  }
  if (b->bytes < bytes) {
    // the old buffer may still be read by earlier launches on this stream
    if (b->p) {
      HIP_OK(hipStreamSynchronize(stream));
      HIP_OK(hipFree(b->p));
    }
    b->p = nullptr;
    b->bytes = 0;
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return fail(PSR_ENOMEM, "LU scratch allocation failed");
    b->p = reinterpret_cast<float *>(p);
    b->bytes = bytes;
  }
  *out = b->p;
  return PSR_OK;
}

// One wavefront per matrix, working copies in a library-owned area per
// (device, stream).
template <typename T>
static psr_status lu_factor_wave(int n, int64_t batch, double *A, int *piv, int *info, hipStream_t stream) {
  int dev = 0, ncu = 0, per_cu = 0;
  const size_t lds = sizeof(psr::luw::WaveLds<T>) * psr::luw::kW;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lu_factor_wave<T>, 256, lds));
  if (per_cu < 1) return fail(PSR_EUNSUPPORTED, "LU kernel does not fit a compute unit");
  const int ldw = psr::luw::pad_ld(n);
  const int64_t grid = std::min<int64_t>((batch + psr::luw::kW - 1) / psr::luw::kW, (int64_t)ncu * per_cu);
  float *work = nullptr;
  const psr_status st =
      lu_scratch(dev, stream, (size_t)grid * psr::luw::kW * psr::luw::pad_rows(n) * ldw * sizeof(T), &work);
  if (st != PSR_OK) return st;
  hipLaunchKernelGGL(k_lu_factor_wave<T>, dim3((unsigned)grid), dim3(256), lds, stream, n, ldw, batch, A, piv, info,
                     reinterpret_cast<T *>(work));
  HIP_OK(hipGetLastError());
  return PSR_OK;
}

extern "C" psr_status psr_lu_factor_batch(int32_t n, int64_t batch, int32_t precision, double *A,
                                          int32_t *piv, int32_t *info, void *stream) {
  if (n <= 0 || batch <= 0 || !A || !piv || !info) return fail(PSR_EINVAL, "bad LU arguments");
  if (batch > 0x7fffffffLL) return fail(PSR_EUNSUPPORTED, "batch above 2^31-1");
  const int lda = (n % 2 == 0) ? n + 1 : n;
  const bool f32 = precision == PSR_MIXED;
  if (n > 64 && n <= (f32 ? psr::luw::Prec<float>::NMAX : psr::luw::Prec<double>::NMAX))
    return f32 ? lu_factor_wave<float>(n, batch, A, piv, info, (hipStream_t)stream)
               : lu_factor_wave<double>(n, batch, A, piv, info, (hipStream_t)stream);
  const size_t lds = ((size_t)n * lda * (f32 ? 4 : 8) + 7) / 8 * 8 + (kBS + 8) * 8 + (size_t)n * 4 + 8;
  if (lds > (size_t)lds_limit_bytes()) return fail(PSR_EUNSUPPORTED, "matrix too large for LDS");
  if (f32)
    hipLaunchKernelGGL(k_lu_factor<float>, dim3((unsigned)batch), dim3(kBS), lds, (hipStream_t)stream,
                       n, A, piv, info);
  else
    hipLaunchKernelGGL(k_lu_factor<double>, dim3((unsigned)batch), dim3(kBS), lds, (hipStream_t)stream,
                       n, A, piv, info);
  HIP_OK(hipGetLastError());
  return PSR_OK;
}

extern "C" psr_status psr_lu_solve_batch(int32_t n, int64_t batch, const double *LU, const int32_t *piv,
                                         double *b, void *stream) {
  if (n <= 0 || batch <= 0 || !LU || !piv || !b) return fail(PSR_EINVAL, "bad LU arguments");
  if (batch > 0x7fffffffLL) return fail(PSR_EUNSUPPORTED, "batch above 2^31-1");
  const int lda = (n % 2 == 0) ? n + 1 : n;
  if (n <= 256) {
    int dev = 0, ncu = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t grid = std::min<int64_t>((batch + 3) / 4, (int64_t)ncu * 8);
    hipLaunchKernelGGL(k_lu_solve_wave, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, n, batch, LU, piv,
                       b);
    HIP_OK(hipGetLastError());
    return PSR_OK;
  }
  const size_t lds = (size_t)n * lda * 8 + (size_t)n * 8 + (size_t)n * 4 + 8;
  if (lds > (size_t)lds_limit_bytes()) return fail(PSR_EUNSUPPORTED, "matrix too large for LDS");
  hipLaunchKernelGGL(k_lu_solve, dim3((unsigned)batch), dim3(kBS), lds, (hipStream_t)stream, n, LU, piv,
                     b);
  HIP_OK(hipGetLastError());
  return PSR_OK;
}

// ------------------------------------------------------------ host: solve

static Opts to_dev_opts(const psr_solve_opts *o) {
  Opts d;
  d.precision = o->precision; d.scheduler = o->scheduler;
  d.rtol = o->rtol; d.atol_Y = o->atol_Y; d.atol_T = o->atol_T; d.ftol = o->ftol;
  d.lambda_min = o->lambda_min; d.T_min = o->T_min; d.T_max = o->T_max;
  d.ts_rtol = o->ts_rtol; d.ts_atol_Y = o->ts_atol_Y; d.ts_atol_T = o->ts_atol_T;
  d.ts_neg_tol = o->ts_neg_tol; d.h0 = o->h0; d.h_max = o->h_max; d.h_min = o->h_min;
  d.nw_h_ratio = o->nw_h_ratio; d.nw_max_it = o->nw_max_it; d.nw_every = o->nw_every;
  d.max_lin = o->max_lin; d.max_refine = o->max_refine;
  d.refine_tol = o->refine_tol;
  d.atol_lnM = o->atol_lnM; d.ts_atol_lnM = o->ts_atol_lnM;
  d.lnM_step = o->lnM_step;
  d.ct_ratio = o->ct_ratio; d.ct_tau_min = o->ct_tau_min; d.ct_min_step = o->ct_min_step;
  d.mixed_max_n = o->mixed_max_n;
  return d;
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Wavefront engine choice: NP (register row length) for n unknowns, or 0.
static int wave_np(int n) { return n <= 16 ? 16 : (n <= 32 ? 32 : (n <= 64 ? 64 : 0)); }

struct WavePlan {
  int NP = 0, rpw = 0;
  int per_cu_cap = 0;  // persistent grid: workgroups per compute unit (0 = all that fit)
  size_t lds = 0;
  int stride = 0;  // plain scheduler area, doubles per reactor
};

// rpw_req: wavefronts per workgroup asked for (0 = the most that fit); the
// largest of 4, 2, 1 not above it that fits the LDS is taken.
static WavePlan wave_plan(psr_mech_t m, int energy, bool mixed, int engine, int rpw_req = 0) {
  WavePlan w;
  const int n = n_unknowns(m->dev, energy);
  // the wavefront engine implements the isothermal and energy-balance rows only
  if (engine == 1 || !m->dev.packed || energy == 2) return w;
  const int NP = wave_np(n);
  if (!NP) return w;
  const size_t tb = wk::wave_area_off(m->N, m->I, m->nnz);
  size_t per = 0;
  switch (NP) {
    case 16: per = (size_t)psr::wave::WArea<16>::doubles(n) * 8; break;
    case 32: per = (size_t)psr::wave::WArea<32>::doubles(n) * 8; break;
    default: per = (size_t)psr::wave::WArea<64>::doubles(n) * 8; break;
  }
  const size_t lim = (size_t)lds_limit_bytes();
  for (int rpw = 4; rpw >= 1; rpw /= 2) {
    if (rpw_req > 0 && rpw > rpw_req) continue;
    if (tb + rpw * per <= lim) {
      w.NP = NP;
      w.rpw = rpw;
      w.lds = tb + rpw * per;
      break;
    }
  }
  if (!w.NP) return w;
  switch (NP) {
    case 16: w.stride = mixed ? wk::plain_stride<16, true>(n) : wk::plain_stride<16, false>(n); break;
    case 32: w.stride = mixed ? wk::plain_stride<32, true>(n) : wk::plain_stride<32, false>(n); break;
    default: w.stride = mixed ? wk::plain_stride<64, true>(n) : wk::plain_stride<64, false>(n); break;
  }
  return w;
}

// Streams on which the groups of one persistent solve run side by side
// (default priority), created on first use and kept for the process.
static psr_status group_stream(int dev, int i, hipStream_t *out) {
  static std::mutex mu;  // calls from several host threads share the pool
  static std::vector<std::vector<hipStream_t>> pool;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)pool.size() <= dev) pool.resize(dev + 1);
  auto &v = pool[dev];
  while ((int)v.size() <= i) {
    hipStream_t s;
    HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    v.push_back(s);
  }
  *out = v[i];
  return PSR_OK;
}

// Drives the plain scheduler after its first round: `period(s)` enqueues one
// check period (counter reset + `per` rounds) on stream s; the host reads the
// active count after each period.  With use_graph the period is captured once
// as a HIP graph on a library stream (after the work already on `stream`) and
// replayed; the counter reset is a kernel, not a memset node.
template <typename F>
static psr_status drive_plain(hipStream_t stream, bool use_graph, int *counters, int per, int max_rounds,
                              F period, int *rounds_out) {
  int active = 1, rounds = 0;
  hipStream_t s = stream;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev = nullptr;
  if (use_graph) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    const psr_status st = group_stream(dev, 0, &s);
    if (st != PSR_OK) return st;
    HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_OK(hipEventRecord(ev, stream));
    HIP_OK(hipStreamWaitEvent(s, ev, 0));
    HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    period(s);
    HIP_OK(hipStreamEndCapture(s, &graph));
    HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  while (active > 0 && rounds < max_rounds) {
    if (exec) HIP_OK(hipGraphLaunch(exec, s));
    else period(s);
    rounds += per;
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(&active, counters, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  if (exec) {
    HIP_OK(hipGraphExecDestroy(exec));
    HIP_OK(hipGraphDestroy(graph));
    HIP_OK(hipEventRecord(ev, s));
    HIP_OK(hipStreamWaitEvent(stream, ev, 0));
    HIP_OK(hipEventDestroy(ev));
  }
  *rounds_out = rounds;
  if (active > 0) return fail(PSR_EDEVICE, "plain scheduler did not retire every reactor");
  return PSR_OK;
}

template <int NP, bool MIXED>
static psr_status launch_wave(const GroupDev &gd, const Opts &od, const WavePlan &w, int scheduler,
                              RState *states, int *counters, double *area, hipStream_t stream,
                              int max_rounds, int *rounds_out, bool use_graph) {
  const int64_t B = gd.B;
  const int threads = 64 * w.rpw;
  if (scheduler == PSR_PERSISTENT) {
    int dev = 0, ncu = 0, per_cu = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wk::k_wpersist<NP, MIXED>, threads, w.lds));
    if (w.per_cu_cap > 0) per_cu = std::min(per_cu, w.per_cu_cap);
    if (per_cu < 1) per_cu = 1;
    const int64_t need = (B + w.rpw - 1) / w.rpw;
    const int64_t grid = std::min<int64_t>(need, (int64_t)ncu * per_cu);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, stream, counters, 64);
    hipLaunchKernelGGL((wk::k_wpersist<NP, MIXED>), dim3((unsigned)grid), dim3(threads), w.lds, stream, gd, od,
                       states, counters);
    HIP_OK(hipGetLastError());
    *rounds_out = 0;
    return PSR_OK;
  }
  const unsigned grid = (unsigned)((B + w.rpw - 1) / w.rpw);
  hipLaunchKernelGGL((wk::k_wround<NP, MIXED, true>), dim3(grid), dim3(threads), w.lds, stream, gd, od, states,
                     area, w.stride, w.rpw, counters);
  HIP_OK(hipGetLastError());
  const int check_every = 4;
  auto period = [&](hipStream_t s) {
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, counters, 1);
    for (int r = 0; r < check_every; r++)
      hipLaunchKernelGGL((wk::k_wround<NP, MIXED, false>), dim3(grid), dim3(threads), w.lds, s, gd, od, states,
                         area, w.stride, w.rpw, counters);
  };
  return drive_plain(stream, use_graph, counters, check_every, max_rounds, period, rounds_out);
}

static psr_status run_wave(const GroupDev &gd, const Opts &od, const WavePlan &w, bool mixed, int scheduler,
                           RState *states, int *counters, double *area, hipStream_t stream, int max_rounds,
                           int *rounds, bool use_graph) {
  switch (w.NP) {
    case 16:
      return mixed ? launch_wave<16, true>(gd, od, w, scheduler, states, counters, area, stream, max_rounds, rounds, use_graph)
                   : launch_wave<16, false>(gd, od, w, scheduler, states, counters, area, stream, max_rounds, rounds, use_graph);
    case 32:
      return mixed ? launch_wave<32, true>(gd, od, w, scheduler, states, counters, area, stream, max_rounds, rounds, use_graph)
                   : launch_wave<32, false>(gd, od, w, scheduler, states, counters, area, stream, max_rounds, rounds, use_graph);
    default:
      return mixed ? launch_wave<64, true>(gd, od, w, scheduler, states, counters, area, stream, max_rounds, rounds, use_graph)
                   : launch_wave<64, false>(gd, od, w, scheduler, states, counters, area, stream, max_rounds, rounds, use_graph);
  }
}

// Persistent solves of several groups run concurrently, each in its own
// workspace region; otherwise groups share one region and run in turn.
static bool concurrent_groups(int32_t n_groups, const psr_solve_opts *o) {
  return n_groups > 1 && o->scheduler == PSR_PERSISTENT;
}

// Workspace of one group: states [B], plain-scheduler areas [B][persist],
// counters.
static size_t group_ws(const psr_group &g, const psr_solve_opts *o) {
  Layout L;
  const bool mixed = o->precision == PSR_MIXED;
  block_layout(g.mech, g.cond.energy, mixed, L);
  size_t bytes = align256(sizeof(RState) * (size_t)g.cond.n_reactors) + 256;
  if (o->scheduler == PSR_PERSISTENT) bytes += align256(sizeof(int) * (size_t)g.cond.n_reactors);  // queue order
  const WavePlan w = wave_plan(g.mech, g.cond.energy, mixed, o->engine, o->rpw);
  if (o->scheduler == PSR_PLAIN)
    bytes += align256((size_t)(w.NP ? w.stride : L.persist + L.mat_total) * 8 * g.cond.n_reactors);
  else if (!w.NP && L.split)
    bytes += align256((size_t)L.mat_total * 8 * block_grid(L, mixed, g.cond.n_reactors, o->grid_per_cu));
  return bytes;
}

// One fused launch for the groups of a persistent solve (wk::k_fused): 2 to
// kMaxFused groups, at most one on the wavefront engine (four wavefronts per
// workgroup), automatic launch shape.  lds: the largest group's LDS plus the
// broadcast slot; mat_stride: the largest HBM matrix area of a workgroup-
// engine group; grid: resident workgroups.
struct FusedPlan {
  bool ok = false;
  int NP = 0;
  size_t lds = 0;
  int next_off = 0;
  int64_t grid = 0, mat_stride = 0;
};

static FusedPlan fused_plan(const psr_group *groups, int32_t n_groups, const psr_solve_opts *o) {
  FusedPlan f;
  if (o->scheduler != PSR_PERSISTENT || n_groups < 2 || n_groups > wk::kMaxFused) return f;
  if (o->engine != 0 || o->rpw != 0 || o->grid_per_cu != 0) return f;
  const bool mixed = o->precision == PSR_MIXED;
  int waves = 0;
  size_t lds = 0;
  int64_t mat = 0, total = 0;
  for (int gi = 0; gi < n_groups; gi++) {
    const psr_group &g = groups[gi];
    if (!g.mech || g.cond.n_reactors <= 0) return f;
    total += g.cond.n_reactors;
    const WavePlan w = wave_plan(g.mech, g.cond.energy, mixed, 0, 4);
    if (w.NP) {
      if (w.rpw != 4) return f;
      waves++;
      f.NP = w.NP;
      lds = std::max(lds, w.lds);
    } else {
      Layout L;
      if (!block_layout(g.mech, g.cond.energy, mixed, L)) return f;
      lds = std::max(lds, (size_t)L.total * 8);
      if (L.split) mat = std::max<int64_t>(mat, L.mat_total);
    }
  }
  if (waves > 1 || total > 0x7fffffffLL) return f;
  f.next_off = (int)wk::align16(lds);
  f.lds = (size_t)f.next_off + 16;
  if (f.lds > (size_t)lds_limit_bytes()) return f;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return f;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return f;
  hipError_t e;
#define PSR_FUSED_OCC(NP_, M_) hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wk::k_fused<NP_, M_>, 256, f.lds)
  switch (f.NP) {
    case 0: e = mixed ? PSR_FUSED_OCC(0, true) : PSR_FUSED_OCC(0, false); break;
    case 16: e = mixed ? PSR_FUSED_OCC(16, true) : PSR_FUSED_OCC(16, false); break;
    case 32: e = mixed ? PSR_FUSED_OCC(32, true) : PSR_FUSED_OCC(32, false); break;
    default: e = mixed ? PSR_FUSED_OCC(64, true) : PSR_FUSED_OCC(64, false); break;
  }
#undef PSR_FUSED_OCC
  if (e != hipSuccess || per_cu < 1) return f;
  f.grid = std::min<int64_t>(total, (int64_t)ncu * per_cu);
  f.mat_stride = mat;
  f.ok = true;
  return f;
}

extern "C" size_t psr_workspace_bytes(const psr_group *groups, int32_t n_groups,
                                      const psr_solve_opts *opts) {
  if (!groups || n_groups <= 0 || !opts) return 0;
  size_t mx = 0, sum = 0;
  for (int gi = 0; gi < n_groups; gi++) {
    if (!groups[gi].mech || groups[gi].cond.n_reactors <= 0) return 0;
    const size_t b = group_ws(groups[gi], opts);
    mx = std::max(mx, b);
    sum += align256(b);
  }
  const FusedPlan f = fused_plan(groups, n_groups, opts);
  if (f.ok) sum += 256 + align256((size_t)f.grid * f.mat_stride * 8);  // queue counter, HBM matrices
  return concurrent_groups(n_groups, opts) ? sum : mx;
}

static psr_status check_opts(const psr_solve_opts *o) {
  if (!o) return fail(PSR_EINVAL, "null opts");
  if (o->precision != PSR_FP64 && o->precision != PSR_MIXED) return fail(PSR_EINVAL, "bad precision");
  if (o->scheduler != PSR_PLAIN && o->scheduler != PSR_PERSISTENT) return fail(PSR_EINVAL, "bad scheduler");
  if (!(o->rtol > 0) || !(o->atol_Y >= 0) || !(o->atol_T >= 0) || !(o->ftol > 0) ||
      !(o->lambda_min >= 0 && o->lambda_min <= 1) || !(o->T_min < o->T_max) || !(o->ts_rtol > 0) ||
      !(o->h0 > 0) || !(o->h_min > 0) || !(o->h_max > 0) || o->nw_max_it < 1 || o->nw_every < 1 ||
      o->max_lin < 1 || o->max_refine < 0 || o->engine < 0 || o->engine > 2 || o->use_graph < 0 ||
      o->use_graph > 1 || !(o->refine_tol > 0 && o->refine_tol < 1) || !(o->atol_lnM >= 0) ||
      !(o->ts_atol_lnM >= 0) || !(o->rpw == 0 || o->rpw == 1 || o->rpw == 2 || o->rpw == 4) ||
      o->grid_per_cu < 0 || o->grid_per_cu > 32 || !(o->lnM_step > 0) ||
      !(o->ct_ratio >= 0) || !(o->ct_tau_min > 0) || !(o->ct_min_step > 0) || o->order < 0 ||
      o->order > 1 || o->mixed_max_n < 0)
    return fail(PSR_EINVAL, "option out of range");
  return PSR_OK;
}


// One group of a solve: its device view, engine plan and workspace region.
struct GroupRun {
  GroupDev gd;
  Layout L;
  WavePlan wplan;
  size_t lds = 0;
  bool mixed = false;
  RState *states = nullptr;
  int *counters = nullptr;
  int *order = nullptr;  // persistent scheduler: device queue order [B]
  double *area = nullptr;
  int rounds = 0;
  std::vector<double> host_tau;  // host copies for the queue order (alive until the call returns)
  std::vector<int> host_order;
};

static psr_status prepare_group(const psr_group &g, const psr_solve_opts *o, void *ws, GroupRun &r) {
  r.mixed = o->precision == PSR_MIXED;
  const bool fits = block_layout(g.mech, g.cond.energy, r.mixed, r.L);
  r.lds = (size_t)r.L.total * 8;
  r.wplan = wave_plan(g.mech, g.cond.energy, r.mixed, o->engine, o->rpw);
  r.wplan.per_cu_cap = o->grid_per_cu;
  if (o->engine == 2 && !r.wplan.NP)
    return fail(PSR_EUNSUPPORTED, "wavefront engine needs n <= 64 and a mechanism that fits its LDS");
  if (!r.wplan.NP && !fits)
    return fail(PSR_EUNSUPPORTED, "reactor working set (" + std::to_string(r.lds) +
                                      " B without matrices) exceeds the LDS of one workgroup");
  GroupDev &gd = r.gd;
  gd.m = g.mech->dev; gd.energy = g.cond.energy; gd.B = g.cond.n_reactors;
  gd.P = g.cond.P; gd.tau = g.cond.tau; gd.Tin = g.cond.T_in; gd.Yin = g.cond.Y_in;
  gd.x = g.x_inout; gd.status = g.status; gd.nlin = g.n_lin;
  gd.order = nullptr;
  char *p = reinterpret_cast<char *>(ws);
  r.states = reinterpret_cast<RState *>(p);
  p += align256(sizeof(RState) * (size_t)gd.B);
  r.counters = reinterpret_cast<int *>(p);
  p += 256;
  if (o->scheduler == PSR_PERSISTENT) {
    r.order = reinterpret_cast<int *>(p);
    p += align256(sizeof(int) * (size_t)gd.B);
  }
  r.area = reinterpret_cast<double *>(p);
  return PSR_OK;
}

// Device queue order of a persistent group: longest residence time first
// (ties by batch index; tau that is not a positive finite number goes last).
// Reads tau back on `stream` (synchronising it) and uploads the permutation.
static psr_status queue_order(GroupRun &r, hipStream_t stream) {
  const int64_t B = r.gd.B;
  r.host_tau.resize(B);
  r.host_order.resize(B);
  HIP_OK(hipMemcpyAsync(r.host_tau.data(), r.gd.tau, sizeof(double) * B, hipMemcpyDeviceToHost, stream));
  HIP_OK(hipStreamSynchronize(stream));
  std::vector<double> &t = r.host_tau;
  for (double &v : t) v = (v > 0.0 && v < HUGE_VAL) ? v : -1.0;
  for (int64_t i = 0; i < B; i++) r.host_order[i] = (int)i;
  std::stable_sort(r.host_order.begin(), r.host_order.end(), [&](int a, int b) { return t[a] > t[b]; });
  HIP_OK(hipMemcpyAsync(r.order, r.host_order.data(), sizeof(int) * B, hipMemcpyHostToDevice, stream));
  r.gd.order = r.order;
  return PSR_OK;
}

// Issue the group's launches on `stream`.  Persistent scheduler: returns
// after the launches (asynchronous).  Plain scheduler: drives the rounds from
// the host and returns when every reactor has retired.
static psr_status launch_group(GroupRun &r, const psr_solve_opts *o, hipStream_t stream) {
  const Opts od = to_dev_opts(o);
  if (o->scheduler == PSR_PERSISTENT && o->order) {
    const psr_status st = queue_order(r, stream);
    if (st != PSR_OK) return st;
  }
  const GroupDev &gd = r.gd;
  const int64_t B = gd.B;
  const bool mixed = r.mixed;
  const Layout &L = r.L;
  const size_t lds = r.lds;
  RState *states = r.states;
  int *counters = r.counters;
  double *area = r.area;
  r.rounds = 0;
  if (r.wplan.NP)
    return run_wave(gd, od, r.wplan, mixed, o->scheduler, states, counters, area, stream, o->max_lin * 2 + 8,
                    &r.rounds, o->use_graph != 0);
  if (o->scheduler == PSR_PERSISTENT) {
    const int64_t grid = block_grid(L, mixed, B, o->grid_per_cu);
    if (grid <= 0) return fail(PSR_EDEVICE, "occupancy query failed");
    double *matws = L.split ? area : nullptr;  // one HBM matrix area per resident workgroup
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, stream, counters, 64);
    const bool big = L.n > 64;
    if (mixed && big)
      hipLaunchKernelGGL((k_persistent<true, true>), dim3((unsigned)grid), dim3(kBS), lds, stream, gd, od, states,
                         counters, matws);
    else if (mixed)
      hipLaunchKernelGGL((k_persistent<true, false>), dim3((unsigned)grid), dim3(kBS), lds, stream, gd, od,
                         states, counters, matws);
    else if (big)
      hipLaunchKernelGGL((k_persistent<false, true>), dim3((unsigned)grid), dim3(kBS), lds, stream, gd, od,
                         states, counters, matws);
    else
      hipLaunchKernelGGL((k_persistent<false, false>), dim3((unsigned)grid), dim3(kBS), lds, stream, gd, od,
                         states, counters, matws);
    HIP_OK(hipGetLastError());
    return PSR_OK;
  }
  const int check_every = 4;
  const bool big = L.n > 64;
  // k_round<MIXED, FIRST, BIG>
  auto launch_round = [&](hipStream_t s, bool first) {
#define PSR_ROUND(M, F, G)                                                                                    \
  hipLaunchKernelGGL((k_round<M, F, G>), dim3((unsigned)B), dim3(kBS), lds, s, gd, od, states, area, L.split, \
                     counters)
    if (mixed) {
      if (first) { if (big) PSR_ROUND(true, true, true); else PSR_ROUND(true, true, false); }
      else { if (big) PSR_ROUND(true, false, true); else PSR_ROUND(true, false, false); }
    } else {
      if (first) { if (big) PSR_ROUND(false, true, true); else PSR_ROUND(false, true, false); }
      else { if (big) PSR_ROUND(false, false, true); else PSR_ROUND(false, false, false); }
    }
#undef PSR_ROUND
  };
  launch_round(stream, true);
  HIP_OK(hipGetLastError());
  auto period = [&](hipStream_t s) {
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, counters, 1);
    for (int k = 0; k < check_every; k++) launch_round(s, false);
  };
  return drive_plain(stream, o->use_graph != 0, counters, check_every, o->max_lin * 2 + 8, period, &r.rounds);
}

// Add one group's totals to acc from its per-reactor controller states (the
// group must have finished: the copy is synchronous).
static psr_status collect_group(const GroupRun &r, psr_solve_stats *acc) {
  if (!acc) return PSR_OK;
  const int64_t B = r.gd.B;
  std::vector<RState> hs(B);
  HIP_OK(hipMemcpy(hs.data(), r.states, sizeof(RState) * B, hipMemcpyDeviceToHost));
  acc->reactors += B;
  for (const RState &s : hs) {
    acc->converged += s.status == RS_CONVERGED;
    acc->lin_total += s.n_lin;
    acc->lin_max = std::max<int64_t>(acc->lin_max, s.n_lin);
    acc->jac_total += s.n_jac;
    acc->fp64_fallbacks += s.n_fb64;
  }
  acc->rounds += r.rounds;
  return PSR_OK;
}


extern "C" psr_status psr_solve_batch(const psr_group *groups, int32_t n_groups, const psr_solve_opts *opts,
                                      void *workspace, size_t workspace_bytes, psr_solve_stats *stats,
                                      void *stream) {
  psr_status st = check_opts(opts);
  if (st != PSR_OK) return st;
  if (!groups || n_groups <= 0) return fail(PSR_EINVAL, "no groups");
  for (int gi = 0; gi < n_groups; gi++) {
    st = check_cond(groups[gi].mech, &groups[gi].cond);
    if (st != PSR_OK) return st;
    if (!groups[gi].x_inout || !groups[gi].status) return fail(PSR_EINVAL, "null x_inout or status");
  }
  const size_t need = psr_workspace_bytes(groups, n_groups, opts);
  if (!workspace || workspace_bytes < need)
    return fail(PSR_ENOMEM, "workspace smaller than psr_workspace_bytes() = " + std::to_string(need));
  if (stats) memset(stats, 0, sizeof(*stats));
  const hipStream_t cs = (hipStream_t)stream;
  const bool conc = concurrent_groups(n_groups, opts);
  std::vector<GroupRun> runs(n_groups);
  char *region = reinterpret_cast<char *>(workspace);
  for (int gi = 0; gi < n_groups; gi++) {
    st = prepare_group(groups[gi], opts, region, runs[gi]);
    if (st != PSR_OK) return st;
    if (conc) region += align256(group_ws(groups[gi], opts));
  }
  const FusedPlan fp = fused_plan(groups, n_groups, opts);
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  HIP_OK(hipEventRecord(e0, cs));
  if (fp.ok) {
    // every group in one launch over one queue: workgroup-engine groups
    // largest n first, then the wavefront-engine group
    int *fcounter = reinterpret_cast<int *>(region);
    double *fmat = reinterpret_cast<double *>(region + 256);
    std::vector<int> seq;
    for (int gi = 0; gi < n_groups; gi++)
      if (!runs[gi].wplan.NP) seq.push_back(gi);
    std::stable_sort(seq.begin(), seq.end(), [&](int a, int b) {
      return n_unknowns(groups[a].mech->dev, groups[a].cond.energy) >
             n_unknowns(groups[b].mech->dev, groups[b].cond.energy);
    });
    for (int gi = 0; gi < n_groups; gi++)
      if (runs[gi].wplan.NP) seq.push_back(gi);
    wk::FusedDev fd{};
    int64_t start = 0;
    for (int k = 0; k < n_groups; k++) {
      GroupRun &r = runs[seq[k]];
      if (opts->order) {
        st = queue_order(r, cs);
        if (st != PSR_OK) return st;
      }
      fd.grp[k].g = r.gd;
      fd.grp[k].states = r.states;
      fd.grp[k].start = start;
      fd.grp[k].wave = r.wplan.NP ? 1 : 0;
      fd.grp[k].split = r.L.split;
      start += r.gd.B;
    }
    fd.ng = n_groups;
    fd.total = start;
    fd.matws = fmat;
    fd.mat_stride = fp.mat_stride;
    fd.next_off = fp.next_off;
    const Opts od = to_dev_opts(opts);
    const bool mixed = opts->precision == PSR_MIXED;
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, cs, fcounter, 64);
    const dim3 grid((unsigned)fp.grid), blk(256);
#define PSR_FUSED(NP_, M_) hipLaunchKernelGGL((wk::k_fused<NP_, M_>), grid, blk, fp.lds, cs, fd, od, fcounter)
    switch (fp.NP) {
      case 0: if (mixed) PSR_FUSED(0, true); else PSR_FUSED(0, false); break;
      case 16: if (mixed) PSR_FUSED(16, true); else PSR_FUSED(16, false); break;
      case 32: if (mixed) PSR_FUSED(32, true); else PSR_FUSED(32, false); break;
      default: if (mixed) PSR_FUSED(64, true); else PSR_FUSED(64, false); break;
    }
#undef PSR_FUSED
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(e1, cs));
    HIP_OK(hipEventSynchronize(e1));
  } else if (conc) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::vector<hipEvent_t> done(n_groups);
    // launch order: largest systems first when ordering by cost
    std::vector<int> seq(n_groups);
    for (int gi = 0; gi < n_groups; gi++) seq[gi] = gi;
    if (opts->order)
      std::stable_sort(seq.begin(), seq.end(), [&](int a, int b) {
        return n_unknowns(groups[a].mech->dev, groups[a].cond.energy) >
               n_unknowns(groups[b].mech->dev, groups[b].cond.energy);
      });
    for (int si = 0; si < n_groups; si++) {
      const int gi = seq[si];
      hipStream_t gs;
      st = group_stream(dev, gi, &gs);
      if (st != PSR_OK) return st;
      HIP_OK(hipStreamWaitEvent(gs, e0, 0));
      st = launch_group(runs[gi], opts, gs);
      if (st != PSR_OK) return st;
      HIP_OK(hipEventCreateWithFlags(&done[gi], hipEventDisableTiming));
      HIP_OK(hipEventRecord(done[gi], gs));
      HIP_OK(hipStreamWaitEvent(cs, done[gi], 0));
    }
    HIP_OK(hipEventRecord(e1, cs));
    HIP_OK(hipEventSynchronize(e1));
    for (hipEvent_t e : done) hipEventDestroy(e);
  } else {
    // the groups run in turn on one workspace region: each group's totals are
    // read before the next group overwrites its controller states
    for (int gi = 0; gi < n_groups; gi++) {
      st = launch_group(runs[gi], opts, cs);
      if (st != PSR_OK) return st;
      if (stats && n_groups > 1) {
        HIP_OK(hipStreamSynchronize(cs));
        st = collect_group(runs[gi], stats);
        if (st != PSR_OK) return st;
      }
    }
    HIP_OK(hipEventRecord(e1, cs));
    HIP_OK(hipEventSynchronize(e1));
  }
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (conc || n_groups == 1) {
    for (int gi = 0; gi < n_groups; gi++) {
      st = collect_group(runs[gi], stats);
      if (st != PSR_OK) return st;
    }
  }
  if (stats) stats->kernel_ms = ms;
  return PSR_OK;
}

// ------------------------------------------------------------ host: continuation sweep

// Each step is one batched solve whose swept condition points at that step's
// row of `values` and whose initial guess is the state the previous step left
// in x_inout (the warm start of a continuation).  The state and status after
// each step are copied out on the same stream before the next solve starts.
extern "C" psr_status psr_sweep_batch(const psr_group *group, int32_t param, int32_t n_steps,
                                      const double *values, const psr_solve_opts *opts, void *workspace,
                                      size_t workspace_bytes, double *x_path, int32_t *status_path,
                                      psr_solve_stats *stats, void *stream) {
  if (!group) return fail(PSR_EINVAL, "null group");
  if (param != PSR_SWEEP_T_IN && param != PSR_SWEEP_TAU) return fail(PSR_EINVAL, "unknown sweep parameter");
  if (n_steps < 1) return fail(PSR_EINVAL, "n_steps must be >= 1");
  if (!values) return fail(PSR_EINVAL, "null values");
  if (!group->mech) return fail(PSR_EINVAL, "null mechanism");
  const hipStream_t cs = (hipStream_t)stream;
  const int64_t B = group->cond.n_reactors;
  if (B <= 0) return fail(PSR_EINVAL, "n_reactors must be positive");
  const int64_t n = psr_num_unknowns(group->mech, group->cond.energy);
  psr_group g = *group;
  psr_solve_stats total{}, one{};
  for (int32_t k = 0; k < n_steps; k++) {
    const double *row = values + (size_t)k * (size_t)B;
    if (param == PSR_SWEEP_T_IN) g.cond.T_in = row;
    else g.cond.tau = row;
    psr_status st = psr_solve_batch(&g, 1, opts, workspace, workspace_bytes, stats ? &one : nullptr, stream);
    if (st != PSR_OK) return st;
    if (x_path)
      HIP_OK(hipMemcpyAsync(x_path + (size_t)k * (size_t)(n * B), g.x_inout, sizeof(double) * (size_t)(n * B),
                            hipMemcpyDeviceToDevice, cs));
    if (status_path)
      HIP_OK(hipMemcpyAsync(status_path + (size_t)k * (size_t)B, g.status, sizeof(int32_t) * (size_t)B,
                            hipMemcpyDeviceToDevice, cs));
    if (stats) {
      total.reactors += one.reactors;
      total.converged += one.converged;
      total.lin_total += one.lin_total;
      total.lin_max = std::max(total.lin_max, one.lin_max);
      total.jac_total += one.jac_total;
      total.fp64_fallbacks += one.fp64_fallbacks;
      total.rounds += one.rounds;
      total.kernel_ms += one.kernel_ms;
    }
  }
  HIP_OK(hipStreamSynchronize(cs));
  if (stats) *stats = total;
  return PSR_OK;
}

// ------------------------------------------------------------ host: autotuner

namespace {

// Device buffers of one group's sample: copies of the first S reactors' state
// and inlet composition ([var][S]), and the sample's own status array.
struct TuneSample {
  psr_group g{};
  double *x0 = nullptr, *x = nullptr, *Yin = nullptr;
  int32_t *status = nullptr;
  size_t xbytes = 0;
};

void free_samples(std::vector<TuneSample> &v) {
  for (TuneSample &t : v) {
    if (t.x0) (void)hipFree(t.x0);
    if (t.x) (void)hipFree(t.x);
    if (t.Yin) (void)hipFree(t.Yin);
    if (t.status) (void)hipFree(t.status);
    t = TuneSample{};
  }
}

std::string tune_key(const psr_group *groups, int32_t n_groups, const psr_solve_opts *o, int64_t sample) {
  int dev = 0, ncu = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
  for (char &ch : arch)
    if (ch == ' ' || ch == '\t') ch = '_';
  std::string k = arch + "/cu" + std::to_string(ncu) + "/p" + std::to_string(o->precision) + "/s" +
                  std::to_string(o->scheduler);
  for (int gi = 0; gi < n_groups; gi++) {
    const psr_mech_t m = groups[gi].mech;
    const int64_t S = std::min<int64_t>(sample, groups[gi].cond.n_reactors);
    k += "/g" + std::to_string(m->N) + "," + std::to_string(m->I) + "," + std::to_string(m->nnz) + "," +
         std::to_string(m->dev.soot ? 1 : 0) + "," + std::to_string(groups[gi].cond.energy) + "," +
         std::to_string(S);
  }
  return k;
}

// Last line of the cache whose key matches; false when there is none.
bool cache_lookup(const char *path, const std::string &key, psr_tune_result *r) {
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[2048], k[1024];
  bool hit = false;
  while (fgets(line, sizeof line, f)) {
    psr_tune_result t{};
    if (sscanf(line, "%1023s engine=%d rpw=%d grid_per_cu=%d ms=%lf solves_per_s=%lf", k, &t.engine, &t.rpw,
               &t.grid_per_cu, &t.ms, &t.solves_per_s) == 6 &&
        key == k && t.engine >= 0 && t.engine <= 2 && (t.rpw == 0 || t.rpw == 1 || t.rpw == 2 || t.rpw == 4) &&
        t.grid_per_cu >= 0 && t.grid_per_cu <= 32) {
      *r = t;
      hit = true;
    }
  }
  fclose(f);
  return hit;
}

}  // namespace

extern "C" psr_status psr_autotune(const psr_group *groups, int32_t n_groups, psr_solve_opts *opts, int64_t sample,
                                   const char *cache_path, psr_tune_result *result, void *stream) {
  psr_status st = check_opts(opts);
  if (st != PSR_OK) return st;
  if (!groups || n_groups <= 0) return fail(PSR_EINVAL, "no groups");
  if (sample < 1) return fail(PSR_EINVAL, "sample must be >= 1");
  for (int gi = 0; gi < n_groups; gi++) {
    st = check_cond(groups[gi].mech, &groups[gi].cond);
    if (st != PSR_OK) return st;
    if (!groups[gi].x_inout) return fail(PSR_EINVAL, "null x_inout");
  }
  const std::string key = tune_key(groups, n_groups, opts, sample);
  if (key.size() >= 1000) return fail(PSR_EINVAL, "too many groups for the autotune cache key");
  psr_tune_result best{};
  if (cache_path && cache_lookup(cache_path, key, &best)) {
    best.candidates = 0;
    best.default_ms = 0;
    opts->engine = best.engine;
    opts->rpw = best.rpw;
    opts->grid_per_cu = best.grid_per_cu;
    if (result) *result = best;
    return PSR_OK;
  }

  // Candidate shapes.  The automatic shape comes first and wins ties within
  // 2 %, so noise does not move the choice off it.
  const bool mixed = opts->precision == PSR_MIXED;
  bool any_wave = false;
  for (int gi = 0; gi < n_groups; gi++)
    any_wave |= wave_plan(groups[gi].mech, groups[gi].cond.energy, mixed, 0).NP != 0;
  struct Shape { int engine, rpw, grid; };
  std::vector<Shape> shapes;
  std::vector<int> grids = {0};
  if (opts->scheduler == PSR_PERSISTENT) grids = {0, 1, 2};
  // rpw values whose plans on the wave groups repeat an earlier value's are
  // not tried.
  std::vector<int> rpws;
  std::vector<std::vector<int>> seen;
  for (int rpw : {0, 2, 1}) {
    std::vector<int> eff;
    for (int gi = 0; gi < n_groups; gi++)
      eff.push_back(wave_plan(groups[gi].mech, groups[gi].cond.energy, mixed, 0, rpw).rpw);
    if (std::find(seen.begin(), seen.end(), eff) != seen.end()) continue;
    seen.push_back(eff);
    rpws.push_back(rpw);
  }
  for (int gr : grids) {
    for (int rpw : rpws) shapes.push_back({0, rpw, gr});
    if (any_wave) shapes.push_back({1, 0, gr});
  }

  // Sample copies.
  std::vector<TuneSample> smp(n_groups);
  auto cleanup = [&]() { free_samples(smp); };
  const hipStream_t cs = (hipStream_t)stream;
#define TUNE_OK(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      cleanup();                                                                          \
      return fail(PSR_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(e_));   \
    }                                                                                     \
  } while (0)
  TUNE_OK(hipStreamSynchronize(cs));
  for (int gi = 0; gi < n_groups; gi++) {
    const psr_group &src = groups[gi];
    TuneSample &t = smp[gi];
    const int64_t B = src.cond.n_reactors;
    const int64_t S = std::min<int64_t>(sample, B);
    const int n = n_unknowns(src.mech->dev, src.cond.energy);
    const int N = src.mech->N;
    t.xbytes = (size_t)n * S * 8;
    TUNE_OK(hipMalloc(&t.x0, t.xbytes));
    TUNE_OK(hipMalloc(&t.x, t.xbytes));
    TUNE_OK(hipMalloc(&t.Yin, (size_t)N * S * 8));
    TUNE_OK(hipMalloc(&t.status, (size_t)S * 4));
    TUNE_OK(hipMemcpy2DAsync(t.x0, S * 8, src.x_inout, B * 8, S * 8, n, hipMemcpyDeviceToDevice, cs));
    TUNE_OK(hipMemcpy2DAsync(t.Yin, S * 8, src.cond.Y_in, B * 8, S * 8, N, hipMemcpyDeviceToDevice, cs));
    t.g.mech = src.mech;
    t.g.cond = src.cond;  // P, tau, T_in: the first S entries of the caller's arrays
    t.g.cond.n_reactors = S;
    t.g.cond.Y_in = t.Yin;
    t.g.x_inout = t.x;
    t.g.status = t.status;
    t.g.n_lin = nullptr;
  }
  TUNE_OK(hipStreamSynchronize(cs));
  std::vector<psr_group> sg(n_groups);
  for (int gi = 0; gi < n_groups; gi++) sg[gi] = smp[gi].g;

  void *ws = nullptr;
  size_t ws_bytes = 0;
  psr_status last = PSR_OK;
  std::string last_err;
  double best_score = -1;
  bool have = false;
  int timed = 0;
  double default_ms = 0;
  for (size_t ci = 0; ci < shapes.size(); ci++) {
    psr_solve_opts o = *opts;
    o.engine = shapes[ci].engine;
    o.rpw = shapes[ci].rpw;
    o.grid_per_cu = shapes[ci].grid;
    const size_t need = psr_workspace_bytes(sg.data(), n_groups, &o);
    if (need == 0) {
      if (ws) (void)hipFree(ws);
      cleanup();
      return fail(PSR_EINVAL, "psr_workspace_bytes failed for the sample");
    }
    if (need > ws_bytes) {
      if (ws) (void)hipFree(ws);
      ws = nullptr;
      ws_bytes = 0;
      hipError_t e = hipMalloc(&ws, need);
      if (e != hipSuccess) {
        cleanup();
        return fail(PSR_ENOMEM, std::string("autotune workspace: ") + hipGetErrorString(e));
      }
      ws_bytes = need;
    }
    double ms = 1e300;
    int64_t conv = 0;
    psr_status rs = PSR_OK;
    for (int rep = 0; rep < 3 && rs == PSR_OK; rep++) {
      for (int gi = 0; gi < n_groups && rs == PSR_OK; gi++)
        if (hipMemcpyAsync(smp[gi].x, smp[gi].x0, smp[gi].xbytes, hipMemcpyDeviceToDevice, cs) != hipSuccess)
          rs = fail(PSR_EDEVICE, "autotune: restoring the sample state failed");
      if (rs != PSR_OK) break;
      psr_solve_stats stt{};
      rs = psr_solve_batch(sg.data(), n_groups, &o, ws, ws_bytes, &stt, stream);
      if (rs == PSR_OK && rep > 0) {  // the first run is untimed
        ms = std::min(ms, stt.kernel_ms);
        conv = stt.converged;
      }
    }
    if (rs == PSR_EUNSUPPORTED || rs == PSR_EINVAL) {  // this shape does not apply here
      last = rs;
      last_err = g_err;
      continue;
    }
    if (rs != PSR_OK) {
      (void)hipFree(ws);
      cleanup();
      return rs;
    }
    timed++;
    if (ci == 0) default_ms = ms;
    const double score = (double)conv / (ms * 1e-3);
    if (!have || score > best_score * 1.02) {
      have = true;
      best_score = score;
      best.engine = o.engine;
      best.rpw = o.rpw;
      best.grid_per_cu = o.grid_per_cu;
      best.ms = ms;
      best.solves_per_s = score;
    }
  }
  if (ws) (void)hipFree(ws);
  cleanup();
#undef TUNE_OK
  if (!have) return fail(last == PSR_OK ? PSR_EINVAL : last, "autotune: no candidate shape ran: " + last_err);
  best.candidates = timed;
  best.default_ms = default_ms;
  opts->engine = best.engine;
  opts->rpw = best.rpw;
  opts->grid_per_cu = best.grid_per_cu;
  if (result) *result = best;
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (!f) return fail(PSR_EINVAL, std::string("autotune: cannot append to cache file ") + cache_path);
    fprintf(f, "%s engine=%d rpw=%d grid_per_cu=%d ms=%.6f solves_per_s=%.3f\n", key.c_str(), best.engine,
            best.rpw, best.grid_per_cu, best.ms, best.solves_per_s);
    fclose(f);
  }
  return PSR_OK;
}
