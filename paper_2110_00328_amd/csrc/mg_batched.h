// mg_batched.h -- many independent boxes in one persistent launch.
//
// The paper runs independent realisations side by side (MPI over nodes,
// Sec. 3.1); here a single cooperative launch takes a list of boxes of
// different sizes and models.  The grid is exactly the set of workgroups that
// can be resident at once.  The host splits it into teams: a box gets a team
// whose size follows its cell count (so a 128^3 box gets several workgroups
// and a 64^3 box one), or, when there are more boxes than workgroups, teams of
// one workgroup each run a static longest-first list of boxes.  A team runs
// its box's whole FP32-refined solve -- FP64 outer residuals, FP32 correction
// cycles over all levels, the coarsest-level solve -- then the fifth force.
//
// Inside a team, fine-level operations are split over the team's workgroups
// and separated by team barriers; levels of n <= 16 are run by the team's
// first workgroup alone.  A team barrier is an arrival counter in device
// memory with a bounded wait: if any wait exceeds its spin limit the
// workgroup raises a launch-wide abort flag, every workgroup leaves at its
// next barrier or box, and the host reports an error.  So every wave always
// reaches the end of the kernel.
#pragma once
#include "mg_kernels.h"

namespace mgg {

// Pointers read from a descriptor in device memory are generic to the
// compiler, so accesses through them would be flat memory operations (which
// also count against the LDS/scalar counter and force full waits).  These
// pointers always address global memory; passing them through an integer
// into the global address space lets the compiler use global operations.
template <typename T>
__device__ __forceinline__ T* glb(T* p) {
  typedef __attribute__((address_space(1))) T gT;
  return (T*)(gT*)(uintptr_t)p;
}

constexpr int kMaxLevB = 8;
constexpr int kMaxOpsB = 160;
constexpr int kLeadN = 16;                 // levels of n <= 16 run on one workgroup
constexpr unsigned kSpinLimit = 1u << 25;  // ~2 s of s_sleep(2) polls

struct BoxDev {
  int model, nlev, vec, nops;
  int nu1, nu2, fixed_inner, max_outer, coarse_sweeps, use_field_in;
  int trial;  // tuning run: no outputs written
  int pad0;
  double tol;
  Lev L[kMaxLevB];
  float h2[kMaxLevB];
  Consts C;
  const float* delta;  // natural, n^3
  double* field;       // natural, n^3: initial guess (if use_field_in) and solution
  float* force;        // natural [3][n^3] or null
  double* w;           // FP64 master, packed
  float* e[kMaxLevB];
  float* X[kMaxLevB];
  float* rho[kMaxLevB];
  float* dens[kMaxLevB];
  float* eR[kMaxLevB];
  Op op[kMaxOpsB];  // one cycle over levels 0 .. nlev-1
};

struct BoxOut {
  int outer, vcycles, status, pad;
  double rel;
};

// one team: `size` workgroups run boxes order[first .. first + count)
struct TeamDev {
  int size, first, count, part_off;
};

// A workgroup's view of its team.  `gtid`/`gnt` spread a loop over the team
// (or over this workgroup alone for the one-workgroup view).  The counters of
// barriers and reductions live in LDS (uniform per workgroup), so the view
// itself is passed by value.
struct Team {
  unsigned* ctr;    // arrival counter (monotonic over the launch)
  double* part;     // 2 x size reduction slots
  int* abort;
  int* s_ok;        // LDS: outcome of the last barrier
  unsigned* s_gen;  // LDS: barriers passed (thread 0 only)
  unsigned* s_red;  // LDS: reductions done (slot parity)
  int size, rank;
  uint32_t gtid, gnt;
};

__device__ __forceinline__ Team solo_view(Team T) {
  T.size = 1;
  T.rank = 0;
  T.gtid = threadIdx.x;
  T.gnt = blockDim.x;
  return T;
}

// Team barrier: every thread releases its writes at device scope, one thread
// arrives and waits (bounded), then acquires.  Returns false on abort.
__device__ bool team_sync(const Team& T) {
  if (T.size == 1) {
    __syncthreads();
    return true;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen = *T.s_gen + 1u;
    *T.s_gen = gen;
    atomicAdd(glb(T.ctr), 1u);
    const unsigned target = gen * (unsigned)T.size;
    unsigned spins = 0;
    int ok = 1;
    while (__hip_atomic_load(glb(T.ctr), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(glb(T.abort), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > kSpinLimit) {
        ok = 0;
        atomicExch(glb(T.abort), 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    *T.s_ok = ok;
  }
  __syncthreads();
  return *T.s_ok != 0;
}

// Sum of v over the team, same value (same summation order) in every
// workgroup.  Returns false on abort.
__device__ bool team_sum(const Team& T, double v, double* sh, double* out) {
  double t = block_sum(v, sh);  // valid in thread 0
  if (T.size == 1) {
    __syncthreads();
    if (threadIdx.x == 0) sh[16] = t;
    __syncthreads();
    *out = sh[16];
    __syncthreads();
    return true;
  }
  const unsigned r = *T.s_red;  // read by every thread before the barrier below
  double* slot = glb(T.part) + (r & 1u) * (unsigned)T.size;
  if (threadIdx.x == 0)
    __hip_atomic_store(slot + T.rank, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!team_sync(T)) return false;
  double s = 0.0;
  for (int q = 0; q < T.size; ++q)
    s += __hip_atomic_load(slot + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) *T.s_red = r + 1u;  // next reader passes a barrier first
  *out = s;
  return true;
}

__device__ __noinline__ int b_plan(int fixed, double rel, double rel_prev, int k_prev,
                                      double tol) {
  if (fixed > 0) return fixed;
  if (rel_prev <= 0.0 || k_prev <= 0 || !(rel < rel_prev)) return 2;
  double rho = pow(rel / rel_prev, 1.0 / k_prev);
  rho = rho < 0.01 ? 0.01 : (rho > 0.9 ? 0.9 : rho);
  int k = (int)ceil(1.05 * log(tol / rel) / log(rho));
  return k < 1 ? 1 : (k > 8 ? 8 : k);  // as the single-box planner
}

template <int M>
__device__ __noinline__ bool b_smooth(const BoxDev& B, Team T, int l, int sweeps) {
  const Lev L = B.L[l];
  const bool vec = B.vec && (L.nh % 4) == 0;
  float* e = glb(B.e[l]);
  const float* X = glb(B.X[l]);
  const float* dn = glb(B.dens[l]);
  const float* rho = glb(B.rho[l]);
  for (int it = 0; it < sweeps; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      if (vec) {
        for (uint32_t g4 = T.gtid; g4 < (uint32_t)(L.half / 4); g4 += T.gnt)
          op_smooth_corr_v<M>(L, e, X, dn, rho, colour, B.h2[l], B.C, g4);
      } else {
        for (int64_t g = T.gtid; g < L.half; g += T.gnt)
          op_smooth_corr<M>(L, e, X, dn, rho, colour, B.h2[l], B.C, g);
      }
      if (!team_sync(T)) return false;
    }
  return true;
}

template <int M>
__device__ __noinline__ bool b_down(const BoxDev& B, Team T, int l, bool rx) {
  const Lev Lf = B.L[l], Lc = B.L[l + 1];
  const float* e = glb(B.e[l]);
  const float* X = glb(B.X[l]);
  const float* dn = glb(B.dens[l]);
  const float* rho = glb(B.rho[l]);
  float* eH = glb(B.e[l + 1]);
  float* eRH = glb(B.eR[l + 1]);
  float* XH1 = glb(B.X[l + 1]);
  const float* dnH = glb(B.dens[l + 1]);
  float* rhoH = glb(B.rho[l + 1]);
  float* XH = rx ? XH1 : nullptr;
  if (B.vec && (Lc.n % 4) == 0) {
    for (uint32_t g4 = T.gtid; g4 < (uint32_t)(2 * Lc.half / 4); g4 += T.gnt)
      op_resid_restrict_corr_v<M>(Lf, Lc, e, X, dn, rho, B.h2[l], eH, eRH, rhoH, XH, B.C,
                                  (M != CQ && B.nu1 > 0) ? 1 : 0, g4);
  } else {
    for (int64_t g = T.gtid; g < 2 * Lc.half; g += T.gnt)
      op_resid_restrict_corr<M>(Lf, Lc, e, X, dn, rho, B.h2[l], eH, eRH, rhoH, XH, B.C, g);
  }
  if (!team_sync(T)) return false;
  for (int64_t g = T.gtid; g < 2 * Lc.half; g += T.gnt)
    op_coarse_src_corr<M>(Lc, eRH, XH1, dnH, rhoH, B.h2[l + 1], B.C, g);
  return team_sync(T);
}

template <int M>
__device__ __noinline__ bool b_up(const BoxDev& B, Team T, int l) {
  const Lev Lf = B.L[l], Lc = B.L[l + 1];
  float* e = glb(B.e[l]);
  float* eH = glb(B.e[l + 1]);
  float* eRH = glb(B.eR[l + 1]);
  if (B.vec && (Lc.n % 4) == 0) {
    // e += P(e_H - R e) in one pass; colour 0 too only for CQ's Newton smoother
    for (uint32_t g4 = T.gtid; g4 < (uint32_t)(2 * Lc.half / 4); g4 += T.gnt)
      op_prolong_v<float, M == CQ ? 0 : 1>(Lf, Lc, e, eH, eRH, g4);
  } else {
    for (int64_t g = T.gtid; g < 2 * Lc.half; g += T.gnt)
      eRH[g] = eH[g] - eRH[g];
    if (!team_sync(T)) return false;
    for (int64_t g = T.gtid; g < 2 * Lc.half; g += T.gnt)
      op_prolong_block<float>(Lf, Lc, e, eRH, g);
  }
  return team_sync(T);
}

// Coarsest level, one workgroup: relax until the RMS residual has dropped by
// 1e-8 (checked every 4 sweeps); coupled quintessence adds a Newton step on
// the uniform mode at each check.
template <int M>
__device__ __noinline__ void b_coarsest(const BoxDev& B, int l, double* sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const Lev L = B.L[l];
  float* e = glb(B.e[l]);
  const float* X = glb(B.X[l]);
  const float* dn = glb(B.dens[l]);
  const float* rho = glb(B.rho[l]);
  double r0 = -1.0;
  for (int it = 0; it < B.coarse_sweeps; ++it) {
    for (int colour = 0; colour < 2; ++colour) {
      for (int64_t g = tid; g < L.half; g += nt)
        op_smooth_corr<M>(L, e, X, dn, rho, colour, B.h2[l], B.C, g);
      __syncthreads();
    }
    if ((it & 3) != 3 && it + 1 < B.coarse_sweeps) continue;
    double s2 = 0.0, sd = 0.0, sj = 0.0;
    for (int64_t g = tid; g < 2 * L.half; g += nt) {
      double d = double(cell_resid_corr<M>(L, e, X, dn, rho, B.h2[l], B.C, g));
      s2 += d * d;
      if (M == CQ) {
        sd += d;
        sj += double(corr_diag<M>(B.C, B.h2[l], e[g], X[g], dn[g])) +
              6.0 / double(B.h2[l]);
      }
    }
    double tot = block_sum_all(s2, sh);
    if (M == CQ) {
      double D = block_sum_all(sd, sh);
      double Jd = block_sum_all(sj, sh);
      if (Jd != 0.0) {
        float mu = float(-D / Jd);
        for (int64_t g = tid; g < 2 * L.half; g += nt) e[g] += mu;
      }
      __syncthreads();
    }
    if (r0 < 0.0) r0 = tot;
    if (tot <= 1e-16 * r0 || tot == 0.0) break;
  }
}

__device__ __forceinline__ bool op_is_lead(const BoxDev& B, const Op& op) {
  return op.kind == OP_COARSEST || B.L[op.lev].n <= kLeadN;
}

template <int M>
__device__ bool b_run_op(const BoxDev& B, const Team& V, const Op& op, bool rx, double* sh) {
  if (op.kind == OP_SMOOTH) return b_smooth<M>(B, V, op.lev, op.count);
  if (op.kind == OP_DOWN) return b_down<M>(B, V, op.lev, rx);
  if (op.kind == OP_UP) return b_up<M>(B, V, op.lev);
  b_coarsest<M>(B, op.lev, sh);
  return true;
}

// One cycle.  Operations on small levels run on the team's first workgroup
// (the others skip them); a team barrier separates them from team-wide ones.
template <int M>
__device__ __noinline__ bool b_cycle(const BoxDev& B, Team T, bool rx, double* sh) {
  bool prev_lead = false;
  for (int o = 0; o < B.nops; ++o) {
    const Op op = B.op[o];
    if (T.size > 1 && op_is_lead(B, op)) {
      if (T.rank == 0) {
        Team S = solo_view(T);
        b_run_op<M>(B, S, op, rx, sh);
      }
      prev_lead = true;
    } else {
      if (prev_lead && !team_sync(T)) return false;
      if (!b_run_op<M>(B, T, op, rx, sh)) return false;
      prev_lead = false;
    }
  }
  if (prev_lead) return team_sync(T);
  return true;
}

// natural -> packed inputs; returns the squared background residual summed
// over the team in *bsq_out
template <int M>
__device__ __noinline__ bool b_pack(const BoxDev& B, Team T, double* sh, double* bsq_out) {
  const Lev L0 = B.L[0];
  const int64_t m = 2 * L0.half;
  const double sgn = (M == FR) ? -1.0 : 1.0;
  double bsq = 0.0;
  for (int64_t g = T.gtid; g < m; g += T.gnt) {
    int i, j, k;
    dec_nat(g, L0, i, j, k);
    uint32_t pk = pk_of(L0, i, j, k);
    float d = glb(B.delta)[g];
    glb(B.dens[0])[pk] = d;
    glb(B.w)[pk] = (B.use_field_in && !B.trial) ? sgn * glb(B.field)[g] : B.C.bg;
    double t = B.C.bg_coef * double(d);
    bsq += t * t;
  }
  if (!team_sum(T, bsq, sh, bsq_out)) return false;
  if (M != FR) {
    for (int l = 0; l + 1 < B.nlev; ++l) {
      for (int64_t g = T.gtid; g < 2 * B.L[l + 1].half; g += T.gnt)
        op_restrict<float, float>(B.L[l], B.L[l + 1], glb(B.dens[l]), glb(B.dens[l + 1]), g);
      if (!team_sync(T)) return false;
    }
  }
  return true;
}

// w += e (when add), then the FP64 residual of w and the FP32 correction
// problem for the next step; squared residual summed over the team
template <int M>
__device__ __noinline__ bool b_outer(const BoxDev& B, Team T, bool add, double* sh,
                                     double* sq_out) {
  const Lev L0 = B.L[0];
  const int64_t m = 2 * L0.half;
  if (add) {
    for (int64_t g = T.gtid; g < m; g += T.gnt) glb(B.w)[g] += double(glb(B.e[0])[g]);
    if (!team_sync(T)) return false;
  }
  double acc = 0.0;
  for (int64_t g = T.gtid; g < m; g += T.gnt) {
    double d = cell_resid_direct<M, double, float>(L0, glb(B.w), glb(B.dens[0]),
                                                   (const double*)nullptr, 1.0, B.C, g);
    acc += d * d;
    glb(B.rho[0])[g] = float(-d);
    glb(B.X[0])[g] = float(glb(B.w)[g]);
    glb(B.e[0])[g] = 0.0f;
  }
  return team_sum(T, acc, sh, sq_out);
}

// packed -> natural solution, then the fifth force from it
template <int M>
__device__ __noinline__ bool b_finish(const BoxDev& B, Team T) {
  const Lev L0 = B.L[0];
  const int64_t m = 2 * L0.half;
  const double sgn = (M == FR) ? -1.0 : 1.0;
  for (int64_t g = T.gtid; g < m; g += T.gnt) {
    int i, j, k;
    dec_nat(g, L0, i, j, k);
    glb(B.field)[g] = sgn * glb(B.w)[pk_of(L0, i, j, k)];
  }
  if (!team_sync(T)) return false;
  if (B.force) {
    const int n = L0.n;
    const double* f = glb(B.field);
    for (int64_t g = T.gtid; g < m; g += T.gnt) {
      int i, j, k;
      dec_nat(g, L0, i, j, k);
      int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
      int jp = j + 1 == n ? 0 : j + 1, jm = j == 0 ? n - 1 : j - 1;
      int kp = k + 1 == n ? 0 : k + 1, km = k == 0 ? n - 1 : k - 1;
      auto phi = [&](double v) {  // rounded products: equal values give a zero difference
        return M == FR ? -__dmul_rn(B.C.phi5, v)
                       : (M == SYM ? __dmul_rn(__dmul_rn(B.C.phi5, v), v) : __dmul_rn(B.C.phi5, v));
      };
      int64_t row = (int64_t)k * n + j;
      glb(B.force)[g] = float(-0.5 * (phi(f[row * n + ip]) - phi(f[row * n + im])));
      glb(B.force)[m + g] = float(-0.5 * (phi(f[((int64_t)k * n + jp) * n + i]) -
                                     phi(f[((int64_t)k * n + jm) * n + i])));
      glb(B.force)[2 * m + g] = float(-0.5 * (phi(f[((int64_t)kp * n + j) * n + i]) -
                                         phi(f[((int64_t)km * n + j) * n + i])));
    }
  }
  return true;
}

// One box on one team: pack, outer FP64 steps with FP32 correction cycles,
// then the outputs.  false = aborted.
template <int M>
__device__ __noinline__ bool box_solve(const BoxDev& B, Team T, BoxOut* out, double* sh) {
  const double m = 2.0 * double(B.L[0].half);
  double tot = 0.0;
  if (!b_pack<M>(B, T, sh, &tot)) return false;
  double eps_bg = sqrt(tot / m);  // delta = 0: the residual of a unit contrast
  if (!(eps_bg > 0.0)) eps_bg = B.C.bg_coef > 0.0 ? B.C.bg_coef : 1.0;
  int outer = 0, vc = 0, k_prev = 0, status = 0;
  double rel = 0.0, rel_prev = -1.0;
  for (;;) {
    if (!b_outer<M>(B, T, outer > 0, sh, &tot)) return false;
    rel = sqrt(tot / m) / eps_bg;
    if (!isfinite(rel)) {
      status = -3;
      break;
    }
    if (rel <= B.tol) break;
    if (outer >= B.max_outer) {
      status = -2;
      break;
    }
    int kc = b_plan(B.fixed_inner, rel, rel_prev, k_prev, B.tol);
    for (int it = 0; it < kc; ++it)
      if (!b_cycle<M>(B, T, it == 0, sh)) return false;
    vc += kc;
    rel_prev = rel;
    k_prev = kc;
    ++outer;
  }
  if (!B.trial && !b_finish<M>(B, T)) return false;
  if (T.rank == 0 && threadIdx.x == 0) {
    out->outer = outer;
    out->vcycles = vc;
    out->status = status;
    out->rel = rel;
  }
  // the team's workspace may be reused by its next box
  return team_sync(T);
}

// The persistent cooperative launch: wg[b] = (team, rank) of workgroup b
// (team < 0: idle).  Each team runs its list of boxes.
template <int BS>
__global__ __launch_bounds__(BS) void k_batched(const BoxDev* __restrict__ boxes,
                                                const int* __restrict__ order,
                                                const TeamDev* __restrict__ teams,
                                                const int2* __restrict__ wg,
                                                BoxOut* __restrict__ outs, unsigned* ctr,
                                                double* parts, int* abort) {
  __shared__ double sh[32];
  __shared__ int s_ok;
  __shared__ unsigned s_gen, s_red;
  const int2 me = wg[blockIdx.x];
  if (me.x < 0) return;
  const TeamDev TD = teams[me.x];
  if (threadIdx.x == 0) {
    s_gen = 0u;
    s_red = 0u;
  }
  __syncthreads();
  Team T;
  T.ctr = ctr + me.x;
  T.part = parts + TD.part_off;
  T.abort = abort;
  T.s_ok = &s_ok;
  T.s_gen = &s_gen;
  T.s_red = &s_red;
  T.size = TD.size;
  T.rank = me.y;
  T.gtid = (uint32_t)me.y * blockDim.x + threadIdx.x;
  T.gnt = (uint32_t)TD.size * blockDim.x;
  for (int q = 0; q < TD.count; ++q) {
    // leave once any workgroup has aborted (same decision for the whole workgroup)
    if (threadIdx.x == 0)
      s_ok = __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    __syncthreads();
    const bool go = s_ok != 0;
    __syncthreads();
    if (!go) break;
    const int b = order[TD.first + q];
    const BoxDev& B = boxes[b];
    bool ok;
    if (B.model == FR) ok = box_solve<FR>(B, T, outs + b, sh);
    else if (B.model == SYM) ok = box_solve<SYM>(B, T, outs + b, sh);
    else ok = box_solve<CQ>(B, T, outs + b, sh);
    if (!ok) break;
  }
}

}  // namespace mgg
