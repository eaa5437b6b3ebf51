// mg_grouped.h -- many independent boxes as grouped level launches.
//
// Boxes of the same grid size and model form a class and run the same cycle
// program, so each level operation of the refined solve (the FP64 outer
// step, the half-sweeps, residual/restriction, coarse source, prolongation,
// the single-workgroup program of the small levels) is one launch per class
// with the box in blockIdx.y: the level kernels keep the register budget and
// the full occupancy of the single-box path, and the launch count no longer
// grows with the number of boxes.  Per-box constants, level geometry and
// workspace pointers come from a table in device memory; a per-box control
// word switches a box off once it has converged or has run its planned
// cycles.  Same per-cell arithmetic as the single-box kernels.
#pragma once
#include "mg_batched.h"

namespace mgg {

struct GBox {
  int nlev, fused_from, pad, use_field_in;
  Lev L[kMaxLevB];
  float h2[kMaxLevB];
  Consts C;
  const float* delta;  // natural n^3
  double* field;       // natural n^3: initial guess (use_field_in) and solution
  float* force;        // natural [3][n^3] or null
  double* w;           // FP64 master, packed
  float* e[kMaxLevB];
  float* X[kMaxLevB];
  float* rho[kMaxLevB];
  float* dens[kMaxLevB];
  float* eR[kMaxLevB];
  FusedCorr F;         // levels fused_from .. nlev-1 (the single-workgroup program)
};

// per-box control of the current outer step: cycles to run (kb), whether
// the outer step is taken (on) and the pending correction is to be added
struct GCtl {
  int on, kb, add, pad;
};

__device__ __forceinline__ uint32_t gthread() {
  return (uint32_t)blockIdx.x * blockDim.x + threadIdx.x;
}

// natural -> packed density and master; block partials of (bg_coef delta)^2
template <int M>
__global__ __launch_bounds__(kBlock) void kg_pack(const GBox* __restrict__ tab, double* part,
                                                  int pstride) {
  __shared__ double sh[32];
  const GBox& B = tab[blockIdx.y];
  const Lev& L0 = B.L[0];
  const int64_t m = 2 * L0.half;
  const uint32_t g = gthread();
  double t2 = 0.0;
  if (g < (uint32_t)m) {
    int i, j, k;
    dec_nat(g, L0, i, j, k);
    const uint32_t pk = pk_of(L0, i, j, k);
    const float d = B.delta[g];
    B.dens[0][pk] = d;
    B.w[pk] = B.use_field_in ? (M == FR ? -B.field[g] : B.field[g]) : B.C.bg;
    const double t = B.C.bg_coef * double(d);
    t2 = t * t;
  }
  const double s = block_sum(t2, sh);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * pstride + blockIdx.x] = s;
}

// density pyramid for the models whose correction operator uses it
__global__ __launch_bounds__(kBlock) void kg_restrict_dens(const GBox* __restrict__ tab, int l) {
  const GBox& B = tab[blockIdx.y];
  const uint32_t g = gthread();
  if (g < (uint32_t)(2 * B.L[l + 1].half))
    op_restrict<float, float>(B.L[l], B.L[l + 1], B.dens[l], B.dens[l + 1], g);
}

// w += e (the pending FP32 correction) where the box takes this outer step
__global__ __launch_bounds__(kBlock) void kg_update(const GBox* __restrict__ tab,
                                                    const GCtl* __restrict__ ctl) {
  const GCtl c = ctl[blockIdx.y];
  if (!c.on || !c.add) return;
  const GBox& B = tab[blockIdx.y];
  const uint32_t g = gthread();
  if (g < (uint32_t)(2 * B.L[0].half)) B.w[g] += double(B.e[0][g]);
}

// FP64 residual d = F(w), rho = -d, X = w, e = 0; block partials of d^2
template <int M>
__global__ __launch_bounds__(kBlock) void kg_outer(const GBox* __restrict__ tab,
                                                   const GCtl* __restrict__ ctl, double* part,
                                                   int pstride) {
  __shared__ double sh[32];
  const GCtl c = ctl[blockIdx.y];
  if (!c.on) return;  // uniform over the block: no block_sum below is skipped halfway
  const GBox& B = tab[blockIdx.y];
  const Lev& L0 = B.L[0];
  const uint32_t g = gthread();
  double d = 0.0;
  if (g < (uint32_t)(2 * L0.half)) {
    d = cell_resid_direct<M, double, float>(L0, B.w, B.dens[0], (const double*)nullptr, 1.0, B.C,
                                            g);
    B.rho[0][g] = float(-d);
    B.X[0][g] = float(B.w[g]);
    B.e[0][g] = 0.0f;
  }
  const double s = block_sum(d * d, sh);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * pstride + blockIdx.x] = s;
}

// per-box sums of the block partials: one block per box
__global__ __launch_bounds__(256) void kg_sum_box(const double* __restrict__ part, int pstride,
                                                  int nparts, double* __restrict__ out) {
  __shared__ double sh[32];
  double s = 0.0;
  const double* p = part + (int64_t)blockIdx.x * pstride;
  for (int q = threadIdx.x; q < nparts; q += blockDim.x) s += p[q];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// vec: 4 packed cells per thread (the level's rows hold a multiple of 4)
template <int M>
__global__ __launch_bounds__(kBlock) void kg_smooth(const GBox* __restrict__ tab,
                                                    const GCtl* __restrict__ ctl, int it, int l,
                                                    int colour, int vec) {
  if (it >= ctl[blockIdx.y].kb) return;
  const GBox& B = tab[blockIdx.y];
  const Lev& L = B.L[l];
  const uint32_t g = gthread();
  if (vec) {
    if (g < (uint32_t)(L.half / 4))
      op_smooth_corr_v<M>(L, B.e[l], B.X[l], B.dens[l], B.rho[l], colour, B.h2[l], B.C, g);
  } else if (g < (uint32_t)L.half) {
    op_smooth_corr<M>(L, B.e[l], B.X[l], B.dens[l], B.rho[l], colour, B.h2[l], B.C, g);
  }
}

// the same half-sweep marching in z over kt planes (blocks of one box in x)
template <int M>
__global__ __launch_bounds__(kBlock) void kg_smooth_kv(const GBox* __restrict__ tab,
                                                       const GCtl* __restrict__ ctl, int it, int l,
                                                       int colour, int kt) {
  if (it >= ctl[blockIdx.y].kb) return;
  const GBox& B = tab[blockIdx.y];
  op_smooth_corr_kv<M, float, float>(B.L[l], B.e[l], B.X[l], B.dens[l], B.rho[l], colour,
                                     B.h2[l], B.C, 0, kt, Store{1.0f, 1.0f, 1.0f, 1.0f});
}

// residual + restriction of level l in the shifted form (store_coarse_corr):
// the coarse problem is posed around X_H = R X + R e (R X of level l kept in
// eR[l+1], formed again with rx), the coarse correction starts at zero and
// no coarse-source pass follows.
// vec: 4 coarse cells per thread (the coarse side is a multiple of 4)
template <int M>
__global__ __launch_bounds__(kBlock) void kg_down(const GBox* __restrict__ tab,
                                                  const GCtl* __restrict__ ctl, int it, int l,
                                                  int rx, int skip1, int vec) {
  if (it >= ctl[blockIdx.y].kb) return;
  const GBox& B = tab[blockIdx.y];
  const Lev& Lf = B.L[l];
  const Lev& Lc = B.L[l + 1];
  const uint32_t g = gthread();
  if (vec) {
    if (g < (uint32_t)(2 * Lc.half / 4))
      op_resid_restrict_corr_v<M>(Lf, Lc, B.e[l], B.X[l], B.dens[l], B.rho[l], B.h2[l],
                                  B.e[l + 1], (float*)nullptr, B.rho[l + 1], B.X[l + 1], B.C,
                                  skip1, g, Store{1, 1, 1, 1}, B.eR[l + 1], rx);
  } else if (g < (uint32_t)(2 * Lc.half)) {
    op_resid_restrict_corr<M>(Lf, Lc, B.e[l], B.X[l], B.dens[l], B.rho[l], B.h2[l], B.e[l + 1],
                              (float*)nullptr, B.rho[l + 1], B.X[l + 1], B.C, g, B.eR[l + 1], rx);
  }
}
// e_l += P e_H (the coarse correction of the shifted form); with COL0 = 1
// colour 0 is left to the next exact half-sweep (not for the Newton
// smoother of CQ)
template <int COL0>
__global__ __launch_bounds__(kBlock) void kg_up(const GBox* __restrict__ tab,
                                                const GCtl* __restrict__ ctl, int it, int l) {
  if (it >= ctl[blockIdx.y].kb) return;
  const GBox& B = tab[blockIdx.y];
  const uint32_t g = gthread();
  if (g < (uint32_t)(2 * B.L[l + 1].half / 4))
    op_prolong_v<float, COL0>(B.L[l], B.L[l + 1], B.e[l], B.e[l + 1], (const float*)nullptr, g);
}
__global__ __launch_bounds__(kBlock) void kg_up_block(const GBox* __restrict__ tab,
                                                      const GCtl* __restrict__ ctl, int it,
                                                      int l) {
  if (it >= ctl[blockIdx.y].kb) return;
  const GBox& B = tab[blockIdx.y];
  const uint32_t g = gthread();
  if (g < (uint32_t)(2 * B.L[l + 1].half))
    op_prolong_block<float>(B.L[l], B.L[l + 1], B.e[l], B.e[l + 1], g);
}

// the small levels of every box of the class: one workgroup per box
template <int M>
__global__ __launch_bounds__(kFusedThreads) void kg_fused(const GBox* __restrict__ tab,
                                                          const GCtl* __restrict__ ctl, int it,
                                                          FusedProg P) {
  __shared__ double sh[32];
  if (it >= ctl[blockIdx.x].kb) return;
  const GBox& B = tab[blockIdx.x];
  fused_corr_body<M>(B.F, P, B.C, sh);
}

// packed master -> natural field
template <int M>
__global__ __launch_bounds__(kBlock) void kg_unpack(const GBox* __restrict__ tab) {
  const GBox& B = tab[blockIdx.y];
  const Lev& L0 = B.L[0];
  const uint32_t g = gthread();
  if (g >= (uint32_t)(2 * L0.half)) return;
  int i, j, k;
  dec_nat(g, L0, i, j, k);
  const double v = B.w[pk_of(L0, i, j, k)];
  B.field[g] = M == FR ? -v : v;
}

// fifth force from the natural field, by central differences of Phi5 (the
// same rounded products as the single-box kernels)
template <int M>
__global__ __launch_bounds__(kBlock) void kg_force(const GBox* __restrict__ tab) {
  const GBox& B = tab[blockIdx.y];
  if (!B.force) return;
  const Lev& L0 = B.L[0];
  const int64_t m = 2 * L0.half;
  const uint32_t g = gthread();
  if (g >= (uint32_t)m) return;
  int i, j, k;
  dec_nat(g, L0, i, j, k);
  const int n = L0.n;
  const int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
  const int jp = j + 1 == n ? 0 : j + 1, jm = j == 0 ? n - 1 : j - 1;
  const int kp = k + 1 == n ? 0 : k + 1, km = k == 0 ? n - 1 : k - 1;
  const double* f = B.field;
  auto phi = [&](double v) {
    return M == FR ? -__dmul_rn(B.C.phi5, v)
                   : (M == SYM ? __dmul_rn(__dmul_rn(B.C.phi5, v), v) : __dmul_rn(B.C.phi5, v));
  };
  const int64_t row = (int64_t)k * n + j;
  B.force[g] = float(-0.5 * (phi(f[row * n + ip]) - phi(f[row * n + im])));
  B.force[m + g] = float(-0.5 * (phi(f[((int64_t)k * n + jp) * n + i]) -
                                 phi(f[((int64_t)k * n + jm) * n + i])));
  B.force[2 * m + g] = float(-0.5 * (phi(f[((int64_t)kp * n + j) * n + i]) -
                                     phi(f[((int64_t)km * n + j) * n + i])));
}

}  // namespace mgg
