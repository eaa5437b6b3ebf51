// mg_batched.h -- many independent boxes in one persistent launch.
//
// The paper runs independent realisations side by side (MPI over nodes,
// Sec. 3.1); here a single launch takes a list of boxes of different sizes
// and models.  The grid never exceeds the number of workgroups that can be
// resident at once, and each workgroup repeatedly takes the next box from an
// atomic ticket and runs that box's whole refined solve: FP64 outer
// residuals, FP32 correction V-cycles over all of its levels (block-strided
// level operations separated by __syncthreads), the coarsest-level solve,
// and optionally the fifth force.  No workgroup ever waits for another, so
// the launch cannot deadlock and every wave leaves once the tickets run out.
#pragma once
#include "mg_kernels.h"

namespace mgg {

constexpr int kMaxLevB = 8;
constexpr int kMaxOpsB = 160;

struct BoxDev {
  int model, nlev, vec, nops;
  int nu1, nu2, fixed_inner, max_outer, coarse_sweeps, use_field_in;
  int trial;  // tuning run: no outputs written
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

__device__ __forceinline__ int b_plan(int fixed, double rel, double rel_prev, int k_prev,
                                      double tol) {
  if (fixed > 0) return fixed;
  if (rel_prev <= 0.0 || k_prev <= 0 || !(rel < rel_prev)) return 2;
  double rho = pow(rel / rel_prev, 1.0 / k_prev);
  rho = rho < 0.01 ? 0.01 : (rho > 0.9 ? 0.9 : rho);
  int k = (int)ceil(1.05 * log(tol / rel) / log(rho));
  return k < 1 ? 1 : (k > 4 ? 4 : k);
}

template <int M>
__device__ void b_smooth(const BoxDev& B, int l, int sweeps) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const Lev L = B.L[l];
  const bool vec = B.vec && (L.nh % 4) == 0;
  for (int it = 0; it < sweeps; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      if (vec) {
        for (uint32_t g4 = tid; g4 < (uint32_t)(L.half / 4); g4 += nt)
          op_smooth_corr_v<M>(L, B.e[l], B.X[l], B.dens[l], B.rho[l], colour, B.h2[l], B.C, g4);
      } else {
        for (int64_t g = tid; g < L.half; g += nt)
          op_smooth_corr<M>(L, B.e[l], B.X[l], B.dens[l], B.rho[l], colour, B.h2[l], B.C, g);
      }
      __syncthreads();
    }
}

template <int M>
__device__ void b_down(const BoxDev& B, int l, bool rx) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const Lev Lf = B.L[l], Lc = B.L[l + 1];
  float* XH = rx ? B.X[l + 1] : nullptr;
  if (B.vec && (Lc.n % 4) == 0) {
    for (uint32_t g4 = tid; g4 < (uint32_t)(2 * Lc.half / 4); g4 += nt)
      op_resid_restrict_corr_v<M>(Lf, Lc, B.e[l], B.X[l], B.dens[l], B.rho[l], B.h2[l],
                                  B.e[l + 1], B.eR[l + 1], B.rho[l + 1], XH, B.C, g4);
  } else {
    for (int64_t g = tid; g < 2 * Lc.half; g += nt)
      op_resid_restrict_corr<M>(Lf, Lc, B.e[l], B.X[l], B.dens[l], B.rho[l], B.h2[l], B.e[l + 1],
                                B.eR[l + 1], B.rho[l + 1], XH, B.C, g);
  }
  __syncthreads();
  for (int64_t g = tid; g < 2 * Lc.half; g += nt)
    op_coarse_src_corr<M>(Lc, B.eR[l + 1], B.X[l + 1], B.dens[l + 1], B.rho[l + 1], B.h2[l + 1],
                          B.C, g);
  __syncthreads();
}

__device__ __forceinline__ void b_up(const BoxDev& B, int l) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const Lev Lf = B.L[l], Lc = B.L[l + 1];
  for (int64_t g = tid; g < 2 * Lc.half; g += nt) B.eR[l + 1][g] = B.e[l + 1][g] - B.eR[l + 1][g];
  __syncthreads();
  if (B.vec && (Lc.n % 4) == 0) {
    for (uint32_t g4 = tid; g4 < (uint32_t)(2 * Lc.half / 4); g4 += nt)
      op_prolong_v<float>(Lf, Lc, B.e[l], B.eR[l + 1], g4);
  } else {
    for (int64_t g = tid; g < 2 * Lc.half; g += nt)
      op_prolong_block<float>(Lf, Lc, B.e[l], B.eR[l + 1], g);
  }
  __syncthreads();
}

// relax until the RMS residual has dropped by 1e-8 (checked every 4 sweeps);
// coupled quintessence adds a Newton step on the uniform mode at each check
template <int M>
__device__ void b_coarsest(const BoxDev& B, int l, double* sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const Lev L = B.L[l];
  double r0 = -1.0;
  for (int it = 0; it < B.coarse_sweeps; ++it) {
    for (int colour = 0; colour < 2; ++colour) {
      for (int64_t g = tid; g < L.half; g += nt)
        op_smooth_corr<M>(L, B.e[l], B.X[l], B.dens[l], B.rho[l], colour, B.h2[l], B.C, g);
      __syncthreads();
    }
    if ((it & 3) != 3 && it + 1 < B.coarse_sweeps) continue;
    double s2 = 0.0, sd = 0.0, sj = 0.0;
    for (int64_t g = tid; g < 2 * L.half; g += nt) {
      double d = double(cell_resid_corr<M>(L, B.e[l], B.X[l], B.dens[l], B.rho[l], B.h2[l], B.C, g));
      s2 += d * d;
      if (M == CQ) {
        sd += d;
        sj += double(corr_diag<M>(B.C, B.h2[l], B.e[l][g], B.X[l][g], B.dens[l][g])) +
              6.0 / double(B.h2[l]);
      }
    }
    double tot = block_sum_all(s2, sh);
    if (M == CQ) {
      double D = block_sum_all(sd, sh);
      double Jd = block_sum_all(sj, sh);
      if (Jd != 0.0) {
        float mu = float(-D / Jd);
        for (int64_t g = tid; g < 2 * L.half; g += nt) B.e[l][g] += mu;
      }
      __syncthreads();
    }
    if (r0 < 0.0) r0 = tot;
    if (tot <= 1e-16 * r0 || tot == 0.0) break;
  }
}

template <int M>
__device__ void b_cycle(const BoxDev& B, bool rx, double* sh) {
  for (int o = 0; o < B.nops; ++o) {
    const Op op = B.op[o];
    if (op.kind == OP_SMOOTH) b_smooth<M>(B, op.lev, op.count);
    else if (op.kind == OP_DOWN) b_down<M>(B, op.lev, rx);
    else if (op.kind == OP_UP) b_up(B, op.lev);
    else b_coarsest<M>(B, op.lev, sh);
  }
}

template <int M>
__device__ void box_solve(const BoxDev& B, BoxOut* out, double* sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const Lev L0 = B.L[0];
  const int64_t m = 2 * L0.half;
  const double sgn = (M == FR) ? -1.0 : 1.0;
  // natural -> packed inputs; background residual
  double bsq = 0.0;
  for (int64_t g = tid; g < m; g += nt) {
    int i, j, k;
    dec_nat(g, L0, i, j, k);
    uint32_t pk = pk_of(L0, i, j, k);
    float d = B.delta[g];
    B.dens[0][pk] = d;
    B.w[pk] = (B.use_field_in && !B.trial) ? sgn * B.field[g] : B.C.bg;
    double t = B.C.bg_coef * double(d);
    bsq += t * t;
  }
  double eps_bg = sqrt(block_sum_all(bsq, sh) / double(m));
  if (!(eps_bg > 0.0)) eps_bg = 1.0;
  if (M != FR) {
    for (int l = 0; l + 1 < B.nlev; ++l) {
      for (int64_t g = tid; g < 2 * B.L[l + 1].half; g += nt)
        op_restrict<float, float>(B.L[l], B.L[l + 1], B.dens[l], B.dens[l + 1], g);
      __syncthreads();
    }
  }
  int outer = 0, vc = 0, k_prev = 0, status = 0;
  double rel = 0.0, rel_prev = -1.0;
  for (;;) {
    // FP64 residual of the master; correction problem for the next step
    double acc = 0.0;
    for (int64_t g = tid; g < m; g += nt) {
      double d = cell_resid_direct<M, double, float>(L0, B.w, B.dens[0], (const double*)nullptr,
                                                     1.0, B.C, g);
      acc += d * d;
      B.rho[0][g] = float(-d);
      B.X[0][g] = float(B.w[g]);
      B.e[0][g] = 0.0f;
    }
    rel = sqrt(block_sum_all(acc, sh) / double(m)) / eps_bg;
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
    for (int it = 0; it < kc; ++it) b_cycle<M>(B, it == 0, sh);
    for (int64_t g = tid; g < m; g += nt) B.w[g] += double(B.e[0][g]);
    __syncthreads();
    vc += kc;
    rel_prev = rel;
    k_prev = kc;
    ++outer;
  }
  if (B.trial) {
    if (tid == 0) {
      out->outer = outer;
      out->vcycles = vc;
      out->status = status;
      out->rel = rel;
    }
    __syncthreads();
    return;
  }
  // packed -> natural solution, then the force from it
  for (int64_t g = tid; g < m; g += nt) {
    int i, j, k;
    dec_nat(g, L0, i, j, k);
    B.field[g] = sgn * B.w[pk_of(L0, i, j, k)];
  }
  __syncthreads();
  if (B.force) {
    const int n = L0.n;
    for (int64_t g = tid; g < m; g += nt) {
      int i, j, k;
      dec_nat(g, L0, i, j, k);
      int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
      int jp = j + 1 == n ? 0 : j + 1, jm = j == 0 ? n - 1 : j - 1;
      int kp = k + 1 == n ? 0 : k + 1, km = k == 0 ? n - 1 : k - 1;
      const double* f = B.field;
      auto phi = [&](double v) {
        return M == FR ? -B.C.phi5 * v : (M == SYM ? B.C.phi5 * v * v : B.C.phi5 * v);
      };
      int64_t row = (int64_t)k * n + j;
      B.force[g] = float(-0.5 * (phi(f[row * n + ip]) - phi(f[row * n + im])));
      B.force[m + g] = float(-0.5 * (phi(f[((int64_t)k * n + jp) * n + i]) -
                                     phi(f[((int64_t)k * n + jm) * n + i])));
      B.force[2 * m + g] = float(-0.5 * (phi(f[((int64_t)kp * n + j) * n + i]) -
                                         phi(f[((int64_t)km * n + j) * n + i])));
    }
  }
  if (tid == 0) {
    out->outer = outer;
    out->vcycles = vc;
    out->status = status;
    out->rel = rel;
  }
  __syncthreads();
}

// The persistent launch: grid <= resident workgroups, boxes taken by ticket.
template <int BS>
__global__ __launch_bounds__(BS) void k_batched(const BoxDev* __restrict__ boxes, int nbox,
                                                BoxOut* __restrict__ outs, unsigned* ticket) {
  __shared__ double sh[32];
  __shared__ int bid;
  for (;;) {
    if (threadIdx.x == 0) bid = (int)atomicAdd(ticket, 1u);
    __syncthreads();
    const int b = bid;
    __syncthreads();
    if (b >= nbox) break;
    const BoxDev& B = boxes[b];
    if (B.model == FR) box_solve<FR>(B, outs + b, sh);
    else if (B.model == SYM) box_solve<SYM>(B, outs + b, sh);
    else box_solve<CQ>(B, outs + b, sh);
  }
}

}  // namespace mgg
