// mggpu.hip -- host driver and C ABI of the MI355X multigrid hot path.
//
// One context owns the level pyramid of one grid size on one HIP stream.
// Kernels are in mg_kernels.h / mg_device.h; this file holds the cycle
// control (V/F/W recursion over the large levels, a precomputed program for
// the small levels run by one workgroup), the FP64-refined outer loop, the
// adjoint's linear multigrid, and the CIC / force entry points.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <algorithm>
#include <cstdlib>
#include <type_traits>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include <dlfcn.h>
#include <rocfft/rocfft.h>  // declarations only: the library is opened at first use

#include "mg_batched.h"
#include "mg_grouped.h"
#include "mg_kernels.h"
#include "mggpu.h"

using namespace mgg;

namespace {

constexpr int kMaxLev = 24;
constexpr int kFuseN = 16;  // levels with n <= 16 run inside the fused kernel
constexpr double kCOverH0 = 2997.92458;  // Mpc/h

struct Work64 {  // FP64 direct mode
  double* v[kMaxLev] = {};
  double* dens[kMaxLev] = {};  // l >= 1
  double* S[kMaxLev] = {};     // l >= 1
  double* Rv[kMaxLev] = {};    // l >= 1
  float* dens0 = nullptr;      // finest level, packed float
};
struct Work32 {  // FP32 correction mode
  double* w = nullptr;         // FP64 master, packed (current)
  double* wbuf[2] = {};        // ping-pong pair for the fused update
  float* ebuf[2] = {};         // ping-pong pair for the level-0 correction
  float* e[kMaxLev] = {};
  float* X[kMaxLev] = {};
  float* rho[kMaxLev] = {};
  float* dens[kMaxLev] = {};
  // levels run one kernel at a time: R X of the next finer level's
  // linearisation point (the coarse problem's fixed part); levels inside the
  // single-workgroup kernel: R e of the finer level
  float* eR[kMaxLev] = {};
  h16* X16 = nullptr;          // level-0 X in 16 bits (when the context stores 16-bit data)
  h16* R16 = nullptr;          // level-0 rho in 16 bits
};
template <typename T>
struct WorkLin {  // adjoint linear multigrid in precision T
  T* ebuf[2] = {};  // ping-pong pair for the level-0 correction
  T* e[kMaxLev] = {};
  T* r[kMaxLev] = {};
  T* dg[kMaxLev] = {};
  h16* dg16 = nullptr;  // level-0 dg and r in 16 bits (FP32 solve only)
  h16* r16 = nullptr;
};
struct WorkAdj {
  double* v = nullptr;    // forward field (solved variable), packed
  double* dg = nullptr;   // FP64 diagonal, packed
  double* b = nullptr;    // right-hand side s * dL/dv, packed
  double* lam = nullptr;  // FP64 solution, packed (current)
  double* lambuf[2] = {}; // ping-pong pair for the fused update
  WorkLin<float> w32;
  WorkLin<double> w64;
  bool have32 = false, have64 = false;
};

}  // namespace

struct mg_ctx {
  int n = 0;
  hipStream_t stream = nullptr;
  // the z-marching smoother and residual/restriction kernels are used from
  // this many workgroups up (below it a grid is too sparse to hide the
  // march: at 512^3 the 256^3 level's smoother, 2048 workgroups, is faster
  // per row, 32.9 against 33.2 ms per step); MGGPU_MARCH_MIN_BLOCKS
  // overrides it at context creation
  unsigned march_min_blocks = 4096;
  // planes per thread of the z-marching FP32 smoother on large levels (0:
  // the per-row kernel); 4 was fastest with 16-bit X and rho at 512^3
  // (164 us per half-sweep against 175 per row; 2, 8, 16: 171, 169, 171);
  // MGGPU_SMOOTH_MARCH_KT overrides it at context creation
  int smooth_march_kt = 4;
  // coarse planes per workgroup of the prolongation fused into the first
  // post-smoothing half-sweep (0: separate prolongation and half-sweep),
  // halved where the grid would be too small (psmooth_min_blocks).  On the
  // finest level of a 512^3 f(R) solve (plain coarse form) a step took 31.7
  // ms with 8, 31.8 with 4, 32.1 with 2, 32.2 with 16 and 32.9 unfused;
  // MGGPU_PROLONG_SMOOTH_KT overrides it at context creation
  int psmooth_kt = 8;
  // fewest workgroups of a fused prolongation launch (the depth is halved to
  // reach it).  512 also fuses the 256^3 level of a 512^3 solve (4 planes
  // per workgroup): 29.89 ms per step against 29.95 / 30.00 with 1024 / 2048
  // (2 and 1 planes there) and 29.99 with 256; MGGPU_PROLONG_SMOOTH_MIN_BLOCKS
  // overrides it at context creation
  unsigned psmooth_min_blocks = 512;
  // scale applied to each FP32 correction before the FP64 update (1: the
  // method; another value forces the divergence path from the host in tests;
  // MGGPU_TEST_CORRECTION_SCALE overrides it at context creation)
  float test_escale = 1.0f;
  // set while mg_solve_noalloc runs on the static scratch array: any device
  // allocation is then an error instead
  bool noalloc = false;
  // finest-level X and rho of the FP32-refined solve in 16-bit floats
  // (MGGPU_FP16_STORAGE=0 at context creation keeps them in FP32)
  bool fp16 = true;
  // storage of level 0 in the current outer step of the refined solve
  struct {
    bool x16 = false, r16 = false;
    Store S{1.0f, 1.0f, 1.0f, 1.0f};
  } s0;
  double* part4 = nullptr;     // block maxima (same capacity as part)
  // storage of level 0's dg and r in the current adjoint solve (16-bit when
  // on; x_* scales dg, r_* scales r)
  struct {
    bool on = false;
    Store S{1.0f, 1.0f, 1.0f, 1.0f};
  } a0;
  // device facts for the cooperative batched launch, queried once (property
  // queries cost milliseconds per call): CU count, cooperative support, and
  // resident workgroups per CU for each workgroup size (index log2(BS) - 8)
  int bdev_cus = 0, bdev_coop = -1;
  int bocc[3] = {0, 0, 0};
  std::string arch;  // gcnArchName, part of the tuning-cache key
  std::string err;
  int nlev = 0;
  Lev L[kMaxLev];
  int fused_from = 0;
  bool have64 = false, have32 = false, haveAdj = false;
  Work64 w64;
  Work32 w32;
  WorkAdj adj;
  double* part = nullptr;
  double* part2 = nullptr;
  double* part3 = nullptr;     // second set of block partials (same capacity as part)
  int64_t part_cap = 0;
  double* scal = nullptr;      // device scalars
  double* hscal = nullptr;     // pinned host mirror
  int64_t* cic = nullptr;      // CIC fixed-point accumulator (direct path)
  uint2* cic_rec = nullptr;     // binned CIC: run records, one region per count block
  uint32_t* cic_nrec = nullptr;  // records per region
  unsigned long long* cic_runs = nullptr;  // runs in (tile, class) bin order
  int64_t cic_np = 0;
  uint32_t* cic_cnt = nullptr;  // counts, offsets, cursors per (tile, class) bin
  int cic_direct = 0;           // 1: always the direct atomic path (MGGPU_CIC_DIRECT)
  // batched solves
  void* bpool = nullptr;
  size_t bpool_bytes = 0;
  BoxDev* bdev = nullptr;
  BoxOut* bout = nullptr;
  int bcap = 0;
  // team plan of the batched launch (device copies) and its sync state
  int* border = nullptr;
  TeamDev* bteams = nullptr;
  int2* bwg = nullptr;
  unsigned* bctr = nullptr;
  double* bparts = nullptr;
  int* babort = nullptr;
  int bplan_cap = 0;  // capacity (entries) of border/bteams/bwg/bctr; bparts holds 2x
  int bblock = 0, bvec = -1, bteam = -1;  // last tile shape used
  bool bpinned = false;                    // shape fixed by mg_batched_set_config
  std::string bkey;
  // grouped level launches: per-box table, control words, block partials,
  // per-box sums (device and pinned host)
  GBox* gtab = nullptr;
  GCtl* gctl = nullptr;
  double* gpart = nullptr;
  double* gsum = nullptr;
  double* ghsum = nullptr;
  int gcap = 0;
  int64_t gpart_cap = 0;
  // classes are independent: each runs on one of these streams (default
  // priority), forked from and joined back into the context's stream
  static constexpr int kGStreams = 4;
  hipStream_t gst[kGStreams] = {};
  hipEvent_t gfork = nullptr, gjoin[kGStreams] = {};
  double* nat64 = nullptr;     // natural-layout scratch (debug entry points)
  // Newtonian potential by FFT (rocFFT, FP64), created at first use
  bool fft_ready = false;
  rocfft_plan fft_fwd = nullptr, fft_inv = nullptr;
  rocfft_execution_info fft_info = nullptr;
  void* fft_work = nullptr;
  size_t fft_work_bytes = 0;
  double2* fft_c = nullptr;    // n * n * (n/2 + 1) complex
  double* fft_s2 = nullptr;    // sin^2(pi m / n), m in [0, n)
  std::vector<void*> allocs;
  // event timing of the finest-level smoothers
  bool prof = false;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> ev_cls;
  int ev_used = 0;
  double prof_ms[4] = {0, 0, 0, 0};
  int64_t prof_n[4] = {0, 0, 0, 0};
};

namespace {

inline unsigned nblk(int64_t m) { return (unsigned)((m + kBlock - 1) / kBlock); }

constexpr int kEvPairs = 512;

// accumulate the recorded event pairs (waits for the last one)
void prof_flush(mg_ctx* ctx) {
  if (ctx->ev_used == 0) return;
  (void)hipEventSynchronize(ctx->ev[2 * ctx->ev_used - 1]);
  for (int q = 0; q < ctx->ev_used; ++q) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[2 * q], ctx->ev[2 * q + 1]) == hipSuccess) {
      ctx->prof_ms[ctx->ev_cls[q]] += ms;
      ctx->prof_n[ctx->ev_cls[q]] += 1;
    }
  }
  ctx->ev_used = 0;
}
// returns the pair index to close with prof_end, or -1 when timing is off
int prof_begin(mg_ctx* ctx, int cls) {
  if (!ctx->prof) return -1;
  if (ctx->ev_used == kEvPairs) prof_flush(ctx);
  int q = ctx->ev_used++;
  ctx->ev_cls[q] = cls;
  (void)hipEventRecord(ctx->ev[2 * q], ctx->stream);
  return q;
}
void prof_end(mg_ctx* ctx, int q) {
  if (q >= 0) (void)hipEventRecord(ctx->ev[2 * q + 1], ctx->stream);
}

int fail(mg_ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

#define HIPCHK(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, MG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK()                                                                   \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, MG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
int dalloc(mg_ctx* ctx, T** p, int64_t count) {
  if (ctx->noalloc) {
    *p = nullptr;
    return fail(ctx, MG_EHIP, "device allocation requested inside mg_solve_noalloc");
  }
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (size_t)count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(ctx, MG_EHIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  ctx->allocs.push_back(q);
  *p = (T*)q;
  return MG_OK;
}

#define ACHK(x)                 \
  do {                          \
    int rc_ = (x);              \
    if (rc_ != MG_OK) return rc_; \
  } while (0)

int64_t cells(const Lev& L) { return 2 * L.half; }

int ensure64(mg_ctx* ctx) {
  if (ctx->have64) return MG_OK;
  Work64& W = ctx->w64;
  ACHK(dalloc(ctx, &W.dens0, cells(ctx->L[0])));
  for (int l = 0; l < ctx->nlev; ++l) {
    int64_t m = cells(ctx->L[l]);
    ACHK(dalloc(ctx, &W.v[l], m));
    if (l > 0) {
      ACHK(dalloc(ctx, &W.dens[l], m));
      ACHK(dalloc(ctx, &W.S[l], m));
      ACHK(dalloc(ctx, &W.Rv[l], m));
    }
  }
  ctx->have64 = true;
  return MG_OK;
}

int ensure32(mg_ctx* ctx) {
  if (ctx->have32) return MG_OK;
  Work32& W = ctx->w32;
  ACHK(dalloc(ctx, &W.wbuf[0], cells(ctx->L[0])));
  ACHK(dalloc(ctx, &W.wbuf[1], cells(ctx->L[0])));
  ACHK(dalloc(ctx, &W.ebuf[1], cells(ctx->L[0])));
  W.w = W.wbuf[0];
  for (int l = 0; l < ctx->nlev; ++l) {
    int64_t m = cells(ctx->L[l]);
    ACHK(dalloc(ctx, &W.e[l], m));
    if (l == 0) W.ebuf[0] = W.e[0];
    ACHK(dalloc(ctx, &W.X[l], m));
    ACHK(dalloc(ctx, &W.rho[l], m));
    ACHK(dalloc(ctx, &W.dens[l], m));
    if (l > 0) ACHK(dalloc(ctx, &W.eR[l], m));
  }
  ACHK(dalloc(ctx, &W.X16, cells(ctx->L[0])));
  ACHK(dalloc(ctx, &W.R16, cells(ctx->L[0])));
  ctx->have32 = true;
  return MG_OK;
}

// caller arrays may be accessed 16 bytes at a time only when so aligned
inline bool al16(const void* a, const void* b = nullptr) {
  return (((uintptr_t)a | (uintptr_t)b) & 15u) == 0;
}

// natural <-> packed transposes, 8 cells per thread when n % 8 == 0
template <typename TI, typename TO>
void launch_pack(mg_ctx* ctx, const Lev& L, const TI* nat, TO* pk, double scale) {
  if (L.n % 8 == 0 && al16(nat, pk))
    k_pack8<TI, TO><<<nblk(cells(L) / 8), kBlock, 0, ctx->stream>>>(L, nat, pk, scale);
  else
    k_pack<TI, TO><<<nblk(cells(L)), kBlock, 0, ctx->stream>>>(L, nat, pk, scale);
}
template <typename TI, typename TO>
void launch_unpack(mg_ctx* ctx, const Lev& L, const TI* pk, TO* nat, double scale) {
  if (L.n % 8 == 0 && al16(nat, pk))
    k_unpack8<TI, TO><<<nblk(cells(L) / 8), kBlock, 0, ctx->stream>>>(L, pk, nat, scale);
  else
    k_unpack<TI, TO><<<nblk(cells(L)), kBlock, 0, ctx->stream>>>(L, pk, nat, scale);
}

// v += P(c - c2) (c2 may be null): the z-marching kernel when the coarse
// side is a multiple of 4 (the caller guarantees nc % Vec<T>::V == 0)
constexpr int kProlongKT = 4;  // coarse planes per marching thread
constexpr int kRestrictKT = 4;
template <typename T, int COL0>
void launch_prolong(mg_ctx* ctx, const Lev& Lf, const Lev& Lc, T* v, const T* c, const T* c2) {
  if (Lc.n % 4 == 0 && Lc.n >= 8) {
    k_prolong_kv<T, COL0><<<prolong_march_blocks(Lc.n, kProlongKT), kBlock, 0, ctx->stream>>>(
        Lf, Lc, v, c, c2, kProlongKT);
  } else {
    k_prolong_v<T, COL0><<<nblk(cells(Lc) / Vec<T>::V), kBlock, 0, ctx->stream>>>(Lf, Lc, v, c,
                                                                                  c2);
  }
}

template <typename T>
int ensure_lin(mg_ctx* ctx, WorkLin<T>& W) {
  for (int l = 0; l < ctx->nlev; ++l) {
    int64_t m = cells(ctx->L[l]);
    ACHK(dalloc(ctx, &W.e[l], m));
    ACHK(dalloc(ctx, &W.r[l], m));
    if (l > 0 || sizeof(T) == 4) ACHK(dalloc(ctx, &W.dg[l], m));
  }
  W.ebuf[0] = W.e[0];
  ACHK(dalloc(ctx, &W.ebuf[1], cells(ctx->L[0])));
  if (sizeof(T) == 4) {
    ACHK(dalloc(ctx, &W.dg16, cells(ctx->L[0])));
    ACHK(dalloc(ctx, &W.r16, cells(ctx->L[0])));
  }
  return MG_OK;
}

// Calls fn(dg, r) with the level's dg and r in the adjoint's current storage
// (16-bit on level 0 of an FP32 solve when ctx->a0.on).
template <typename T, typename Fn>
void with_lin_store(mg_ctx* ctx, WorkLin<T>& W, int l, Fn&& fn) {
  if constexpr (sizeof(T) == 4) {
    if (l == 0 && ctx->a0.on) {
      fn(W.dg16, W.r16);
      return;
    }
  }
  fn(W.dg[l], W.r[l]);
}

int ensure_adj(mg_ctx* ctx, int precision) {
  WorkAdj& A = ctx->adj;
  int64_t m = cells(ctx->L[0]);
  if (!ctx->haveAdj) {
    ACHK(dalloc(ctx, &A.v, m));
    ACHK(dalloc(ctx, &A.dg, m));
    ACHK(dalloc(ctx, &A.b, m));
    ACHK(dalloc(ctx, &A.lambuf[0], m));
    ACHK(dalloc(ctx, &A.lambuf[1], m));
    A.lam = A.lambuf[0];
    ctx->haveAdj = true;
  }
  if (precision == MG_FP32_REFINED && !A.have32) {
    ACHK(ensure_lin<float>(ctx, A.w32));
    A.have32 = true;
  }
  if (precision == MG_FP64 && !A.have64) {
    ACHK(ensure_lin<double>(ctx, A.w64));
    A.w64.dg[0] = A.dg;
    A.have64 = true;
  }
  return MG_OK;
}

// ---------------------------------------------------------------------------
// rocFFT, opened by full path at first use so that it binds to the same HIP
// runtime as this library (a process may hold other copies of it)
// ---------------------------------------------------------------------------
struct RocfftApi {
  void* h = nullptr;
  decltype(&rocfft_setup) setup = nullptr;
  decltype(&rocfft_plan_create) plan_create = nullptr;
  decltype(&rocfft_plan_get_work_buffer_size) work_size = nullptr;
  decltype(&rocfft_execution_info_create) info_create = nullptr;
  decltype(&rocfft_execution_info_set_work_buffer) info_set_work = nullptr;
  decltype(&rocfft_execution_info_set_stream) info_set_stream = nullptr;
  decltype(&rocfft_execute) execute = nullptr;
  decltype(&rocfft_plan_destroy) plan_destroy = nullptr;
  decltype(&rocfft_execution_info_destroy) info_destroy = nullptr;
};

const RocfftApi* rocfft_api(std::string* err) {
  static RocfftApi A;
  static bool tried = false;
  static std::string why;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (!tried) {
    tried = true;
    const char* root = getenv("ROCM_PATH");
    std::string path = std::string(root && *root ? root : "/opt/rocm") + "/lib/librocfft.so.0";
    A.h = dlopen(path.c_str(), RTLD_NOW | RTLD_LOCAL);
    if (!A.h) {
      why = "cannot open " + path;
    } else {
      bool ok = true;
      auto get = [&](auto& f, const char* name) {
        f = reinterpret_cast<std::remove_reference_t<decltype(f)>>(dlsym(A.h, name));
        ok = ok && f != nullptr;
      };
      get(A.setup, "rocfft_setup");
      get(A.plan_create, "rocfft_plan_create");
      get(A.work_size, "rocfft_plan_get_work_buffer_size");
      get(A.info_create, "rocfft_execution_info_create");
      get(A.info_set_work, "rocfft_execution_info_set_work_buffer");
      get(A.info_set_stream, "rocfft_execution_info_set_stream");
      get(A.execute, "rocfft_execute");
      get(A.plan_destroy, "rocfft_plan_destroy");
      get(A.info_destroy, "rocfft_execution_info_destroy");
      if (!ok || A.setup() != rocfft_status_success) {
        why = "rocFFT symbols or setup failed";
        A.h = nullptr;
      }
    }
  }
  if (!A.h) {
    *err = why;
    return nullptr;
  }
  return &A;
}

// ---------------------------------------------------------------------------
// constants and validation
// ---------------------------------------------------------------------------
int make_consts(mg_ctx* ctx, int model, const mg_model_params* P, int n, Consts* out) {
  if (!P) return fail(ctx, MG_EINVAL, "params is NULL");
  if (model < MG_FR || model > MG_CQ) return fail(ctx, MG_EINVAL, "unknown model");
  if (!(P->a > 0.0) || !(P->box_mpch > 0.0) || !(P->omega_m > 0.0) || !(P->omega_m <= 1.0))
    return fail(ctx, MG_EINVAL, "need a > 0, box > 0, 0 < omega_m <= 1");
  Consts C;
  memset(&C, 0, sizeof C);
  C.model = model;
  double a = P->a, om = P->omega_m, ol = 1.0 - om;
  double ct = n * kCOverH0 / P->box_mpch;
  C.ct2 = ct * ct;
  C.om_a = om / a;
  if (model == MG_FR) {
    if (P->fr_n < 0 || P->fr_n > 2) return fail(ctx, MG_EINVAL, "f(R): n must be 0, 1 or 2");
    if (!(P->fr_fr0_abs > 0.0)) return fail(ctx, MG_EINVAL, "f(R): |f_R0| must be > 0");
    // R-bar(a)/H0^2 = 3 (Om a^-3 + 4 OL); K = R-bar a^2 / 3
    double ra = om / (a * a * a) + 4.0 * ol;
    C.K = ra * a * a;
    double ratio = (om + 4.0 * ol) / ra;  // R-bar_0 / R-bar(a)
    C.fr_n = P->fr_n;
    C.wbar = P->fr_fr0_abs * pow(ratio, double(P->fr_n + 1));
    C.wpow = pow(C.wbar, 1.0 / double(P->fr_n + 1));
    C.phi5 = 0.5 * C.ct2;
    C.bg = C.wbar;
    C.bg_coef = C.om_a;
  } else if (model == MG_SYMMETRON) {
    if (!(P->sym_xi > 0.0)) return fail(ctx, MG_EINVAL, "symmetron: xi must be > 0");
    if (!(P->sym_a_star > 0.0) || !(P->sym_a_star < a))
      return fail(ctx, MG_EINVAL, "symmetron: need 0 < a_* < a (background u > 0)");
    C.s_ratio = pow(P->sym_a_star / a, 3.0);
    C.s_amp = a * a / (2.0 * P->sym_xi * P->sym_xi);
    C.ubar = sqrt(1.0 - C.s_ratio);
    C.phi5 = 3.0 * P->sym_xi * P->sym_xi * om * P->sym_beta_star * P->sym_beta_star * C.ct2 /
             pow(P->sym_a_star, 3.0);
    C.bg = C.ubar;
    C.bg_coef = C.s_amp * C.s_ratio * C.ubar;
  } else {
    if (!(P->cq_phibar > 0.0) || !(P->cq_alpha > 0.0))
      return fail(ctx, MG_EINVAL, "CQ: need phibar > 0 and alpha > 0");
    C.beta = P->cq_beta;
    C.alpha = P->cq_alpha;
    C.phibar = P->cq_phibar;
    C.cq_keep_exp = P->cq_keep_exp ? 1 : 0;
    C.cq_src = 3.0 * P->cq_beta * om / a * exp(P->cq_beta * P->cq_phibar);
    C.cq_pot = P->cq_alpha * P->cq_lambda * P->cq_lambda * a * a;
    C.cq_pb = pow(P->cq_phibar, -(1.0 + P->cq_alpha));
    C.phi5 = P->cq_beta;
    C.bg = 0.0;
    C.bg_coef = fabs(C.cq_src);
  }
  C.f_ct2 = float(C.ct2);
  C.f_kw = float(C.K * C.wpow);
  C.f_s_ratio = float(C.s_ratio);
  C.f_s_amp = float(C.s_amp);
  C.f_beta = float(C.beta);
  C.f_alpha = float(C.alpha);
  C.f_phibar = float(C.phibar);
  C.f_cq_src = float(C.cq_src);
  C.f_cq_pot = float(C.cq_pot);
  C.f_i6ct2 = float(1.0 / (6.0 * C.ct2));
  C.f_ict2 = float(1.0 / C.ct2);
  C.f_isamp = C.s_amp > 0.0 ? float(1.0 / C.s_amp) : 0.0f;
  C.f_ct2_samp = C.s_amp > 0.0 ? float(C.ct2 / C.s_amp) : 0.0f;
  *out = C;
  return MG_OK;
}

int check_opts(mg_ctx* ctx, const mg_solver_opts* o) {
  if (!o) return fail(ctx, MG_EINVAL, "opts is NULL");
  if (o->cycle < 0 || o->cycle > 2) return fail(ctx, MG_EINVAL, "cycle must be 0 (V), 1 (F), 2 (W)");
  if (o->nu_pre < 0 || o->nu_pre > 16 || o->nu_post < 1 || o->nu_post > 16)
    return fail(ctx, MG_EINVAL, "need 0 <= nu_pre <= 16 and 1 <= nu_post <= 16");
  if (o->max_cycles < 1 || o->max_cycles > 64) return fail(ctx, MG_EINVAL, "max_cycles in 1..64");
  if (o->precision != MG_FP64 && o->precision != MG_FP32_REFINED)
    return fail(ctx, MG_EINVAL, "precision must be MG_FP64 or MG_FP32_REFINED");
  if (o->inner_cycles < 0 || o->inner_cycles > 16)
    return fail(ctx, MG_EINVAL, "inner_cycles in 0 (automatic) .. 16");
  if (o->coarse_sweeps < 0 || o->coarse_sweeps > 5000)
    return fail(ctx, MG_EINVAL, "coarse_sweeps in 0..5000");
  if (o->fixed_cycles < 0 || o->fixed_cycles > 64)
    return fail(ctx, MG_EINVAL, "fixed_cycles in 0 (iterate to tol) .. 64");
  return MG_OK;
}

// Divergence test of the outer loops: the FP64 residual grew at two
// consecutive checks and is above twice the best seen.  A monotone problem
// contracts at every check, so this does not fire on a converging solve (at
// a rounding floor the residual wanders by far less than a factor of two).
struct GrowthWatch {
  int grew = 0;
  double best = HUGE_VAL, last = -1.0;
  bool diverging(double rel) {
    grew = (last >= 0.0 && rel > last) ? grew + 1 : 0;
    last = rel;
    if (rel < best) best = rel;
    return grew >= 2 && rel > 2.0 * best;
  }
};

double lev_h2(int l) { return double(1u << l) * double(1u << l); }

// Cap on Gauss-Seidel sweeps of the coarsest level (they stop early once the
// RMS residual has dropped by 1e-8).  For the usual 4^3 / 6^3 / 8^3: 24 when
// the hierarchy has at most 4 levels, where the coarsest solve sets the
// cycle's contraction; 8 from 5 levels up, where the cycle contraction was
// measured to be the same with 4 to 24 sweeps.  A larger coarsest level
// (n = odd * 2^l with a big odd factor) needs about 2 n^2 sweeps, the slowest
// mode contracting by 1 - O(1/n^2) per sweep.
int default_coarse_sweeps(int nc, int nlev) {
  if (nc <= 8) return nlev >= 5 ? 8 : 24;
  return 2 * nc * nc;
}

// Sweeps per cycle of a grid that cannot be coarsened (n/2 odd or < 4):
// it is its own coarsest level, relaxed without the early stop.
int single_level_sweeps(const mg_ctx* ctx, const mg_solver_opts* o) {
  int cap = o->coarse_sweeps > 0 ? o->coarse_sweeps : default_coarse_sweeps(ctx->L[0].n, 1);
  int nu = o->nu_pre + o->nu_post;
  return cap > nu ? cap : nu;
}

// Cycles to run before the next residual check.  fixed > 0: that many.
// Otherwise from the contraction per cycle seen so far: enough to reach
// tol with 5% margin, between 1 and kMaxPlanned (2 before anything is
// measured).  In the refined mode one check's FP32 cycles can reduce the
// residual by up to ~1e-6 before FP32 rounding of the correction matters.
constexpr int kMaxPlanned = 8;
// Cycles to the next FP64 check, from the contraction measured over the last
// group of cycles.  On large grids that rate is taken no better than
// kRhoFloor: the first cycles damp the rough error fast (per-cycle rates of
// 0.06-0.16 at 512^3) and the rate then settles near 0.2 for V(1,1), so the
// early rate stops a cycle short of tol and costs an extra FP64 check, a
// full pass over the master that is worth about half a cycle there.  On
// small grids a check is cheap next to a cycle and the measured rate is used.
constexpr double kRhoFloor = 0.18;
// Reduction one outer step is asked for when level 0's X and rho are stored
// in 16 bits (their rounding, ~1e-4 relative, perturbs the inner operator
// and right-hand side, which bounds what one step can deliver).
constexpr double kStore16Step = 1e-3;
constexpr int64_t kRhoFloorCells = int64_t(1) << 24;  // 256^3
// step_floor > 0: one check's cycles aim no lower than rel * step_floor (the
// reduction one outer step can deliver when the finest level's data are
// stored in 16 bits); first: cycles before anything is measured.
int plan_cycles(int fixed, double rel, double rel_prev, int k_prev, double tol, int64_t cells,
                double step_floor = 0.0, int first = 2) {
  if (fixed > 0) return fixed;
  if (rel_prev <= 0.0 || k_prev <= 0 || !(rel < rel_prev)) return first;
  double rho = pow(rel / rel_prev, 1.0 / k_prev);
  const double floor_rho = cells >= kRhoFloorCells ? kRhoFloor : 0.01;
  if (rho < floor_rho) rho = floor_rho;
  if (rho > 0.9) rho = 0.9;
  const double target = tol > rel * step_floor ? tol : rel * step_floor;
  double need = 1.05 * log(target / rel) / log(rho);
  int k = (int)ceil(need);
  return k < 1 ? 1 : (k > kMaxPlanned ? kMaxPlanned : k);
}

// ---------------------------------------------------------------------------
// reductions to the host
// ---------------------------------------------------------------------------
// deterministic: fixed chunks summed by up to 256 blocks, then one block
int sum_on_device(mg_ctx* ctx, int64_t nparts, double* dst, const double* src = nullptr) {
  int64_t nb = (nparts + 2047) / 2048;
  if (nb > 256) nb = 256;
  int64_t chunk = (nparts + nb - 1) / nb;
  k_sum_chunks<<<(unsigned)nb, 256, 0, ctx->stream>>>(src ? src : ctx->part, nparts, chunk,
                                                      ctx->part2);
  k_sum_partials<<<1, 256, 0, ctx->stream>>>(ctx->part2, nb, dst, 0);
  LAUNCHCHK();
  return MG_OK;
}

// the same for maxima of non-negative partials: src -> *dst on the device
int max_on_device(mg_ctx* ctx, int64_t nparts, const double* src, double* dst) {
  int64_t nb = (nparts + 2047) / 2048;
  if (nb > 256) nb = 256;
  const int64_t chunk = (nparts + nb - 1) / nb;
  k_max_chunks<<<(unsigned)nb, 256, 0, ctx->stream>>>(src, nparts, chunk, ctx->part2);
  k_max_partials<<<1, 256, 0, ctx->stream>>>(ctx->part2, nb, dst);
  LAUNCHCHK();
  return MG_OK;
}

int sum_to_host(mg_ctx* ctx, int64_t nparts, double* out, const double* src = nullptr) {
  ACHK(sum_on_device(ctx, nparts, ctx->scal, src));
  HIPCHK(hipMemcpyAsync(ctx->hscal, ctx->scal, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *out = ctx->hscal[0];
  return MG_OK;
}

// two sums with one synchronisation: ctx->part -> *a, src_b -> *b
int sum2_to_host(mg_ctx* ctx, int64_t nparts, double* a, double* b, const double* src_b) {
  ACHK(sum_on_device(ctx, nparts, ctx->scal));
  ACHK(sum_on_device(ctx, nparts, ctx->scal + 1, src_b));
  HIPCHK(hipMemcpyAsync(ctx->hscal, ctx->scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *a = ctx->hscal[0];
  *b = ctx->hscal[1];
  return MG_OK;
}

// Reductions of one refined outer pass with one synchronisation: sum d^2
// (ctx->part) -> *s; with bg, sum (bg_coef delta)^2 (ctx->part3) -> *sb; with
// mx_on, max |d| (ctx->part4) -> *mx.
int outer_sums(mg_ctx* ctx, int64_t nparts, bool bg, bool mx_on, double* s, double* sb,
               double* mx) {
  ACHK(sum_on_device(ctx, nparts, ctx->scal));
  if (bg) ACHK(sum_on_device(ctx, nparts, ctx->scal + 1, ctx->part3));
  if (mx_on) ACHK(max_on_device(ctx, nparts, ctx->part4, ctx->scal + 2));
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(ctx->hscal, ctx->scal, 3 * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *s = ctx->hscal[0];
  if (bg) *sb = ctx->hscal[1];
  if (mx_on) *mx = ctx->hscal[2];
  return MG_OK;
}

// Normaliser of the relative residual: RMS of the background residual,
// bg_coef RMS(delta).  For delta = 0 the background solves the equation and
// the ratio is undefined; the residual of a unit contrast, bg_coef, is used,
// which keeps the test scale-aware (rounding noise at the background then
// reads as converged).
inline double bg_norm_of(const Consts& C, double r) {
  if (r > 0.0) return r;
  return C.bg_coef > 0.0 ? C.bg_coef : 1.0;
}

int bg_rms(mg_ctx* ctx, const Consts& C, const float* delta, double* out) {
  int64_t m = cells(ctx->L[0]);
  k_bg_norm<<<nblk(m), kBlock, 0, ctx->stream>>>(m, delta, C.bg_coef, ctx->part);
  LAUNCHCHK();
  double s;
  ACHK(sum_to_host(ctx, nblk(m), &s));
  *out = bg_norm_of(C, sqrt(s / double(m)));
  return MG_OK;
}

// ---------------------------------------------------------------------------
// fused-program generation (same recursion as the grid levels)
// ---------------------------------------------------------------------------
// A cycle program in a fixed host buffer (no heap allocation per cycle);
// 'over' records a program longer than the buffer.
struct OpList {
  static constexpr int kCap = kMaxOpsB > kMaxOps ? kMaxOpsB : kMaxOps;
  Op op[kCap];
  int n = 0;
  bool over = false;
  void push(Op o) {
    if (n < kCap) op[n++] = o;
    else over = true;
  }
};

void gen_prog(OpList& ops, int l, int lmax, int type, int nu1, int nu2) {
  if (ops.over) return;
  if (l == lmax) {
    ops.push(Op{OP_COARSEST, (uint8_t)l, 0, 0});
    return;
  }
  if (nu1 > 0) ops.push(Op{OP_SMOOTH, (uint8_t)l, (uint8_t)nu1, 0});
  ops.push(Op{OP_DOWN, (uint8_t)l, 0, 0});
  if (type == MG_CYCLE_V) {
    gen_prog(ops, l + 1, lmax, MG_CYCLE_V, nu1, nu2);
  } else if (type == MG_CYCLE_W) {
    gen_prog(ops, l + 1, lmax, MG_CYCLE_W, nu1, nu2);
    gen_prog(ops, l + 1, lmax, MG_CYCLE_W, nu1, nu2);
  } else {
    gen_prog(ops, l + 1, lmax, MG_CYCLE_F, nu1, nu2);
    gen_prog(ops, l + 1, lmax, MG_CYCLE_V, nu1, nu2);
  }
  ops.push(Op{OP_UP, (uint8_t)l, 0, 0});
  ops.push(Op{OP_SMOOTH, (uint8_t)l, (uint8_t)nu2, 0});
}

int make_prog(mg_ctx* ctx, int l, const mg_solver_opts* o, int type, FusedProg* P, int rx = 0) {
  OpList ops;
  int f = ctx->fused_from;
  gen_prog(ops, l - f, ctx->nlev - 1 - f, type, o->nu_pre, o->nu_post);
  if (ops.over || ops.n > kMaxOps) return fail(ctx, MG_EINVAL, "fused cycle program too long");
  P->nops = ops.n;
  P->coarse_sweeps =
      o->coarse_sweeps > 0 ? o->coarse_sweeps : default_coarse_sweeps(ctx->L[ctx->nlev - 1].n, ctx->nlev);
  P->rx = rx;
  for (int q = 0; q < ops.n; ++q) P->op[q] = ops.op[q];
  return MG_OK;
}

// ---------------------------------------------------------------------------
// FP64 direct multigrid
// ---------------------------------------------------------------------------
template <int M>
int smooth64(mg_ctx* ctx, const Consts& C, int l, int sweeps) {
  Work64& W = ctx->w64;
  const Lev& L = ctx->L[l];
  const bool vec = (L.nh % Vec<double>::V) == 0;
  const int64_t nv = L.half / Vec<double>::V;
  for (int s = 0; s < sweeps; ++s)
    for (int colour = 0; colour < 2; ++colour) {
      if (l == 0) {
        int q = prof_begin(ctx, MG_PROF_SMOOTH64);
        if (vec)
          k_smooth_direct_v<M, float><<<nblk(nv), kBlock, 0, ctx->stream>>>(
              L, W.v[0], W.dens0, (const double*)nullptr, colour, 1.0, C);
        else
          k_smooth_direct<M, double, float><<<nblk(L.half), kBlock, 0, ctx->stream>>>(
              L, W.v[0], W.dens0, (const double*)nullptr, colour, 1.0, C);
        prof_end(ctx, q);
      } else if (vec) {
        k_smooth_direct_v<M, double><<<nblk(nv), kBlock, 0, ctx->stream>>>(
            L, W.v[l], W.dens[l], W.S[l], colour, lev_h2(l), C);
      } else {
        k_smooth_direct<M, double, double><<<nblk(L.half), kBlock, 0, ctx->stream>>>(
            L, W.v[l], W.dens[l], W.S[l], colour, lev_h2(l), C);
      }
    }
  LAUNCHCHK();
  return MG_OK;
}

template <int M>
int cycle64(mg_ctx* ctx, const Consts& C, const mg_solver_opts* o, int l, int type) {
  Work64& W = ctx->w64;
  if (l >= ctx->fused_from) {
    FusedDirect<double, double> F;
    memset(&F, 0, sizeof F);
    int f = ctx->fused_from;
    F.nlev = ctx->nlev - f;
    for (int q = 0; q < F.nlev; ++q) {
      F.L[q] = ctx->L[f + q];
      F.h2[q] = lev_h2(f + q);
      F.v[q] = W.v[f + q];
      F.dens[q] = W.dens[f + q];
      F.S[q] = W.S[f + q];
      F.Rv[q] = W.Rv[f + q];
    }
    FusedProg P;
    ACHK(make_prog(ctx, l, o, type, &P));
    k_fused_direct<M, double, double><<<1, kFusedThreads, 0, ctx->stream>>>(F, P, C);
    LAUNCHCHK();
    return MG_OK;
  }
  if (l == ctx->nlev - 1) {  // single-level grid: relax only
    return smooth64<M>(ctx, C, l, single_level_sweeps(ctx, o));
  }
  const Lev& Lf = ctx->L[l];
  const Lev& Lc = ctx->L[l + 1];
  ACHK(smooth64<M>(ctx, C, l, o->nu_pre));
  const bool vec = Lc.n % Vec<double>::V == 0;
  const int64_t ncv = cells(Lc) / Vec<double>::V;
  // f(R) and the symmetron solve each cell exactly: after a pre-smoothing
  // sweep the colour updated last has zero residual
  const int skip1 = (M != CQ && o->nu_pre > 0) ? 1 : 0;
  if (l == 0 && vec)
    k_resid_restrict_direct_v<M, float><<<nblk(ncv), kBlock, 0, ctx->stream>>>(
        Lf, Lc, W.v[0], W.dens0, (const double*)nullptr, 1.0, W.Rv[1], W.v[1], W.S[1], C, skip1);
  else if (l == 0)
    k_resid_restrict_direct<M, double, float><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(
        Lf, Lc, W.v[0], W.dens0, (const double*)nullptr, 1.0, W.Rv[1], W.v[1], W.S[1], C);
  else if (vec)
    k_resid_restrict_direct_v<M, double><<<nblk(ncv), kBlock, 0, ctx->stream>>>(
        Lf, Lc, W.v[l], W.dens[l], W.S[l], lev_h2(l), W.Rv[l + 1], W.v[l + 1], W.S[l + 1], C,
        skip1);
  else
    k_resid_restrict_direct<M, double, double><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(
        Lf, Lc, W.v[l], W.dens[l], W.S[l], lev_h2(l), W.Rv[l + 1], W.v[l + 1], W.S[l + 1], C);
  k_coarse_src_direct<M, double, double><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(
      Lc, W.Rv[l + 1], W.dens[l + 1], W.S[l + 1], lev_h2(l + 1), C);
  LAUNCHCHK();
  if (type == MG_CYCLE_V) {
    ACHK(cycle64<M>(ctx, C, o, l + 1, MG_CYCLE_V));
  } else if (type == MG_CYCLE_W) {
    ACHK(cycle64<M>(ctx, C, o, l + 1, MG_CYCLE_W));
    ACHK(cycle64<M>(ctx, C, o, l + 1, MG_CYCLE_W));
  } else {
    ACHK(cycle64<M>(ctx, C, o, l + 1, MG_CYCLE_F));
    ACHK(cycle64<M>(ctx, C, o, l + 1, MG_CYCLE_V));
  }
  if (vec) {
    // v += P(v_H - R v); colour 0 only for the Newton (CQ) smoother
    launch_prolong<double, M == CQ ? 0 : 1>(ctx, Lf, Lc, W.v[l], W.v[l + 1], W.Rv[l + 1]);
  } else {
    k_coarse_diff<double><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(cells(Lc), W.v[l + 1],
                                                                         W.Rv[l + 1]);
    k_prolong_block<double><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(Lf, Lc, W.v[l],
                                                                           W.Rv[l + 1]);
  }
  LAUNCHCHK();
  return smooth64<M>(ctx, C, l, o->nu_post);
}

template <int M>
int resid64(mg_ctx* ctx, const Consts& C, double eps_bg, double* rel, double* d_nat) {
  const Lev& L = ctx->L[0];
  int64_t nparts;
  if (L.nh % Vec<double>::V == 0) {
    nparts = nblk(L.half / Vec<double>::V);
    k_resid_norm_v<M, float><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
        L, ctx->w64.v[0], ctx->w64.dens0, C, ctx->part, d_nat);
  } else {
    nparts = nblk(cells(L));
    k_resid_norm_direct<M, double, float><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
        L, ctx->w64.v[0], ctx->w64.dens0, 1.0, C, ctx->part, d_nat);
  }
  LAUNCHCHK();
  double s;
  ACHK(sum_to_host(ctx, nparts, &s));
  *rel = sqrt(s / double(cells(L))) / eps_bg;
  return MG_OK;
}

// pack the finest-level inputs and restrict the density pyramid (FP64 mode)
int setup64(mg_ctx* ctx, const Consts& C, const float* delta, const double* field_in) {
  Work64& W = ctx->w64;
  const Lev& L0 = ctx->L[0];
  int64_t m = cells(L0);
  launch_pack<float, float>(ctx, L0, delta, W.dens0, 1.0);
  for (int l = 0; l + 1 < ctx->nlev; ++l) {
    if (l == 0)
      k_restrict<float, double><<<nblk(cells(ctx->L[1])), kBlock, 0, ctx->stream>>>(
          L0, ctx->L[1], W.dens0, W.dens[1]);
    else
      k_restrict<double, double><<<nblk(cells(ctx->L[l + 1])), kBlock, 0, ctx->stream>>>(
          ctx->L[l], ctx->L[l + 1], W.dens[l], W.dens[l + 1]);
  }
  double sgn = (C.model == FR) ? -1.0 : 1.0;  // f(R): w = -f_R
  if (field_in)
    launch_pack<double, double>(ctx, L0, field_in, W.v[0], sgn);
  else
    k_fill<double><<<nblk(m), kBlock, 0, ctx->stream>>>(W.v[0], m, C.bg);
  LAUNCHCHK();
  return MG_OK;
}

template <int M>
int solve64(mg_ctx* ctx, const Consts& C, const mg_solver_opts* o, const float* delta,
            const double* field_in, double* field_out, double tol, mg_stats* st) {
  ACHK(ensure64(ctx));
  ACHK(setup64(ctx, C, delta, field_in));
  double sgn = (C.model == FR) ? -1.0 : 1.0;
  const Lev& L0 = ctx->L[0];
  if (o->fixed_cycles > 0) {
    // the paper's fixed cycles per time step: no residual unless asked for
    for (int it = 0; it < o->fixed_cycles; ++it) ACHK(cycle64<M>(ctx, C, o, 0, o->cycle));
    int rc = MG_OK;
    if (st) {
      double eps_bg, rel;
      ACHK(bg_rms(ctx, C, delta, &eps_bg));
      ACHK(resid64<M>(ctx, C, eps_bg, &rel, nullptr));
      st->cycles = 1;
      st->vcycles = o->fixed_cycles;
      st->rel_resid = rel;
      st->resid_hist[0] = rel;
      if (!std::isfinite(rel)) rc = fail(ctx, MG_ENAN, "non-finite residual");
    }
    launch_unpack<double, double>(ctx, L0, ctx->w64.v[0], field_out, sgn);
    LAUNCHCHK();
    return rc;
  }
  double eps_bg;
  ACHK(bg_rms(ctx, C, delta, &eps_bg));
  double rel;
  ACHK(resid64<M>(ctx, C, eps_bg, &rel, nullptr));
  int cyc = 0, checks = 0, k_prev = 0;
  double rel_prev = -1.0;
  int rc = MG_OK;
  GrowthWatch watch;
  watch.diverging(rel);
  if (!std::isfinite(rel)) rc = fail(ctx, MG_ENAN, "non-finite residual");
  while (rc == MG_OK && rel > tol && cyc < o->max_cycles) {
    // the residual is checked after each planned group of cycles
    int k = plan_cycles(o->inner_cycles, rel, rel_prev, k_prev, tol, cells(ctx->L[0]));
    if (k > o->max_cycles - cyc) k = o->max_cycles - cyc;
    for (int it = 0; it < k; ++it) ACHK(cycle64<M>(ctx, C, o, 0, o->cycle));
    cyc += k;
    rel_prev = rel;
    k_prev = k;
    ACHK(resid64<M>(ctx, C, eps_bg, &rel, nullptr));
    if (st && checks < 64) st->resid_hist[checks] = rel;
    ++checks;
    if (!std::isfinite(rel)) {
      rc = fail(ctx, MG_ENAN, "non-finite residual");
      break;
    }
    if (rel > tol && watch.diverging(rel)) {
      rc = fail(ctx, MG_ENOCONV, "residual grew at two consecutive checks (diverging)");
      break;
    }
  }
  if (rc == MG_OK && rel > tol) rc = fail(ctx, MG_ENOCONV, "max_cycles reached");
  launch_unpack<double, double>(ctx, L0, ctx->w64.v[0], field_out, sgn);
  LAUNCHCHK();
  if (st) {
    st->cycles = checks;
    st->vcycles = cyc;
    st->rel_resid = rel;
  }
  return rc;
}

// ---------------------------------------------------------------------------
// FP32 correction multigrid inside an FP64 outer loop
// ---------------------------------------------------------------------------
// Calls fn(X, rho) with level 0's X and rho in the current outer step's
// storage (FP32 or 16-bit); other levels are FP32.
template <typename Fn>
void with_level_store(mg_ctx* ctx, int l, Fn&& fn) {
  Work32& W = ctx->w32;
  const bool x16 = l == 0 && ctx->s0.x16, r16 = l == 0 && ctx->s0.r16;
  if (x16 && r16) fn(W.X16, W.R16);
  else if (x16) fn(W.X16, W.rho[l]);
  else if (r16) fn(W.X[l], W.R16);
  else fn(W.X[l], W.rho[l]);
}
inline Store level_store(const mg_ctx* ctx, int l) {
  return l == 0 ? ctx->s0.S : Store{1.0f, 1.0f, 1.0f, 1.0f};
}

// e *= s over m cells (the divergence test hook, MGGPU_TEST_CORRECTION_SCALE)
__global__ __launch_bounds__(kBlock) void k_scale(float* __restrict__ e, int64_t m, float s) {
  const int64_t g = gid();
  if (g < m) e[g] *= s;
}

template <int M>
// fresh: the correction buffer was not cleared; the first sweep takes it as 0
// skip0: the first colour-0 half-sweep was done by the fused prolongation
int smooth32(mg_ctx* ctx, const Consts& C, int l, int sweeps, bool fresh = false,
             bool skip0 = false) {
  Work32& W = ctx->w32;
  const Lev& L = ctx->L[l];
  const bool vec = (L.nh % Vec<float>::V) == 0;
  const int64_t nv = L.half / Vec<float>::V;
  for (int s = 0; s < sweeps; ++s)
    for (int colour = 0; colour < 2; ++colour) {
      if (skip0 && s == 0 && colour == 0) continue;
      // timed class: full half-sweeps of the finest level (a fresh colour-0
      // half-sweep reads no neighbours and is left out)
      const bool light = fresh && s == 0 && colour == 0;
      int q = (l == 0 && !light) ? prof_begin(ctx, MG_PROF_SMOOTH32) : -1;
      const int kt = ctx->smooth_march_kt;
      const Store S = level_store(ctx, l);
      const int fr = (fresh && s == 0) ? 1 : 0;
      if (vec && kt > 0 && march_blocks(L, kt, Vec<float>::V) >= ctx->march_min_blocks)
        with_level_store(ctx, l, [&](auto* X, auto* R) {
          using TX = std::remove_pointer_t<decltype(X)>;
          using TR = std::remove_pointer_t<decltype(R)>;
          k_smooth_corr_kv<M, TX, TR>
              <<<march_blocks(L, kt, Vec<float>::V), kBlock, 0, ctx->stream>>>(
                  L, W.e[l], X, W.dens[l], R, colour, float(lev_h2(l)), C, fr, kt, S);
        });
      else if (vec)
        with_level_store(ctx, l, [&](auto* X, auto* R) {
          using TX = std::remove_pointer_t<decltype(X)>;
          using TR = std::remove_pointer_t<decltype(R)>;
          k_smooth_corr_v<M, TX, TR><<<nblk(nv), kBlock, 0, ctx->stream>>>(
              L, W.e[l], X, W.dens[l], R, colour, float(lev_h2(l)), C, fr, S);
        });
      else
        k_smooth_corr<M><<<nblk(L.half), kBlock, 0, ctx->stream>>>(L, W.e[l], W.X[l], W.dens[l],
                                                                   W.rho[l], colour,
                                                                   float(lev_h2(l)), C);
      prof_end(ctx, q);
    }
  LAUNCHCHK();
  return MG_OK;
}

// Coarse planes per workgroup of the prolongation fused into level l's first
// post-smoothing half-sweep (exact per-cell FP32 smoothers), or 0 where the
// two run separately: the configured depth, halved until the grid has
// ctx->psmooth_min_blocks workgroups; 0 if one plane per workgroup is not
// enough or the coarse side does not tile.
int fuse_prolong_kt(const mg_ctx* ctx, int l) {
  const Lev& Lf = ctx->L[l];
  const Lev& Lc = ctx->L[l + 1];
  const int R = prolong_smooth_rows(Lc.n);
  if (ctx->psmooth_kt <= 0 || ctx->smooth_march_kt <= 0 || Lf.nh % 4 != 0 || R == 0) return 0;
  const unsigned ntile = (unsigned)((Lc.n + R - 1) / R);
  for (int kt = ctx->psmooth_kt; kt >= 1; kt /= 2)
    if (ntile * (unsigned)((Lc.n + kt - 1) / kt) >= ctx->psmooth_min_blocks) return kt;
  return 0;
}
bool fuse_prolong(const mg_ctx* ctx, int l) { return fuse_prolong_kt(ctx, l) > 0; }
template <class U>
void launch_prolong_smooth0(mg_ctx* ctx, int l, float* e, const float* c, const float* c2,
                            const U& upd) {
  const Lev& Lf = ctx->L[l];
  const Lev& Lc = ctx->L[l + 1];
  const int R = prolong_smooth_rows(Lc.n), kt = fuse_prolong_kt(ctx, l);
  const unsigned ntile = (unsigned)((Lc.n + R - 1) / R), nz = (unsigned)((Lc.n + kt - 1) / kt);
  k_prolong_smooth0<U><<<ntile * nz, R * (Lc.n / 4), 0, ctx->stream>>>(Lf, Lc, e, c, c2, kt, upd);
}

// rx: restrict the linearisation point X on the way down (first cycle of
// an outer step)
template <int M>
int cycle32(mg_ctx* ctx, const Consts& C, const mg_solver_opts* o, int l, int type, bool rx,
            bool fresh = false) {
  Work32& W = ctx->w32;
  if (l >= ctx->fused_from) {
    FusedCorr F;
    memset(&F, 0, sizeof F);
    int f = ctx->fused_from;
    F.nlev = ctx->nlev - f;
    for (int q = 0; q < F.nlev; ++q) {
      F.L[q] = ctx->L[f + q];
      F.h2[q] = float(lev_h2(f + q));
      F.e[q] = W.e[f + q];
      F.X[q] = W.X[f + q];
      F.dens[q] = W.dens[f + q];
      F.rho[q] = W.rho[f + q];
      F.eR[q] = W.eR[f + q];
    }
    FusedProg P;
    ACHK(make_prog(ctx, l, o, type, &P, rx ? 1 : 0));
    k_fused_corr<M><<<1, kFusedThreads, 0, ctx->stream>>>(F, P, C);
    LAUNCHCHK();
    return MG_OK;
  }
  if (l == ctx->nlev - 1) return smooth32<M>(ctx, C, l, single_level_sweeps(ctx, o), fresh);
  const Lev& Lf = ctx->L[l];
  const Lev& Lc = ctx->L[l + 1];
  ACHK(smooth32<M>(ctx, C, l, o->nu_pre, fresh));
  const bool vec = Lc.n % Vec<float>::V == 0;
  const int64_t ncv = cells(Lc) / Vec<float>::V;
  // exact per-cell smoothers (f(R), symmetron): the colour swept last has
  // zero residual
  const int skip1 = (M != CQ && o->nu_pre > 0) ? 1 : 0;
  const Store S = level_store(ctx, l);
  // The coarse problem is posed around the restricted current approximation
  // (the restriction's shifted form): W.X[l+1] = R X + R e, where R X of
  // this level's linearisation point is formed when that point has changed
  // (rx) and kept in W.eR[l+1] otherwise; the coarse correction starts at
  // zero and is prolonged as it is.  It starts fresh where the coarse
  // level's first half-sweep can take the uncleared buffer as zero (a
  // vectorised smoother that sweeps before anything reads e); elsewhere the
  // restriction writes zeros.
  const Lev& Lc1 = ctx->L[l + 1];
  const bool cfresh = l + 1 < ctx->fused_from && Lc1.nh % Vec<float>::V == 0 &&
                      (o->nu_pre > 0 || l + 1 == ctx->nlev - 1);
  float* ezero = cfresh ? (float*)nullptr : W.e[l + 1];
  float* Xf = W.eR[l + 1];
  const int rxi = rx ? 1 : 0;
  if (skip1 && Lc.n % 4 == 0 && Lc.n >= 8 &&
      prolong_march_blocks(Lc.n, kRestrictKT) >= ctx->march_min_blocks)
    with_level_store(ctx, l, [&](auto* X, auto* R) {
      using TX = std::remove_pointer_t<decltype(X)>;
      using TR = std::remove_pointer_t<decltype(R)>;
      k_resid_restrict_corr_kv<M, TX, TR>
          <<<prolong_march_blocks(Lc.n, kRestrictKT), kBlock, 0, ctx->stream>>>(
              Lf, Lc, W.e[l], X, W.dens[l], R, float(lev_h2(l)), ezero, (float*)nullptr,
              W.rho[l + 1], W.X[l + 1], C, kRestrictKT, S, Xf, rxi);
    });
  else if (vec)
    with_level_store(ctx, l, [&](auto* X, auto* R) {
      using TX = std::remove_pointer_t<decltype(X)>;
      using TR = std::remove_pointer_t<decltype(R)>;
      k_resid_restrict_corr_v<M, TX, TR><<<nblk(ncv), kBlock, 0, ctx->stream>>>(
          Lf, Lc, W.e[l], X, W.dens[l], R, float(lev_h2(l)), ezero, (float*)nullptr,
          W.rho[l + 1], W.X[l + 1], C, skip1, S, Xf, rxi);
    });
  else
    k_resid_restrict_corr<M><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(
        Lf, Lc, W.e[l], W.X[l], W.dens[l], W.rho[l], float(lev_h2(l)), ezero, (float*)nullptr,
        W.rho[l + 1], W.X[l + 1], C, Xf, rxi);
  LAUNCHCHK();
  // the coarse level's linearisation point has changed: its own restriction
  // forms R X again on the first visit; a second visit (W, F) continues
  // from the first visit's correction
  if (type == MG_CYCLE_V) {
    ACHK(cycle32<M>(ctx, C, o, l + 1, MG_CYCLE_V, true, cfresh));
  } else if (type == MG_CYCLE_W) {
    ACHK(cycle32<M>(ctx, C, o, l + 1, MG_CYCLE_W, true, cfresh));
    ACHK(cycle32<M>(ctx, C, o, l + 1, MG_CYCLE_W, false));
  } else {
    ACHK(cycle32<M>(ctx, C, o, l + 1, MG_CYCLE_F, true, cfresh));
    ACHK(cycle32<M>(ctx, C, o, l + 1, MG_CYCLE_V, false));
  }
  if (M != CQ && vec && fuse_prolong(ctx, l)) {
    // e += P e_H formed inside the first colour-0 half-sweep
    with_level_store(ctx, l, [&](auto* X, auto* R) {
      using TX = std::remove_pointer_t<decltype(X)>;
      using TR = std::remove_pointer_t<decltype(R)>;
      const UpdCorr<M, TX, TR> U{X, W.dens[l], R, float(lev_h2(l)), level_store(ctx, l), C};
      launch_prolong_smooth0(ctx, l, W.e[l], W.e[l + 1], (const float*)nullptr, U);
    });
    LAUNCHCHK();
    return smooth32<M>(ctx, C, l, o->nu_post, false, true);
  }
  if (vec) {
    // e += P e_H; colour 0 too only for the Newton (CQ) smoother
    launch_prolong<float, M == CQ ? 0 : 1>(ctx, Lf, Lc, W.e[l], W.e[l + 1], (const float*)nullptr);
  } else {
    k_prolong_block<float><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(Lf, Lc, W.e[l],
                                                                          W.e[l + 1]);
  }
  LAUNCHCHK();
  return smooth32<M>(ctx, C, l, o->nu_post);
}

template <int M>
int solve32(mg_ctx* ctx, const Consts& C, const mg_solver_opts* o, const float* delta,
            const double* field_in, double* field_out, double tol, mg_stats* st) {
  ACHK(ensure32(ctx));
  Work32& W = ctx->w32;
  const Lev& L0 = ctx->L[0];
  int64_t m = cells(L0);
  launch_pack<float, float>(ctx, L0, delta, W.dens[0], 1.0);
  // the f(R) correction operator does not involve the density below level 0
  if (M != FR)
    for (int l = 0; l + 1 < ctx->nlev; ++l)
      k_restrict<float, float><<<nblk(cells(ctx->L[l + 1])), kBlock, 0, ctx->stream>>>(
          ctx->L[l], ctx->L[l + 1], W.dens[l], W.dens[l + 1]);
  double sgn = (C.model == FR) ? -1.0 : 1.0;
  int cur = 0, eb = 0;  // current master buffer, current level-0 correction buffer
  W.w = W.wbuf[cur];
  W.e[0] = W.ebuf[eb];
  const bool fused = L0.nh % kVOuter == 0;
  // Starting from the uniform background, the first two outer kernels take
  // the master as that constant instead of reading it; the first residual is
  // then exactly the background residual whose RMS normalises rel.
  const bool uni = fused && !field_in;
  // 16-bit storage of level 0's X (f(R), symmetron: X/scale near 1 in
  // [2^-24, 32]) and rho (scaled per outer step by a power of two); the
  // first step from a given field keeps rho in FP32 (its scale is unknown).
  // Not for CQ: its Newton smoother is bound by its exp/log arithmetic, so
  // the bytes saved do not pay for the extra cycle the 16-bit floor costs
  // (29.0 against 26.5 ms for the 512^3 solve and force).
  const bool f16 = ctx->fp16 && fused && L0.n % 8 == 0 && M != CQ;
  struct Store0Reset {  // level 0 is FP32 again outside this solve
    mg_ctx* c;
    ~Store0Reset() {
      c->s0.x16 = c->s0.r16 = false;
      c->s0.S = Store{1.0f, 1.0f, 1.0f, 1.0f};
    }
  } store0_reset{ctx};
  ctx->s0.x16 = f16;
  ctx->s0.r16 = false;
  ctx->s0.S = Store{1.0f, 1.0f, 1.0f, 1.0f};
  if (ctx->s0.x16) {
    const double xs = (M == FR ? 1024.0 / C.wbar : 1024.0);
    ctx->s0.S.x_enc = float(xs);
    ctx->s0.S.x_dec = float(1.0 / xs);
  }
  double eps_bg = 1.0;
  if (field_in)
    launch_pack<double, double>(ctx, L0, field_in, W.w, sgn);
  else if (!uni)
    k_fill<double><<<nblk(m), kBlock, 0, ctx->stream>>>(W.w, m, C.bg);
  LAUNCHCHK();
  if (!uni) ACHK(bg_rms(ctx, C, delta, &eps_bg));
  int outer = 0, rc = MG_OK, vc = 0, k_prev = 0;
  double rel = 0.0, rel_prev = -1.0;
  const bool fixed = o->fixed_cycles > 0;
  bool diverged = false;
  GrowthWatch watch;
  // the first pre-smoothing sweep of each outer step treats the correction
  // as zero, so the buffer need not be cleared (not when level 0 is relaxed
  // by the single-block kernel, which reads it, or without pre-smoothing)
  // (only the vectorised level-0 smoother takes the uncleared buffer as zero)
  const bool fresh = fused && L0.nh % Vec<float>::V == 0 && o->nu_pre > 0 && ctx->fused_from > 0;
  const float* pending = nullptr;  // correction not yet added to the master
  for (;;) {
    int64_t nparts;
    double s, sb = 0.0;
    if (fused) {
      // w_new = w + pending, residual at w_new, next correction buffer zeroed
      nparts = march_blocks(L0, kMarchKT, kVOuter);
      double* wn = pending ? W.wbuf[1 - cur] : W.w;
      float* ez = fresh ? nullptr : W.ebuf[pending ? 1 - eb : eb];
      const double* wsrc = (uni && outer <= 1) ? nullptr : W.w;
      // rho's scale: the residual's RMS expected at this check mapped to 2^4
      // (at a uniform start bg_coef delta, whose delta = 1 then maps to 1;
      // after cycles 1/100 of the last check's); a pass whose largest |rho|
      // would overflow is redone with the scale its maximum allows
      const bool r16 = f16 && (uni || outer > 0);
      double rms_pred = outer == 0 ? 16.0 * C.bg_coef : rel * eps_bg * 1e-2;
      int rexp = r16 ? (int)lround(log2(16.0 / (rms_pred > 0.0 ? rms_pred : 1.0))) : 0;
      for (int pass = 0;; ++pass) {
        rexp = rexp > 120 ? 120 : (rexp < -120 ? -120 : rexp);
        ctx->s0.r16 = r16;
        ctx->s0.S.r_enc = float(ldexp(1.0, rexp));
        ctx->s0.S.r_dec = float(ldexp(1.0, -rexp));
        const bool bgsum = uni && outer == 0;
        // the uniform start also sums (bg_coef delta)^2: the background residual
        // in exact arithmetic, which normalises rel (zero for delta = 0, where
        // the computed first residual is rounding noise)
        with_level_store(ctx, 0, [&](auto* X, auto* R) {
          using TX = std::remove_pointer_t<decltype(X)>;
          using TR = std::remove_pointer_t<decltype(R)>;
          k_outer_fused_kv<M, TX, TR><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
              L0, wsrc, pending, wn, W.dens[0], C, R, X, ez, ctx->part,
              bgsum ? ctx->part3 : nullptr, kMarchKT, ctx->s0.S, r16 ? ctx->part4 : nullptr);
        });
        LAUNCHCHK();
        double mx = 0.0;
        ACHK(outer_sums(ctx, nparts, bgsum, r16, &s, &sb, &mx));
        if (!r16 || !(mx * ldexp(1.0, rexp) > 6.0e4) || pass > 0 || !std::isfinite(mx)) break;
        rexp = (int)floor(log2(3.0e4 / mx));
      }
      if (pending) {
        cur = 1 - cur;
        eb = 1 - eb;
        W.w = W.wbuf[cur];
        W.e[0] = W.ebuf[eb];
        pending = nullptr;
      }
    } else {
      nparts = nblk(m);
      k_outer_residual<M><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
          L0, W.w, W.dens[0], C, W.rho[0], W.X[0], W.e[0], ctx->part);
    }
    LAUNCHCHK();
    if (!fused) ACHK(sum_to_host(ctx, nparts, &s));
    if (uni && outer == 0) eps_bg = bg_norm_of(C, sqrt(sb / double(m)));
    rel = sqrt(s / double(m)) / eps_bg;
    if (outer > 0 && st && outer - 1 < 64) st->resid_hist[outer - 1] = rel;
    if (!std::isfinite(rel)) {
      // a finite start that the FP32 cycles turned non-finite: diverged
      if (outer > 0 && !fixed) diverged = true;
      else rc = fail(ctx, MG_ENAN, "non-finite residual");
      break;
    }
    if (fixed ? outer > 0 : rel <= tol) break;
    if (watch.diverging(rel)) {
      diverged = true;
      break;
    }
    if (outer >= o->max_cycles) {
      rc = fail(ctx, MG_ENOCONV, "max_cycles reached");
      break;
    }
    int k = fixed ? o->fixed_cycles
                  : plan_cycles(o->inner_cycles, rel, rel_prev, k_prev, tol, cells(ctx->L[0]),
                                f16 ? kStore16Step : 0.0, f16 ? 4 : 2);
    for (int it = 0; it < k; ++it)
      ACHK(cycle32<M>(ctx, C, o, 0, o->cycle, it == 0, fresh && it == 0));
    if (ctx->test_escale != 1.0f) {
      k_scale<<<nblk(m), kBlock, 0, ctx->stream>>>(W.e[0], m, ctx->test_escale);
      LAUNCHCHK();
    }
    vc += k;
    rel_prev = rel;
    k_prev = k;
    if (fused) {
      pending = W.e[0];  // added by the next fused residual
    } else {
      k_outer_update<<<nblk(m), kBlock, 0, ctx->stream>>>(m, W.w, W.e[0]);
      LAUNCHCHK();
    }
    ++outer;
  }
  if (diverged) {
    // one rerun in plain FP64 from the same start (field_in is unchanged:
    // nothing has been written to field_out yet, which may alias it)
    mg_solver_opts o64 = *o;
    o64.precision = MG_FP64;
    const int rc64 = solve64<M>(ctx, C, &o64, delta, field_in, field_out, tol, st);
    if (st) st->fallback = 1;
    return rc64;
  }
  // stopped before any correction: the master is still the background
  if (uni && outer == 0) k_fill<double><<<nblk(m), kBlock, 0, ctx->stream>>>(W.w, m, C.bg);
  launch_unpack<double, double>(ctx, L0, W.w, field_out, sgn);
  LAUNCHCHK();
  if (st) {
    st->cycles = outer;
    st->vcycles = vc;
    st->rel_resid = rel;
  }
  return rc;
}

// ---------------------------------------------------------------------------
// adjoint: linear multigrid on A lam = b, A = kap(6 - sum)/h^2 + dg
// ---------------------------------------------------------------------------
// The whole adjoint set-up in one pass over the natural cells: the solved
// variable v = sgn field, the Jacobian diagonal dg (FP64, and FP32 when dg32
// is given), the right-hand side b = bsign grad, packed; v itself only when
// the final step needs it (v_out non-null); block partials of b^2.
template <int M>
__global__ __launch_bounds__(kBlock) void k_lin_setup_nat(Lev L, const double* __restrict__ field,
                                                          const float* __restrict__ delta,
                                                          const double* __restrict__ grad,
                                                          double sgn, double bsign, Consts C,
                                                          double* v_out, double* dg, float* dg32,
                                                          double* b, double* part) {
  __shared__ double sh[32];
  int64_t g = gid();
  double bb = 0.0;
  if (g < 2 * L.half) {
    int i, j, k;
    dec_nat(g, L, i, j, k);
    const uint32_t pk = pk_of(L, i, j, k);
    const double v = sgn * field[g];
    const double d = lin_dg<M>(C, v, double(delta[g]));
    dg[pk] = d;
    if (dg32) dg32[pk] = float(d);
    if (v_out) v_out[pk] = v;
    const double bv = bsign * grad[g];
    b[pk] = bv;
    bb = bv * bv;
  }
  double t = block_sum(bb, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
// The same set-up on 8 natural cells of a row per thread (n % 8 == 0,
// 16-byte aligned caller arrays): the row's even cells are 4 consecutive
// packed cells of one colour, its odd cells 4 of the other.
template <int M>
__global__ __launch_bounds__(kBlock) void k_lin_setup_nat8(Lev L, const double* __restrict__ field,
                                                           const float* __restrict__ delta,
                                                           const double* __restrict__ grad,
                                                           double sgn, double bsign, Consts C,
                                                           double* v_out, double* dg, float* dg32,
                                                           double* b, double* part) {
  __shared__ double sh[32];
  const int64_t g8 = gid();
  double bb = 0.0;
  if (g8 < 2 * L.half / 8) {
    const uint32_t g = (uint32_t)g8 * 8u;
    int i0, j, k;
    dec_nat(g, L, i0, j, k);
    const int p = (j + k) & 1;
    const uint32_t row = prow(L, j, k) + (uint32_t)(i0 >> 1);
    const uint32_t pe = (uint32_t)p * (uint32_t)L.half + row;
    const uint32_t po = (uint32_t)(1 - p) * (uint32_t)L.half + row;
    double f[8], gr[8];
    float dl[8];
    ldn<double, 8>(field + g, f);
    ldn<float, 8>(delta + g, dl);
    ldn<double, 8>(grad + g, gr);
    double ve[4], vo[4], de[4], dodd[4], be[4], bo[4];
    float de32[4], do32[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ve[q] = sgn * f[2 * q];
      vo[q] = sgn * f[2 * q + 1];
      de[q] = lin_dg<M>(C, ve[q], double(dl[2 * q]));
      dodd[q] = lin_dg<M>(C, vo[q], double(dl[2 * q + 1]));
      de32[q] = float(de[q]);
      do32[q] = float(dodd[q]);
      be[q] = bsign * gr[2 * q];
      bo[q] = bsign * gr[2 * q + 1];
      bb += be[q] * be[q];
      bb += bo[q] * bo[q];
    }
    stn<double, 4>(dg + pe, de);
    stn<double, 4>(dg + po, dodd);
    if (dg32) {
      stn<float, 4>(dg32 + pe, de32);
      stn<float, 4>(dg32 + po, do32);
    }
    if (v_out) {
      stn<double, 4>(v_out + pe, ve);
      stn<double, 4>(v_out + po, vo);
    }
    stn<double, 4>(b + pe, be);
    stn<double, 4>(b + po, bo);
  }
  double t = block_sum(bb, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_lin_final8(Lev L, const double* v, const double* lam,
                                                       Consts C, double* out_nat) {
  const int64_t g8 = gid();
  if (g8 >= 2 * L.half / 8) return;
  const uint32_t g = (uint32_t)g8 * 8u;
  int i0, j, k;
  dec_nat(g, L, i0, j, k);
  const int p = (j + k) & 1;
  const uint32_t row = prow(L, j, k) + (uint32_t)(i0 >> 1);
  const uint32_t pe = (uint32_t)p * (uint32_t)L.half + row;
  const uint32_t po = (uint32_t)(1 - p) * (uint32_t)L.half + row;
  double le[4], lo[4], ve[4] = {0, 0, 0, 0}, vo[4] = {0, 0, 0, 0}, out[8];
  ldn<double, 4>(lam + pe, le);
  ldn<double, 4>(lam + po, lo);
  if (M != FR) {  // the f(R) source derivative is constant
    ldn<double, 4>(v + pe, ve);
    ldn<double, 4>(v + po, vo);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    out[2 * q] = -lin_dfd<M>(C, ve[q]) * le[q];
    out[2 * q + 1] = -lin_dfd<M>(C, vo[q]) * lo[q];
  }
  stn<double, 8>(out_nat + g, out);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_lin_final(Lev L, const double* v, const double* lam,
                                                      Consts C, double* out_nat) {
  int64_t g = gid();
  if (g >= 2 * L.half) return;
  int colour = g >= L.half ? 1 : 0;
  int64_t gg = g - colour * L.half;
  int ih, j, k;
  dec(gg, L, ih, j, k);
  int i = 2 * ih + ((j + k + colour) & 1);
  const double vv = M == FR ? 0.0 : v[g];  // the f(R) source derivative is constant
  out_nat[((int64_t)k * L.n + j) * L.n + i] = -lin_dfd<M>(C, vv) * lam[g];
}

template <typename T>
int lin_cycle(mg_ctx* ctx, WorkLin<T>& W, double kap, const mg_solver_opts* o, int l, int type,
              bool fresh = false) {
  if (l >= ctx->fused_from) {
    FusedLin<T> F;
    memset(&F, 0, sizeof F);
    int f = ctx->fused_from;
    F.nlev = ctx->nlev - f;
    for (int q = 0; q < F.nlev; ++q) {
      F.L[q] = ctx->L[f + q];
      F.kh2[q] = T(kap / lev_h2(f + q));
      F.e[q] = W.e[f + q];
      F.dg[q] = W.dg[f + q];
      F.r[q] = W.r[f + q];
    }
    FusedProg P;
    ACHK(make_prog(ctx, l, o, type, &P));
    k_fused_lin<T><<<1, kFusedThreads, 0, ctx->stream>>>(F, P);
    LAUNCHCHK();
    return MG_OK;
  }
  const Lev& Lf = ctx->L[l];
  T kh2 = T(kap / lev_h2(l));
  const bool vec = (Lf.nh % Vec<T>::V) == 0;
  const int64_t nv = Lf.half / Vec<T>::V;
  const Store S0 = l == 0 ? ctx->a0.S : Store{1.0f, 1.0f, 1.0f, 1.0f};
  auto smooth = [&](int sweeps, bool first_fresh, bool skip0 = false) {
    for (int s = 0; s < sweeps; ++s)
      for (int colour = 0; colour < 2; ++colour) {
        if (skip0 && s == 0 && colour == 0) continue;  // done by the fused prolongation
        int q = l == 0 ? prof_begin(ctx, sizeof(T) == 4 ? MG_PROF_LIN32 : MG_PROF_LIN64) : -1;
        const int kt = ctx->smooth_march_kt;
        const int fr = (first_fresh && s == 0) ? 1 : 0;
        if (sizeof(T) == 4 && vec && kt > 0 && march_blocks(Lf, kt, 4) >= ctx->march_min_blocks)
          with_lin_store<T>(ctx, W, l, [&](auto* D, auto* R) {
            using TD = std::remove_pointer_t<decltype(D)>;
            using TR = std::remove_pointer_t<decltype(R)>;
            if constexpr (sizeof(T) == 4)
              k_smooth_lin_kv<TD, TR><<<march_blocks(Lf, kt, 4), kBlock, 0, ctx->stream>>>(
                  Lf, (float*)W.e[l], D, R, colour, float(kh2), fr, kt, S0);
          });
        else if (vec)
          with_lin_store<T>(ctx, W, l, [&](auto* D, auto* R) {
            using TD = std::remove_pointer_t<decltype(D)>;
            using TR = std::remove_pointer_t<decltype(R)>;
            k_smooth_lin_v<T, TD, TR><<<nblk(nv), kBlock, 0, ctx->stream>>>(
                Lf, W.e[l], D, R, colour, kh2, fr, S0);
          });
        else
          k_smooth_lin<T><<<nblk(Lf.half), kBlock, 0, ctx->stream>>>(Lf, W.e[l], W.dg[l], W.r[l],
                                                                      colour, kh2);
        prof_end(ctx, q);
      }
  };
  if (l == ctx->nlev - 1) {
    smooth(single_level_sweeps(ctx, o), fresh);
    LAUNCHCHK();
    return MG_OK;
  }
  const Lev& Lc = ctx->L[l + 1];
  smooth(o->nu_pre, fresh);
  const bool cvec = Lc.n % Vec<T>::V == 0;
  const int64_t ncv = cells(Lc) / Vec<T>::V;
  if (o->nu_pre > 0 && Lc.n % 4 == 0 && Lc.n >= 8 &&  // exact per cell: colour 1 skipped
      prolong_march_blocks(Lc.n, kRestrictKT) >= ctx->march_min_blocks)
    with_lin_store<T>(ctx, W, l, [&](auto* D, auto* R) {
      using TD = std::remove_pointer_t<decltype(D)>;
      using TR = std::remove_pointer_t<decltype(R)>;
      k_lin_resid_restrict_kv<T, TD, TR>
          <<<prolong_march_blocks(Lc.n, kRestrictKT), kBlock, 0, ctx->stream>>>(
              Lf, Lc, W.e[l], D, R, kh2, W.r[l + 1], W.e[l + 1], kRestrictKT, S0);
    });
  else if (cvec)  // Gauss-Seidel on a linear system is exact per cell: skip colour 1
    with_lin_store<T>(ctx, W, l, [&](auto* D, auto* R) {
      using TD = std::remove_pointer_t<decltype(D)>;
      using TR = std::remove_pointer_t<decltype(R)>;
      k_lin_resid_restrict_v<T, TD, TR><<<nblk(ncv), kBlock, 0, ctx->stream>>>(
          Lf, Lc, W.e[l], D, R, kh2, W.r[l + 1], W.e[l + 1], o->nu_pre > 0 ? 1 : 0, S0);
    });
  else
    k_lin_resid_restrict<T><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(
        Lf, Lc, W.e[l], W.dg[l], W.r[l], kh2, W.r[l + 1], W.e[l + 1]);
  LAUNCHCHK();
  if (type == MG_CYCLE_V) {
    ACHK(lin_cycle<T>(ctx, W, kap, o, l + 1, MG_CYCLE_V));
  } else if (type == MG_CYCLE_W) {
    ACHK(lin_cycle<T>(ctx, W, kap, o, l + 1, MG_CYCLE_W));
    ACHK(lin_cycle<T>(ctx, W, kap, o, l + 1, MG_CYCLE_W));
  } else {
    ACHK(lin_cycle<T>(ctx, W, kap, o, l + 1, MG_CYCLE_F));
    ACHK(lin_cycle<T>(ctx, W, kap, o, l + 1, MG_CYCLE_V));
  }
  if constexpr (sizeof(T) == 4) {
    if (cvec && fuse_prolong(ctx, l)) {
      with_lin_store<T>(ctx, W, l, [&](auto* D, auto* R) {
        using TD = std::remove_pointer_t<decltype(D)>;
        using TR = std::remove_pointer_t<decltype(R)>;
        const UpdLin<TD, TR> U{D, R, float(kh2), S0};
        launch_prolong_smooth0(ctx, l, (float*)W.e[l], (const float*)W.e[l + 1],
                               (const float*)nullptr, U);
      });
      LAUNCHCHK();
      smooth(o->nu_post, false, true);
      LAUNCHCHK();
      return MG_OK;
    }
  }
  if (cvec)
    launch_prolong<T, 1>(ctx, Lf, Lc, W.e[l], W.e[l + 1], (const T*)nullptr);
  else
    k_prolong_block<T><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(Lf, Lc, W.e[l], W.e[l + 1]);
  smooth(o->nu_post, false);
  LAUNCHCHK();
  return MG_OK;
}

template <int M>
int adjoint_impl(mg_ctx* ctx, const Consts& C, const mg_solver_opts* o, const float* delta,
                 const double* field, const double* grad_field, double* grad_delta, double tol,
                 mg_stats* st) {
  ACHK(ensure_adj(ctx, o->precision));
  WorkAdj& A = ctx->adj;
  const Lev& L0 = ctx->L[0];
  int64_t m = cells(L0);
  double sgn_field = (C.model == FR) ? -1.0 : 1.0;
  const bool f32 = o->precision == MG_FP32_REFINED;
  const bool vec = L0.nh % kVOuter == 0;
  int cur = 0, eb = 0;
  A.lam = A.lambuf[cur];
  if (A.have32) A.w32.e[0] = A.w32.ebuf[eb];
  if (A.have64) A.w64.e[0] = A.w64.ebuf[eb];
  // v, dg, b in one pass; b = s dL/dv, s = +1 (f(R)) / -1, and
  // dL/dv = sgn_field dL/dfield.  v is kept only where dL/d(delta) needs it.
  const bool nat8 = L0.n % 8 == 0 && al16(field, delta) && al16(grad_field, grad_delta);
  const unsigned nb_setup = nat8 ? nblk(m / 8) : nblk(m);
  if (nat8)
    k_lin_setup_nat8<M><<<nb_setup, kBlock, 0, ctx->stream>>>(
        L0, field, delta, grad_field, sgn_field, lin_sign(C) * sgn_field, C,
        M == FR ? (double*)nullptr : A.v, A.dg, f32 ? A.w32.dg[0] : (float*)nullptr, A.b,
        ctx->part);
  else
    k_lin_setup_nat<M><<<nb_setup, kBlock, 0, ctx->stream>>>(
        L0, field, delta, grad_field, sgn_field, lin_sign(C) * sgn_field, C,
        M == FR ? (double*)nullptr : A.v, A.dg, f32 ? A.w32.dg[0] : (float*)nullptr, A.b,
        ctx->part);
  LAUNCHCHK();
  double bb;
  ACHK(sum_to_host(ctx, nb_setup, &bb));
  bb = sqrt(bb);
  if (!(bb > 0.0)) bb = 1.0;
  // lam starts at 0: the fused outer kernels take it as 0 until written
  if (!vec) k_fill<double><<<nblk(m), kBlock, 0, ctx->stream>>>(A.lam, m, 0.0);
  // 16-bit dg and r on level 0 of an FP32 solve (as the forward solve's X and
  // rho; not for CQ): dg scaled so that its largest value maps to ~2^15
  struct A0Reset {  // level 0 is FP32 again outside this solve
    mg_ctx* c;
    ~A0Reset() {
      c->a0.on = false;
      c->a0.S = Store{1.0f, 1.0f, 1.0f, 1.0f};
    }
  } a0_reset{ctx};
  const bool f16 = f32 && ctx->fp16 && vec && L0.n % 8 == 0 && M != CQ;
  if (f32) {
    for (int l = 0; l + 1 < ctx->nlev; ++l)
      k_restrict<float, float><<<nblk(cells(ctx->L[l + 1])), kBlock, 0, ctx->stream>>>(
          ctx->L[l], ctx->L[l + 1], A.w32.dg[l], A.w32.dg[l + 1]);
    if (f16) {
      // at most nblk(m) <= part_cap partials
      const unsigned nb = std::min<unsigned>(kAbsmaxBlocks, nblk((m + 3) / 4));
      k_absmax_f32<<<nb, kBlock, 0, ctx->stream>>>(m, A.w32.dg[0], ctx->part4);
      ACHK(max_on_device(ctx, nb, ctx->part4, ctx->scal + 2));
      HIPCHK(hipMemcpyAsync(ctx->hscal + 2, ctx->scal + 2, sizeof(double), hipMemcpyDeviceToHost,
                            ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      const double dmax = ctx->hscal[2];
      const int dexp = dmax > 0.0 && std::isfinite(dmax) ? (int)floor(log2(3.2e4 / dmax)) : 0;
      ctx->a0.on = std::isfinite(dmax) && dexp > -120 && dexp < 120;
      ctx->a0.S.x_enc = float(ldexp(1.0, dexp));
      ctx->a0.S.x_dec = float(ldexp(1.0, -dexp));
      if (ctx->a0.on) {
        k_to_h16<<<nblk(m / 4), kBlock, 0, ctx->stream>>>(m / 4, A.w32.dg[0], A.w32.dg16,
                                                           ctx->a0.S.x_enc);
        LAUNCHCHK();
      }
    }
  } else {
    for (int l = 0; l + 1 < ctx->nlev; ++l)
      k_restrict<double, double><<<nblk(cells(ctx->L[l + 1])), kBlock, 0, ctx->stream>>>(
          ctx->L[l], ctx->L[l + 1], A.w64.dg[l], A.w64.dg[l + 1]);
  }
  LAUNCHCHK();
  double kap = lin_kap(C);
  int outer = 0, rc = MG_OK, vc = 0, k_prev = 0;
  double rel = 0.0, rel_prev = -1.0;
  const void* pending = nullptr;  // correction not yet added to lam
  // Coupled quintessence: the constant vector is nearly a null vector of A
  // (A 1 = dg, the tiny mass term), so rounding in the inner cycles leaves
  // an inaccurate uniform mode.  Each outer step therefore adds the FP64
  // Galerkin correction along 1, which zeroes sum(b - A lam) exactly:
  //   lam += e + c,  c = (sum r - sum dg e) / sum dg.
  const bool galerkin = C.model == CQ;
  double sum_dg = 0.0, shift = 0.0, sum_r = 0.0;
  if (galerkin) {
    k_dot<double><<<nblk(m), kBlock, 0, ctx->stream>>>(m, A.dg, (const double*)nullptr, ctx->part3);
    LAUNCHCHK();
    ACHK(sum_to_host(ctx, nblk(m), &sum_dg, ctx->part3));
  }
  double* psum = galerkin && sum_dg > 0.0 ? ctx->part3 : nullptr;
  // the first pre-smoothing sweep of each outer step takes the correction as
  // zero, so the fused outer kernel need not clear it
  // (only the vectorised level-0 smoother takes the uncleared buffer as zero)
  const bool fresh = vec && L0.nh % (f32 ? Vec<float>::V : Vec<double>::V) == 0 &&
                     o->nu_pre > 0 && ctx->fused_from > 0;
  for (;;) {
    int64_t nparts = vec ? march_blocks(L0, kMarchKT, kVOuter) : nblk(m);
    double s_pass = -1.0;  // sum r^2 when the 16-bit pass has reduced it already
    if (vec) {
      double* ln = pending ? A.lambuf[1 - cur] : A.lam;
      int ez = pending ? 1 - eb : eb;
      const double* lsrc = outer <= 1 ? nullptr : A.lam;  // null: lam = 0
      if (f32 && ctx->a0.on) {
        // r's scale: its RMS expected at this check mapped to 2^4 (b at the
        // start, 1/100 of the last check's after cycles); a pass whose
        // largest |r| would overflow is redone with the scale that allows
        const double rms_pred = (outer == 0 ? 1.0 : rel * 1e-2) * bb / sqrt(double(m));
        int rexp = (int)lround(log2(16.0 / (rms_pred > 0.0 ? rms_pred : 1.0)));
        for (int pass = 0;; ++pass) {
          rexp = rexp > 120 ? 120 : (rexp < -120 ? -120 : rexp);
          ctx->a0.S.r_enc = float(ldexp(1.0, rexp));
          ctx->a0.S.r_dec = float(ldexp(1.0, -rexp));
          k_lin_outer_fused_kv<float, h16><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
              L0, lsrc, (const float*)pending, ln, A.dg, A.b, kap, A.w32.r16,
              fresh ? (float*)nullptr : A.w32.ebuf[ez], ctx->part, shift, psum, kMarchKT,
              ctx->a0.S, ctx->part4);
          LAUNCHCHK();
          double mx = 0.0, s0 = 0.0, sb0 = 0.0;
          ACHK(outer_sums(ctx, nparts, false, true, &s0, &sb0, &mx));
          s_pass = s0;
          if (!(mx * ldexp(1.0, rexp) > 6.0e4) || pass > 0 || !std::isfinite(mx)) break;
          rexp = (int)floor(log2(3.0e4 / mx));
        }
      } else if (f32)
        k_lin_outer_fused_kv<float><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
            L0, lsrc, (const float*)pending, ln, A.dg, A.b, kap, A.w32.r[0],
            fresh ? (float*)nullptr : A.w32.ebuf[ez], ctx->part, shift, psum, kMarchKT);
      else
        k_lin_outer_fused_kv<double><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
            L0, lsrc, (const double*)pending, ln, A.dg, A.b, kap, A.w64.r[0],
            fresh ? (double*)nullptr : A.w64.ebuf[ez], ctx->part, shift, psum, kMarchKT);
      if (pending) {
        cur = 1 - cur;
        eb = 1 - eb;
        A.lam = A.lambuf[cur];
        if (f32) A.w32.e[0] = A.w32.ebuf[eb];
        else A.w64.e[0] = A.w64.ebuf[eb];
        pending = nullptr;
      }
    } else {
      if (shift != 0.0) k_add_const<<<nblk(m), kBlock, 0, ctx->stream>>>(m, A.lam, shift);
      if (f32)
        k_lin_outer<float><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
            L0, A.lam, A.dg, A.b, kap, A.w32.r[0], A.w32.e[0], ctx->part, psum);
      else
        k_lin_outer<double><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
            L0, A.lam, A.dg, A.b, kap, A.w64.r[0], A.w64.e[0], ctx->part, psum);
    }
    shift = 0.0;
    LAUNCHCHK();
    double s = s_pass;
    if (psum) ACHK(sum_to_host(ctx, nparts, &sum_r, psum));
    if (s < 0.0) ACHK(sum_to_host(ctx, nparts, &s));
    rel = sqrt(s) / bb;
    if (outer > 0 && st && outer - 1 < 64) st->resid_hist[outer - 1] = rel;
    if (!std::isfinite(rel)) {
      rc = fail(ctx, MG_ENAN, "non-finite adjoint residual");
      break;
    }
    if (rel <= tol) break;
    if (outer >= o->max_cycles) {
      rc = fail(ctx, MG_ENOCONV, "max_cycles reached (adjoint)");
      break;
    }
    // correction scheme on r = b - A lam (FP32 or FP64 inner cycles)
    int k = plan_cycles(o->inner_cycles, rel, rel_prev, k_prev, tol, cells(ctx->L[0]),
                        ctx->a0.on ? kStore16Step : 0.0, ctx->a0.on ? 4 : 2);
    if (f32) {
      for (int it = 0; it < k; ++it)
        ACHK(lin_cycle<float>(ctx, A.w32, kap, o, 0, o->cycle, fresh && it == 0));
      if (psum) k_dot<float><<<nblk(m), kBlock, 0, ctx->stream>>>(m, A.w32.e[0], A.dg, ctx->part3);
      if (vec) pending = A.w32.e[0];
      else k_axpy_to64<float><<<nblk(m), kBlock, 0, ctx->stream>>>(m, A.lam, A.w32.e[0]);
    } else {
      for (int it = 0; it < k; ++it)
        ACHK(lin_cycle<double>(ctx, A.w64, kap, o, 0, o->cycle, fresh && it == 0));
      if (psum) k_dot<double><<<nblk(m), kBlock, 0, ctx->stream>>>(m, A.w64.e[0], A.dg, ctx->part3);
      if (vec) pending = A.w64.e[0];
      else k_axpy_to64<double><<<nblk(m), kBlock, 0, ctx->stream>>>(m, A.lam, A.w64.e[0]);
    }
    if (psum) {
      double dge;
      LAUNCHCHK();
      ACHK(sum_to_host(ctx, nblk(m), &dge, ctx->part3));
      shift = (sum_r - dge) / sum_dg;
    }
    vc += k;
    rel_prev = rel;
    k_prev = k;
    LAUNCHCHK();
    ++outer;
  }
  if (vec && outer == 0) k_fill<double><<<nblk(m), kBlock, 0, ctx->stream>>>(A.lam, m, 0.0);
  if (nat8)
    k_lin_final8<M><<<nblk(m / 8), kBlock, 0, ctx->stream>>>(L0, A.v, A.lam, C, grad_delta);
  else
    k_lin_final<M><<<nblk(m), kBlock, 0, ctx->stream>>>(L0, A.v, A.lam, C, grad_delta);
  LAUNCHCHK();
  if (st) {
    st->cycles = outer;
    st->vcycles = vc;
    st->rel_resid = rel;
  }
  return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// natural-layout kernels: force, its transpose, loss, CIC
// ---------------------------------------------------------------------------
namespace {

// Phi5 of the field value (ABI convention: f(R) field = f_R = -w).  The
// products are rounded explicitly: a multiply fused into the difference of
// two potentials would make equal field values give a non-zero force.
__device__ __forceinline__ double phi5_of(const Consts& C, double f) {
  if (C.model == FR) return -__dmul_rn(C.phi5, f);
  if (C.model == SYM) return __dmul_rn(__dmul_rn(C.phi5, f), f);
  return __dmul_rn(C.phi5, f);
}
__device__ __forceinline__ double dphi5_of(const Consts& C, double f) {
  if (C.model == FR) return -C.phi5;
  if (C.model == SYM) return 2.0 * C.phi5 * f;
  return C.phi5;
}

// Phi5 of the field plus, when ADD, a second potential (the Newtonian one)
template <bool ADD>
__device__ __forceinline__ double pot_at(const Consts& C, const double* __restrict__ f,
                                         const double* __restrict__ pn, double sn, int64_t c) {
  const double v = phi5_of(C, f[c]);
  return ADD ? __dadd_rn(v, __dmul_rn(sn, pn[c])) : v;
}

template <bool ADD>
__global__ __launch_bounds__(kBlock) void k_force(Lev L, const double* __restrict__ f,
                                                  const double* __restrict__ pn, double sn,
                                                  Consts C, float* __restrict__ out) {
  int64_t g = gid();
  const int n = L.n;
  int64_t m = 2 * L.half;
  if (g >= m) return;
  int i, j, k;
  dec_nat(g, L, i, j, k);
  int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
  int jp = j + 1 == n ? 0 : j + 1, jm = j == 0 ? n - 1 : j - 1;
  int kp = k + 1 == n ? 0 : k + 1, km = k == 0 ? n - 1 : k - 1;
  int64_t row = (int64_t)k * n + j;
  double gx = -0.5 * (pot_at<ADD>(C, f, pn, sn, row * n + ip) - pot_at<ADD>(C, f, pn, sn, row * n + im));
  double gy = -0.5 * (pot_at<ADD>(C, f, pn, sn, ((int64_t)k * n + jp) * n + i) -
                      pot_at<ADD>(C, f, pn, sn, ((int64_t)k * n + jm) * n + i));
  double gz = -0.5 * (pot_at<ADD>(C, f, pn, sn, ((int64_t)kp * n + j) * n + i) -
                      pot_at<ADD>(C, f, pn, sn, ((int64_t)km * n + j) * n + i));
  out[g] = float(gx);
  out[m + g] = float(gy);
  out[2 * m + g] = float(gz);
}

// The same force with a march in z: a thread owns 4 consecutive cells of a
// row and walks kMarchKT planes, keeping Phi5 of planes k-1, k, k+1 in
// registers (the field is read from HBM once); rows j +- 1 and the row's
// edge cells come from L1/L2.  Requires n % 4 == 0.
template <bool ADD>
__global__ __launch_bounds__(kBlock) void k_force_kv(Lev L, const double* __restrict__ f,
                                                     const double* __restrict__ pn, double sn,
                                                     Consts C, float* __restrict__ out, int kt) {
  constexpr int V = 4;
  const int n = L.n;
  const uint32_t ngrp = (uint32_t)n * (uint32_t)n / V;  // groups per plane
  const uint32_t nchunk = (ngrp + kBlock - 1) / kBlock;
  const uint32_t b = (uint32_t)xcd_block();
  const uint32_t kb = b / nchunk, chunk = b - kb * nchunk;
  const uint32_t grp = chunk * kBlock + threadIdx.x;
  const int k0 = (int)kb * kt;
  if (grp >= ngrp || k0 >= n) return;
  const uint32_t p = grp * V;
  const uint32_t jj = L.dn.div(p);
  const int j = (int)jj, i0 = (int)(p - jj * (uint32_t)n);
  const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
  const int im = i0 == 0 ? n - 1 : i0 - 1, ip = i0 + V == n ? 0 : i0 + V;
  const int k1 = k0 + kt < n ? k0 + kt : n;
  const int64_t m = 2 * L.half;
  auto row = [&](int jr, int kr) { return ((int64_t)kr * n + jr) * n; };
  auto ld = [&](int jr, int kr, double* ph) {
    double v[V];
    ldn<double, V>(f + row(jr, kr) + i0, v);
#pragma unroll
    for (int q = 0; q < V; ++q) ph[q] = phi5_of(C, v[q]);
    if (ADD) {
      ldn<double, V>(pn + row(jr, kr) + i0, v);
#pragma unroll
      for (int q = 0; q < V; ++q) ph[q] = __dadd_rn(ph[q], __dmul_rn(sn, v[q]));
    }
  };
  double win[3][V];
  ld(j, k0 == 0 ? n - 1 : k0 - 1, win[0]);
  ld(j, k0, win[1]);
  for (int k = k0; k < k1; ++k) {
    ld(j, k + 1 == n ? 0 : k + 1, win[2]);
    double ym[V], yp[V], xv[V + 2];
    ld(jm, k, ym);
    ld(jp, k, yp);
    const int64_t r = row(j, k);
    xv[0] = pot_at<ADD>(C, f, pn, sn, r + im);
    xv[V + 1] = pot_at<ADD>(C, f, pn, sn, r + ip);
#pragma unroll
    for (int q = 0; q < V; ++q) xv[q + 1] = win[1][q];
    float gx[V], gy[V], gz[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      gx[q] = float(-0.5 * (xv[q + 2] - xv[q]));
      gy[q] = float(-0.5 * (yp[q] - ym[q]));
      gz[q] = float(-0.5 * (win[2][q] - win[0][q]));
    }
    stn_nt<float, V>(out + r + i0, gx);
    stn_nt<float, V>(out + m + r + i0, gy);
    stn_nt<float, V>(out + 2 * m + r + i0, gz);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      win[0][q] = win[1][q];
      win[1][q] = win[2][q];
    }
  }
}
// The same force on tiles of 64 x 16 cells of a plane (16 threads x 4 cells
// per row, 16 rows), marching kt planes in z.  Plane k's values go through
// LDS, so the y neighbours (and the x neighbours inside the tile) come from
// other threads; only the tile's two edge rows and its x-edge cells are read
// again from memory.  Same arithmetic as k_force_kv, so the same bits.
constexpr int kFTX = 16, kFTY = 16;  // threads per row, rows per tile
template <bool ADD>
__global__ __launch_bounds__(kBlock) void k_force_tile(Lev L, const double* __restrict__ f,
                                                       const double* __restrict__ pn, double sn,
                                                       Consts C, float* __restrict__ out, int kt) {
  constexpr int V = 4, W = kFTX * V;
  __shared__ double sp[2][kFTY + 2][W];
  const int n = L.n;
  const uint32_t ntx = (uint32_t)(n / W), tiles = ntx * (uint32_t)(n / kFTY);
  const uint32_t b = (uint32_t)xcd_block();
  const uint32_t kb = b / tiles, tile = b - kb * tiles;
  const uint32_t ty0 = tile / ntx, tx0 = tile - ty0 * ntx;
  const int tx = (int)threadIdx.x % kFTX, ty = (int)threadIdx.x / kFTX;
  const int i0 = (int)tx0 * W + tx * V, j = (int)ty0 * kFTY + ty;
  const int k0 = (int)kb * kt;
  if (k0 >= n) return;  // the whole workgroup
  const int k1 = k0 + kt < n ? k0 + kt : n;
  const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
  const int im = i0 == 0 ? n - 1 : i0 - 1, ip = i0 + V == n ? 0 : i0 + V;
  const int64_t m = 2 * L.half;
  auto row = [&](int jr, int kr) { return ((int64_t)kr * n + jr) * n; };
  auto ld = [&](int jr, int kr, double* ph) {
    double v[V];
    ldn<double, V>(f + row(jr, kr) + i0, v);
#pragma unroll
    for (int q = 0; q < V; ++q) ph[q] = phi5_of(C, v[q]);
    if (ADD) {
      ldn<double, V>(pn + row(jr, kr) + i0, v);
#pragma unroll
      for (int q = 0; q < V; ++q) ph[q] = __dadd_rn(ph[q], __dmul_rn(sn, v[q]));
    }
  };
  double win[3][V];
  ld(j, k0 == 0 ? n - 1 : k0 - 1, win[0]);
  ld(j, k0, win[1]);
  int buf = 0;
  for (int k = k0; k < k1; ++k, buf ^= 1) {
    ld(j, k + 1 == n ? 0 : k + 1, win[2]);
    double(*s)[W] = sp[buf];
#pragma unroll
    for (int q = 0; q < V; ++q) s[ty + 1][tx * V + q] = win[1][q];
    if (ty == 0 || ty == kFTY - 1) {
      double h[V];
      ld(ty == 0 ? jm : jp, k, h);
#pragma unroll
      for (int q = 0; q < V; ++q) s[ty == 0 ? 0 : kFTY + 1][tx * V + q] = h[q];
    }
    // double-buffered: a buffer is rewritten only after the next barrier
    __syncthreads();
    const int64_t r = row(j, k);
    double ym[V], yp[V], xv[V + 2];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      ym[q] = s[ty][tx * V + q];
      yp[q] = s[ty + 2][tx * V + q];
      xv[q + 1] = win[1][q];
    }
    xv[0] = tx > 0 ? s[ty + 1][tx * V - 1] : pot_at<ADD>(C, f, pn, sn, r + im);
    xv[V + 1] = tx < kFTX - 1 ? s[ty + 1][tx * V + V] : pot_at<ADD>(C, f, pn, sn, r + ip);
    float gx[V], gy[V], gz[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      gx[q] = float(-0.5 * (xv[q + 2] - xv[q]));
      gy[q] = float(-0.5 * (yp[q] - ym[q]));
      gz[q] = float(-0.5 * (win[2][q] - win[0][q]));
    }
    stn_nt<float, V>(out + r + i0, gx);
    stn_nt<float, V>(out + m + r + i0, gy);
    stn_nt<float, V>(out + 2 * m + r + i0, gz);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      win[0][q] = win[1][q];
      win[1][q] = win[2][q];
    }
  }
}
__global__ __launch_bounds__(kBlock) void k_force_adjoint(Lev L, const double* __restrict__ f,
                                                          const float* __restrict__ gf, Consts C,
                                                          double* __restrict__ out) {
  int64_t g = gid();
  const int n = L.n;
  int64_t m = 2 * L.half;
  if (g >= m) return;
  int i, j, k;
  dec_nat(g, L, i, j, k);
  int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
  int jp = j + 1 == n ? 0 : j + 1, jm = j == 0 ? n - 1 : j - 1;
  int kp = k + 1 == n ? 0 : k + 1, km = k == 0 ? n - 1 : k - 1;
  int64_t row = (int64_t)k * n + j;
  // g_a(c) = -(Phi(c+e_a) - Phi(c-e_a))/2  =>  dL/dPhi(c) = sum_a (G_a(c+e_a) - G_a(c-e_a))/2
  double s = (double(gf[row * n + ip]) - double(gf[row * n + im])) +
             (double(gf[m + ((int64_t)k * n + jp) * n + i]) - double(gf[m + ((int64_t)k * n + jm) * n + i])) +
             (double(gf[2 * m + ((int64_t)kp * n + j) * n + i]) -
              double(gf[2 * m + ((int64_t)km * n + j) * n + i]));
  out[g] = 0.5 * s * dphi5_of(C, f[g]);
}

// Transpose of the fifth-force gradient on the force kernel's 64 x 16 tiles,
// marching kt planes in z: the x component's x neighbours and the y
// component's rows j +- 1 come from LDS, the z component's planes k +- 1 from
// a register window.  Same arithmetic, in the same order, as k_force_adjoint.
__global__ __launch_bounds__(kBlock) void k_force_adjoint_tile(
    Lev L, const double* __restrict__ f, const float* __restrict__ gf, Consts C,
    double* __restrict__ out, int kt) {
  constexpr int V = 4, W = kFTX * V;
  __shared__ float sx[2][kFTY][W];
  __shared__ float sy[2][kFTY + 2][W];
  const int n = L.n;
  const uint32_t ntx = (uint32_t)(n / W), tiles = ntx * (uint32_t)(n / kFTY);
  const uint32_t b = (uint32_t)xcd_block();
  const uint32_t kb = b / tiles, tile = b - kb * tiles;
  const uint32_t ty0 = tile / ntx, tx0 = tile - ty0 * ntx;
  const int tx = (int)threadIdx.x % kFTX, ty = (int)threadIdx.x / kFTX;
  const int i0 = (int)tx0 * W + tx * V, j = (int)ty0 * kFTY + ty;
  const int k0 = (int)kb * kt;
  if (k0 >= n) return;  // the whole workgroup
  const int k1 = k0 + kt < n ? k0 + kt : n;
  const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
  const int im = i0 == 0 ? n - 1 : i0 - 1, ip = i0 + V == n ? 0 : i0 + V;
  const int64_t m = 2 * L.half;
  const float* gx = gf;
  const float* gy = gf + m;
  const float* gz = gf + 2 * m;
  auto row = [&](int jr, int kr) { return ((int64_t)kr * n + jr) * n; };
  float zw[3][V];
  ldn<float, V>(gz + row(j, k0 == 0 ? n - 1 : k0 - 1) + i0, zw[0]);
  ldn<float, V>(gz + row(j, k0) + i0, zw[1]);
  int buf = 0;
  for (int k = k0; k < k1; ++k, buf ^= 1) {
    const int64_t r = row(j, k);
    ldn<float, V>(gz + row(j, k + 1 == n ? 0 : k + 1) + i0, zw[2]);
    float xc[V], yc[V];
    ldn<float, V>(gx + r + i0, xc);
    ldn<float, V>(gy + r + i0, yc);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      sx[buf][ty][tx * V + q] = xc[q];
      sy[buf][ty + 1][tx * V + q] = yc[q];
    }
    if (ty == 0 || ty == kFTY - 1) {
      float h[V];
      ldn<float, V>(gy + row(ty == 0 ? jm : jp, k) + i0, h);
#pragma unroll
      for (int q = 0; q < V; ++q) sy[buf][ty == 0 ? 0 : kFTY + 1][tx * V + q] = h[q];
    }
    double fv[V] = {0.0, 0.0, 0.0, 0.0};
    if (C.model != FR) ldn<double, V>(f + r + i0, fv);
    // double-buffered: a buffer is rewritten only after the next barrier
    __syncthreads();
    const float xl = tx > 0 ? sx[buf][ty][tx * V - 1] : gx[r + im];
    const float xr = tx < kFTX - 1 ? sx[buf][ty][tx * V + V] : gx[r + ip];
    double o[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const float xm = q == 0 ? xl : xc[q - 1], xp = q == V - 1 ? xr : xc[q + 1];
      const double s = (double(xp) - double(xm)) +
                       (double(sy[buf][ty + 2][tx * V + q]) - double(sy[buf][ty][tx * V + q])) +
                       (double(zw[2][q]) - double(zw[0][q]));
      o[q] = 0.5 * s * dphi5_of(C, fv[q]);
    }
    stn_nt<double, V>(out + r + i0, o);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      zw[0][q] = zw[1][q];
      zw[1][q] = zw[2][q];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_loss_sq(int64_t m, const float* __restrict__ force,
                                                    const int64_t* __restrict__ cellsv,
                                                    int64_t ncell, float* __restrict__ grad,
                                                    double* part) {
  __shared__ double sh[32];
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (q < ncell) {
    int64_t c = cellsv[q];
    if (c >= 0 && c < m) {
      for (int a = 0; a < 3; ++a) {
        float v = force[a * m + c];
        acc += double(v) * double(v);
        grad[a * m + c] = 2.0f * v;
      }
    }
  }
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

struct CicCell {
  int i0[3];
  double t[3];
};
// lower CIC cell and fractional offsets of one particle
__device__ __forceinline__ CicCell cic_cell(int n, const float* __restrict__ pos, int64_t p) {
  CicCell c;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // For 1 <= x < 2^22, s = x - 1/2, floor(s) and s - floor(s) are exact in
    // FP32 (0.5 is a multiple of ulp(x); s - floor(s) by Sterbenz); other
    // positions take the same three steps in FP64, where they are exact for
    // any float.  Both give the same i0 and the same t.
    const float xf = pos[3 * p + a];
    int q;
    if (xf >= 1.0f && xf < 4194304.0f) {
      const float sf = xf - 0.5f;
      const float fl = floorf(sf);
      c.t[a] = double(sf - fl);
      q = (int)fl;
    } else {
      const double s = double(xf) - 0.5;
      const double fl = floor(s);
      c.t[a] = s - fl;
      q = (int)fl;
    }
    if (q < 0 || q >= n) {  // periodic wrap; only q = -1 for positions in [0, n)
      q %= n;
      if (q < 0) q += n;
    }
    c.i0[a] = q;
  }
  return c;
}
// 8 fixed-point weights (units of 2^-32) summing to exactly 2^32, corner q:
// dx = q&1, dy = (q>>1)&1, dz = q>>2, axis weights (1 - t, t).  The corner
// whose axis weights are all the larger ones ("big", >= 1/8) takes 2^32
// minus the other seven; each of those is (wx wy) (wz 2^32), the first
// product rounded to FP64 and the second rounded once, to the nearest
// integer (ties to even), by a fused multiply-add with 2^52: the result lies
// in [2^52, 2^53), where the spacing of doubles is 1, so its low 32 mantissa
// bits are the weight (at most 2^31: one factor is <= 1/2).  The explicit
// fused multiply-add gives every kernel the same rounding.  No weight is
// negative.
__device__ __forceinline__ void cic_weights(const CicCell& c, long long* w) {
  const double wx[2] = {1.0 - c.t[0], c.t[0]};
  const double wy[2] = {1.0 - c.t[1], c.t[1]};
  const double wz[2] = {(1.0 - c.t[2]) * 4294967296.0, c.t[2] * 4294967296.0};
  const int big = (c.t[0] > 0.5 ? 1 : 0) | (c.t[1] > 0.5 ? 2 : 0) | (c.t[2] > 0.5 ? 4 : 0);
  long long tot = 0;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const double xy = __dmul_rn(wx[dx], wy[dy]);
#pragma unroll
      for (int dz = 0; dz < 2; ++dz) {
        const int q = dx | (dy << 1) | (dz << 2);
        const double r = __fma_rn(xy, wz[dz], 4503599627370496.0);  // + 2^52
        w[q] = q == big ? 0ll : (long long)(uint32_t)__double_as_longlong(r);
        tot += w[q];
      }
    }
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (q == big) w[q] = (1ll << 32) - tot;
}
// CIC: per axis, s = x - 1/2, i0 = floor(s), t = s - i0 (formed in FP64, so
// exact for every float position); weights (1-t, t) to cells i0, i0+1
// (periodic), deposited as 32.32 fixed point (cic_weights).
__global__ __launch_bounds__(kBlock) void k_cic(int n, int64_t np, const float* __restrict__ pos,
                                                unsigned long long* __restrict__ acc) {
  int64_t p = gid();
  if (p >= np) return;
  const CicCell c = cic_cell(n, pos, p);
  const int* i0 = c.i0;
  long long w[8];
  cic_weights(c, w);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (w[q] == 0) continue;
    int di = q & 1, dj = (q >> 1) & 1, dk = (q >> 2) & 1;
    int ii = i0[0] + di == n ? 0 : i0[0] + di;
    int jj = i0[1] + dj == n ? 0 : i0[1] + dj;
    int kk = i0[2] + dk == n ? 0 : i0[2] + dk;
    atomicAdd(&acc[((int64_t)kk * n + jj) * n + ii], (unsigned long long)w[q]);
  }
}
__global__ __launch_bounds__(kBlock) void k_cic_finish(int64_t m, const unsigned long long* acc,
                                                       double scale, float* delta) {
  int64_t g = gid();
  if (g < m) delta[g] = float(double(acc[g]) * scale - 1.0);
}

// ---- binned CIC: tiles of kT^3 cells ------------------------------------
// Particles are sorted by bin = (tile, class).  Bit a of the class is set when
// the particle's lower cell is the last layer of its tile along axis a, so
// that the particle also reaches the next tile along a.  The workgroup of a
// tile deposits its own particles and the reaching classes of its 7 lower
// neighbours, so it holds every contribution to its kT^3 cells and writes δ
// directly.  Sums are 32.32 fixed point: exact, in any order.
constexpr int kT = 16;  // tile edge (cells)
constexpr int kT3 = kT * kT * kT;

__device__ __forceinline__ uint32_t bin_of(const CicCell& c, int nt) {
  const uint32_t t =
      ((uint32_t)(c.i0[2] / kT) * nt + (uint32_t)(c.i0[1] / kT)) * nt + (uint32_t)(c.i0[0] / kT);
  const uint32_t cls = (c.i0[0] % kT == kT - 1 ? 1u : 0u) | (c.i0[1] % kT == kT - 1 ? 2u : 0u) |
                       (c.i0[2] % kT == kT - 1 ? 4u : 0u);
  return 8u * t + cls;
}

// Wave-level runs of equal bins: consecutive lanes (consecutive particles)
// whose particles fall in the same bin.
struct CicRun {
  int leader;    // lane of the run's first particle
  uint32_t len;  // run length (on the leader)
  bool lead;
};
__device__ __forceinline__ CicRun cic_run(uint32_t t, bool valid) {
  const int lane = threadIdx.x & 63;
  const uint32_t prev = __shfl_up(t, 1, 64);
  const bool leader = !valid || lane == 0 || prev != t;
  const unsigned long long lead = __ballot(leader);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  CicRun r;
  r.leader = 63 - __clzll(lead & upto);
  const unsigned long long above = lead & ~upto;
  const int run_end = above ? (__ffsll((long long)above) - 1) : 64;
  r.len = (uint32_t)(run_end - lane);
  r.lead = valid && leader;
  return r;
}

// The count and placement passes take a region of kCicRegion consecutive
// particles per workgroup, kCicRounds rounds of kCicPer groups of kCicCB
// consecutive particles (a wave's 64 lanes hold 64 consecutive particles);
// all loads of a round are issued before their results are used.
constexpr int kCicCB = 512;    // workgroup size of the count and placement passes
constexpr int kCicPer = 4;
constexpr int kCicRounds = 4;
constexpr int kCicRegion = kCicCB * kCicPer * kCicRounds;  // particles (and at most runs)
constexpr int kCicBinBits = 26;  // run record: bin | (length - 1) << 26
// Per-workgroup LDS table bin -> count (open addressing, linear probing):
// the global counters and cursors take one atomic per distinct bin of a
// region instead of one per run.  A bin whose probe window is full is
// counted or placed with its own global atomics (consistent: no entry is
// ever removed, so a bin is either in its window or never inserted).
constexpr int kCicH = 4096;
constexpr int kCicProbe = 32;
constexpr uint32_t kCicEmpty = 0xffffffffu;
__device__ __forceinline__ uint32_t cic_hash(uint32_t bin) {
  return (bin * 2654435761u) >> (32 - 12);
}
// slot of bin in the table, inserting it if absent; -1 if its window is full
__device__ __forceinline__ int cic_insert(uint32_t* key, uint32_t bin) {
  uint32_t h = cic_hash(bin);
  for (int k = 0; k < kCicProbe; ++k) {
    const uint32_t old = atomicCAS(&key[h], kCicEmpty, bin);
    if (old == kCicEmpty || old == bin) return (int)h;
    h = (h + 1) & (kCicH - 1);
  }
  return -1;
}
// slot of bin in the finished table; -1 if it was never inserted
__device__ __forceinline__ int cic_find(const uint32_t* key, uint32_t bin) {
  uint32_t h = cic_hash(bin);
  for (int k = 0; k < kCicProbe; ++k) {
    const uint32_t v = key[h];
    if (v == bin) return (int)h;
    if (v == kCicEmpty) return -1;
    h = (h + 1) & (kCicH - 1);
  }
  return -1;
}
struct CicChunk {
  float x[kCicPer][3];
  uint32_t bin[kCicPer];
  bool valid[kCicPer];
};
// particle first + q kCicCB + threadIdx.x for q < kCicPer
__device__ __forceinline__ void cic_chunk(int n, int nt, int64_t np, const float* __restrict__ pos,
                                          int64_t first, CicChunk& c) {
#pragma unroll
  for (int q = 0; q < kCicPer; ++q) {
    const int64_t p = first + (int64_t)q * kCicCB + threadIdx.x;
    c.valid[q] = p < np;
#pragma unroll
    for (int a = 0; a < 3; ++a) c.x[q][a] = c.valid[q] ? pos[3 * p + a] : 0.f;
  }
#pragma unroll
  for (int q = 0; q < kCicPer; ++q)
    c.bin[q] = c.valid[q] ? bin_of(cic_cell(n, c.x[q], 0), nt) : 0xffffffffu;
}

// Count pass: each run of equal bins becomes one record {first particle,
// bin | (length - 1) << 26}, written compacted into the workgroup's own
// region (no global counter), with the region's record count in nrec;
// cnt[bin] counts runs.  Particles in a spatially coherent order (a
// Lagrangian grid order) give runs of several particles, so the records are
// a small fraction of the positions' bytes; a random order degrades to one
// record per particle and stays correct.
__global__ __launch_bounds__(kCicCB) void k_cic_runs(int n, int nt, int64_t np,
                                                     const float* __restrict__ pos, uint32_t* cnt,
                                                     uint2* __restrict__ rec,
                                                     uint32_t* __restrict__ nrec) {
  constexpr int kW = kCicCB / 64;
  __shared__ uint32_t key[kCicH], val[kCicH];
  __shared__ uint32_t wcount[kCicPer * kW], woff[kCicPer * kW];
  static_assert(kCicPer * kW <= 64, "one wave scans the per-(group, wave) run counts");
  for (int h = threadIdx.x; h < kCicH; h += kCicCB) {
    key[h] = kCicEmpty;
    val[h] = 0u;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint2* R = rec + (int64_t)blockIdx.x * kCicRegion;
  uint32_t rbase = 0;  // records written by the earlier rounds (same on every thread)
  for (int round = 0; round < kCicRounds; ++round) {
    const int64_t first = (int64_t)blockIdx.x * kCicRegion + (int64_t)round * kCicCB * kCicPer;
    CicChunk c;
    cic_chunk(n, nt, np, pos, first, c);
    CicRun r[kCicPer];
    uint32_t rank[kCicPer];
#pragma unroll
    for (int q = 0; q < kCicPer; ++q) {
      r[q] = cic_run(c.bin[q], c.valid[q]);
      const unsigned long long m = __ballot(r[q].lead);
      rank[q] = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wcount[q * kW + wv] = (uint32_t)__popcll(m);
      if (r[q].lead) {
        const int h = cic_insert(key, c.bin[q]);
        if (h >= 0) atomicAdd(&val[h], 1u);
        else atomicAdd(cnt + c.bin[q], 1u);
      }
    }
    __syncthreads();
    if (wv == 0) {  // exclusive scan of the counts in (group, wave) order
      const uint32_t v = lane < kCicPer * kW ? wcount[lane] : 0u;
      uint32_t inc = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
      }
      if (lane < kCicPer * kW) woff[lane] = inc - v;
    }
    __syncthreads();
    const uint32_t total = woff[kCicPer * kW - 1] + wcount[kCicPer * kW - 1];
#pragma unroll
    for (int q = 0; q < kCicPer; ++q)
      if (r[q].lead)
        R[rbase + woff[q * kW + wv] + rank[q]] =
            make_uint2((uint32_t)(first + (int64_t)q * kCicCB + threadIdx.x),
                       c.bin[q] | ((r[q].len - 1u) << kCicBinBits));
    rbase += total;
    __syncthreads();  // wcount and woff are rewritten by the next round; the table is complete after the last
  }
  for (int h = threadIdx.x; h < kCicH; h += kCicCB)
    if (key[h] != kCicEmpty) atomicAdd(cnt + key[h], val[h]);
  if (threadIdx.x == 0) nrec[blockIdx.x] = rbase;
}
// Exclusive scan of the bin counts (8 per tile, a tile's bins contiguous) in
// one block, 1024 tiles per round: bin offsets and placement cursors.
__global__ __launch_bounds__(1024) void k_cic_scan(const uint32_t* __restrict__ cnt,
                                                   int64_t ntiles, uint32_t* __restrict__ boff,
                                                   uint32_t* __restrict__ cur) {
  __shared__ uint32_t wsum[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint4* c4 = reinterpret_cast<const uint4*>(cnt);
  uint4* b4 = reinterpret_cast<uint4*>(boff);
  uint4* u4 = reinterpret_cast<uint4*>(cur);
  uint32_t carry = 0;
  for (int64_t r0 = 0; r0 < ntiles; r0 += 1024) {
    const int64_t q = r0 + threadIdx.x;
    uint4 u = make_uint4(0u, 0u, 0u, 0u), v = u;
    if (q < ntiles) {
      u = c4[2 * q];
      v = c4[2 * q + 1];
    }
    const uint32_t tot = u.x + u.y + u.z + u.w + v.x + v.y + v.z + v.w;
    uint32_t inc = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    uint32_t wpre = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const uint32_t sw = wsum[w];
      wpre += w < wv ? sw : 0u;
      all += sw;
    }
    if (q < ntiles) {
      const uint32_t e0 = carry + wpre + inc - tot;
      const uint4 o0 = make_uint4(e0, e0 + u.x, e0 + u.x + u.y, e0 + u.x + u.y + u.z);
      const uint32_t e1 = o0.w + u.w;
      const uint4 o1 = make_uint4(e1, e1 + v.x, e1 + v.x + v.y, e1 + v.x + v.y + v.z);
      b4[2 * q] = o0;
      b4[2 * q + 1] = o1;
      u4[2 * q] = o0;
      u4[2 * q + 1] = o1;
    }
    carry += all;
    __syncthreads();  // wsum is rewritten by the next round
  }
}
// Placement: each record goes to the next slot of its bin, as the word
// first particle << 6 | (length - 1).  One workgroup per count region: the
// region's runs of one bin take consecutive slots, reserved with one global
// atomic per distinct bin (the table of the count pass, rebuilt).
__global__ __launch_bounds__(kCicCB) void k_cic_place(const uint2* __restrict__ rec,
                                                      const uint32_t* __restrict__ nrec,
                                                      uint32_t* cur,
                                                      unsigned long long* __restrict__ runs) {
  __shared__ uint32_t key[kCicH], val[kCicH], base[kCicH];
  for (int h = threadIdx.x; h < kCicH; h += kCicCB) {
    key[h] = kCicEmpty;
    val[h] = 0u;
  }
  __syncthreads();
  const uint32_t nr = nrec[blockIdx.x];
  const uint2* R = rec + (int64_t)blockIdx.x * kCicRegion;
  for (uint32_t i = threadIdx.x; i < nr; i += kCicCB) {
    const int h = cic_insert(key, R[i].y & ((1u << kCicBinBits) - 1u));
    if (h >= 0) atomicAdd(&val[h], 1u);
  }
  __syncthreads();
  for (int h = threadIdx.x; h < kCicH; h += kCicCB)
    if (key[h] != kCicEmpty) {
      base[h] = atomicAdd(cur + key[h], val[h]);
      val[h] = 0u;
    }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nr; i += kCicCB) {
    const uint2 v = R[i];
    const uint32_t bin = v.y & ((1u << kCicBinBits) - 1u);
    const int h = cic_find(key, bin);
    const uint32_t slot = h >= 0 ? base[h] + atomicAdd(&val[h], 1u) : atomicAdd(cur + bin, 1u);
    runs[slot] = ((unsigned long long)v.x << 6) | (unsigned long long)(v.y >> kCicBinBits);
  }
}
// One workgroup per tile.  Segments: the tile's own 8 bins (one contiguous
// range of runs, role 0) and, for each lower neighbour at offset -s (s a
// non-empty subset of the axes, role s), its bins whose class contains s.
// In role s a particle's local coordinate on axis a is its in-tile layer
// minus kT s_a, and only corners that land inside the tile are added: each
// corner of each particle lands in exactly one (tile, role).  Runs are taken
// in batches of at most kCicTB runs and kCicCap particles: their lengths
// are prefix-summed, the batch's particles numbered consecutively, and a
// bitmap of run starts (with per-word prefix counts) maps a particle number
// to its run in one LDS read, so that consecutive threads read consecutive
// particles of a run.  The LDS footprint (under 40 KB) leaves room for four
// workgroups per CU.  Workgroups of one XCD (every 8th workgroup id) take a
// contiguous range of tiles, so tiles that share position cache lines run
// on the same L2.
constexpr int kCicSegs = 20;  // 1 + 4 + 4 + 2 + 4 + 2 + 2 + 1
constexpr int kCicUnroll = 2;  // particles per thread in flight
constexpr int kCicTB = 512;    // workgroup size of the tile kernel
constexpr int kCicWords = kCicTB;          // bitmap words, one per thread
constexpr int kCicCap = 32 * kCicWords;    // particles per batch (a run is at most 64)
__global__ __launch_bounds__(kCicTB) void k_cic_tile(int n, int nt, const float* __restrict__ pos,
                                                     const unsigned long long* __restrict__ runs,
                                                     const uint32_t* __restrict__ boff,
                                                     const uint32_t* __restrict__ cnt, double scale,
                                                     float* __restrict__ delta) {
  // kT^3 cells, then one slot per lane for the corners outside the tile
  // (every corner is deposited, those outside into the lane's own slot)
  __shared__ unsigned long long acc[kT3 + 64];
  __shared__ uint32_t seg_lo[kCicSegs], seg_end[kCicSegs];
  __shared__ uint8_t seg_role[kCicSegs];
  __shared__ uint32_t rp0[kCicTB];        // run: first particle minus its batch number
  __shared__ uint8_t rrole[kCicTB];       // run: role
  __shared__ uint32_t bmbits[kCicWords];  // run-start bits
  __shared__ uint16_t bmpre[kCicWords];   // runs starting in earlier words
  __shared__ uint32_t wsum[kCicTB / 64];
  __shared__ uint32_t bnum[2];            // runs and particles of the batch
  static_assert(kCicTB <= 65535, "run counts fit 16 bits");
  const uint32_t ntiles = (uint32_t)nt * nt * nt;
  uint32_t t = blockIdx.x;
  if (ntiles % 8 == 0) t = (t & 7u) * (ntiles / 8) + (t >> 3);
  const int ti = (int)(t % nt), tj = (int)((t / nt) % nt), tk = (int)(t / ((uint32_t)nt * nt));
  for (int q = threadIdx.x; q < kT3; q += kCicTB) acc[q] = 0ull;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x < 64) {
    // lane i < kCicSegs: segment i is (role s, class c), enumerated in order
    // of s and then c with (c & s) == s; lane 0 is the own tile's 8 bins
    int s = 0, c = 0;
    if (lane > 0 && lane < kCicSegs) {
      int k = 0;
      for (int ss = 1; ss < 8; ++ss)
        for (int cc = 1; cc < 8; ++cc)
          if ((cc & ss) == ss && ++k == lane) {
            s = ss;
            c = cc;
          }
    }
    uint32_t lo = 0, m = 0;
    if (lane < kCicSegs) {
      const int si = (s & 1) ? (ti == 0 ? nt - 1 : ti - 1) : ti;
      const int sj = (s & 2) ? (tj == 0 ? nt - 1 : tj - 1) : tj;
      const int sk = (s & 4) ? (tk == 0 ? nt - 1 : tk - 1) : tk;
      const uint32_t src = ((uint32_t)sk * nt + (uint32_t)sj) * nt + (uint32_t)si;
      lo = boff[8 * src + c];
      if (lane == 0) {
        const uint4 u = reinterpret_cast<const uint4*>(cnt)[2 * src];
        const uint4 v = reinterpret_cast<const uint4*>(cnt)[2 * src + 1];
        m = u.x + u.y + u.z + u.w + v.x + v.y + v.z + v.w;
      } else {
        m = cnt[8 * src + c];
      }
    }
    uint32_t end = m;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
      const uint32_t y = __shfl_up(end, d, 64);
      if (lane >= d) end += y;
    }
    if (lane < kCicSegs) {
      seg_lo[lane] = lo;
      seg_end[lane] = end;
      seg_role[lane] = (uint8_t)s;
    }
  }
  __syncthreads();
  const uint32_t total = seg_end[kCicSegs - 1];
  int sg = 0;
  for (uint32_t r0 = 0; r0 < total;) {
    // this batch's candidate runs: first particle, role, and the inclusive
    // prefix of the lengths
    bmbits[threadIdx.x] = 0u;
    if (threadIdx.x < 2) bnum[threadIdx.x] = 0u;
    const uint32_t r = r0 + threadIdx.x;
    uint32_t len = 0, p0 = 0;
    int role = 0;
    if (r < total) {
      while (r >= seg_end[sg]) ++sg;
      const uint32_t start = sg ? seg_end[sg - 1] : 0u;
      const unsigned long long v = runs[seg_lo[sg] + (r - start)];
      p0 = (uint32_t)(v >> 6);
      len = (uint32_t)(v & 63ull) + 1u;
      role = seg_role[sg];
    }
    uint32_t inc = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();  // wsum complete; bitmap and batch counters cleared
    uint32_t wpre = 0;
#pragma unroll
    for (int w = 0; w < kCicTB / 64; ++w) wpre += w < wv ? wsum[w] : 0u;
    const uint32_t first = wpre + inc - len, end = wpre + inc;
    // the batch: the leading runs that end within kCicCap particles (at
    // least the first run, whose length is at most 64)
    const bool in = len > 0 && end <= (uint32_t)kCicCap;
    const unsigned long long bal = __ballot(in);
    if (in) {
      rp0[threadIdx.x] = p0 - first;
      rrole[threadIdx.x] = (uint8_t)role;
      atomicOr(&bmbits[first >> 5], 1u << (first & 31));
      // the wave's included runs are a prefix of it: its last one ends last
      if (lane == 63 - __clzll(bal)) {
        atomicAdd(&bnum[0], (uint32_t)__popcll(bal));
        atomicMax(&bnum[1], end);
      }
    }
    __syncthreads();  // bits set, batch counts known; wsum (read above) is reused below
    const uint32_t nb = bnum[0], all = bnum[1];
    {
      // exclusive prefix of the run starts over the words (one per thread)
      const uint32_t c0 = __popc(bmbits[threadIdx.x]);
      uint32_t ic = c0;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(ic, d, 64);
        if (lane >= d) ic += y;
      }
      if (lane == 63) wsum[wv] = ic;
      __syncthreads();
      uint32_t wp = 0;
#pragma unroll
      for (int w = 0; w < kCicTB / 64; ++w) wp += w < wv ? wsum[w] : 0u;
      bmpre[threadIdx.x] = (uint16_t)(wp + ic - c0);
    }
    __syncthreads();
    for (uint32_t g0 = threadIdx.x; g0 < all; g0 += kCicUnroll * kCicTB) {
      CicCell cc[kCicUnroll];
      int rl[kCicUnroll];
      bool ok[kCicUnroll];
#pragma unroll
      for (int u = 0; u < kCicUnroll; ++u) {
        const uint32_t g = g0 + (uint32_t)u * kCicTB;
        ok[u] = g < all;
        rl[u] = 0;
        if (ok[u]) {
          const uint32_t wbits = bmbits[g >> 5];
          const uint32_t k = (uint32_t)bmpre[g >> 5] + __popc(wbits & ((2u << (g & 31)) - 1u)) - 1u;
          rl[u] = (int)rrole[k];
          cc[u] = cic_cell(n, pos, (int64_t)(uint32_t)(rp0[k] + g));
        }
      }
#pragma unroll
      for (int u = 0; u < kCicUnroll; ++u) {
        if (!ok[u]) continue;
        const int s = rl[u];
        long long w[8];
        cic_weights(cc[u], w);
        // local lower corner in [-1, kT - 1] per axis (-1: the lower
        // neighbour's last layer, role bit set)
        const int a = (cc[u].i0[0] & (kT - 1)) - ((s & 1) ? kT : 0);
        const int b = (cc[u].i0[1] & (kT - 1)) - ((s & 2) ? kT : 0);
        const int d = (cc[u].i0[2] & (kT - 1)) - ((s & 4) ? kT : 0);
        const bool ox[2] = {a >= 0, a < kT - 1}, oy[2] = {b >= 0, b < kT - 1},
                   oz[2] = {d >= 0, d < kT - 1};
        const int c0 = (d * kT + b) * kT + a;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
          const int at = ox[dx] && oy[dy] && oz[dz] ? c0 + (dz * kT + dy) * kT + dx : kT3 + lane;
          atomicAdd(&acc[at], (unsigned long long)w[q]);
        }
      }
    }
    __syncthreads();  // rp0, rrole, the bitmap, wsum and bnum are rewritten by the next batch
    r0 += nb;
  }
  for (int q = threadIdx.x; q < kT3; q += kCicTB) {
    const int x = q % kT, y = (q / kT) % kT, z = q / (kT * kT);
    const int64_t cell = ((int64_t)(tk * kT + z) * n + (tj * kT + y)) * n + (ti * kT + x);
    delta[cell] = float(double(acc[q]) * scale - 1.0);
  }
}

template <int M>
int dispatch_solve(mg_ctx* ctx, const Consts& C, const mg_solver_opts* o, const float* delta,
                   const double* fin, double* fout, double tol, mg_stats* st) {
  if (o->precision == MG_FP32_REFINED) return solve32<M>(ctx, C, o, delta, fin, fout, tol, st);
  return solve64<M>(ctx, C, o, delta, fin, fout, tol, st);
}

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace of one n^3 solve (both precisions, so
// the refined mode's FP64 fallback needs nothing more, and the reduction
// partials) lives in one static device array per GPU.  In host code
// 'scratch' names a host-side stand-in: its device address on the current
// GPU comes from hipGetSymbolAddress, looked up once per device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_at[kMaxDevices] = {};

int scratch_base(mg_ctx* ctx, char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ctx, MG_EHIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_at[dev] = (char*)p;
  }
  *out = g_scratch_at[dev];
  return MG_OK;
}

// Carves the workspace of ctx's level pyramid from base (the same roles as
// ensure32 and ensure64 allocate) and returns the bytes it takes; with base
// null it only counts.
struct NoallocWork {
  Work32 w32;
  Work64 w64;
  double *part = nullptr, *part2 = nullptr, *part3 = nullptr, *part4 = nullptr, *scal = nullptr;
};
size_t noalloc_layout(const mg_ctx* ctx, char* base, NoallocWork* W) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)(base + off) : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  W->part = (double*)take(sizeof(double) * (size_t)ctx->part_cap);
  W->part2 = (double*)take(sizeof(double) * 256);
  W->part3 = (double*)take(sizeof(double) * (size_t)ctx->part_cap);
  W->part4 = (double*)take(sizeof(double) * (size_t)ctx->part_cap);
  W->scal = (double*)take(sizeof(double) * 16);
  const size_t m0 = (size_t)cells(ctx->L[0]);
  W->w32.wbuf[0] = (double*)take(8 * m0);
  W->w32.wbuf[1] = (double*)take(8 * m0);
  W->w32.ebuf[1] = (float*)take(4 * m0);
  W->w32.w = W->w32.wbuf[0];
  W->w32.X16 = (h16*)take(2 * m0);
  W->w32.R16 = (h16*)take(2 * m0);
  W->w64.dens0 = (float*)take(4 * m0);
  for (int l = 0; l < ctx->nlev; ++l) {
    const size_t m = (size_t)cells(ctx->L[l]);
    W->w32.e[l] = (float*)take(4 * m);
    W->w32.X[l] = (float*)take(4 * m);
    W->w32.rho[l] = (float*)take(4 * m);
    W->w32.dens[l] = (float*)take(4 * m);
    if (l > 0) W->w32.eR[l] = (float*)take(4 * m);
    W->w64.v[l] = (double*)take(8 * m);
    if (l > 0) {
      W->w64.dens[l] = (double*)take(8 * m);
      W->w64.S[l] = (double*)take(8 * m);
      W->w64.Rv[l] = (double*)take(8 * m);
    }
  }
  W->w32.ebuf[0] = W->w32.e[0];
  return off;
}

// Points ctx's workspace at the scratch array for one call and restores the
// context's own (allocated or not) afterwards.
struct NoallocScope {
  mg_ctx* c;
  Work32 w32;
  Work64 w64;
  bool h32, h64;
  double *part, *part2, *part3, *part4, *scal;
  NoallocScope(mg_ctx* x, const NoallocWork& W)
      : c(x), w32(x->w32), w64(x->w64), h32(x->have32), h64(x->have64), part(x->part),
        part2(x->part2), part3(x->part3), part4(x->part4), scal(x->scal) {
    c->w32 = W.w32;
    c->w64 = W.w64;
    c->have32 = c->have64 = true;
    c->part = W.part;
    c->part2 = W.part2;
    c->part3 = W.part3;
    c->part4 = W.part4;
    c->scal = W.scal;
    c->noalloc = true;
  }
  ~NoallocScope() {
    c->w32 = w32;
    c->w64 = w64;
    c->have32 = h32;
    c->have64 = h64;
    c->part = part;
    c->part2 = part2;
    c->part3 = part3;
    c->part4 = part4;
    c->scal = scal;
    c->noalloc = false;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int mg_ctx_create(mg_ctx** out, int n, void* hip_stream) {
  if (!out) return MG_EINVAL;
  *out = nullptr;
  if (n < 4 || (n & 1) || n > 1600) return MG_EINVAL;  // n^3 < 2^32: 32-bit indices
  mg_ctx* ctx = new mg_ctx();
  ctx->n = n;
  if (const char* mb = getenv("MGGPU_MARCH_MIN_BLOCKS")) ctx->march_min_blocks = (unsigned)atoi(mb);
  if (const char* cd = getenv("MGGPU_CIC_DIRECT")) ctx->cic_direct = atoi(cd) != 0;
  if (const char* ts = getenv("MGGPU_TEST_CORRECTION_SCALE")) ctx->test_escale = (float)atof(ts);
  if (const char* fs = getenv("MGGPU_FP16_STORAGE")) ctx->fp16 = atoi(fs) != 0;
  if (const char* pk = getenv("MGGPU_PROLONG_SMOOTH_KT")) {
    const int kt = atoi(pk);
    ctx->psmooth_kt = kt > 0 && kt <= 64 ? kt : 0;
  }
  if (const char* pm = getenv("MGGPU_PROLONG_SMOOTH_MIN_BLOCKS"))
    ctx->psmooth_min_blocks = (unsigned)atoi(pm);
  if (const char* sk = getenv("MGGPU_SMOOTH_MARCH_KT")) {
    const int kt = atoi(sk);
    ctx->smooth_march_kt = kt > 0 && kt <= 64 ? kt : 0;
  }
  ctx->stream = (hipStream_t)hip_stream;
  // pyramid: halve while the half is even and >= 4
  int m = n, l = 0;
  for (;;) {
    ctx->L[l].n = m;
    ctx->L[l].nh = m / 2;
    ctx->L[l].half = (int64_t)m * m * m / 2;
    ctx->L[l].dnh = FastDiv::make((uint32_t)(m / 2));
    ctx->L[l].dn = FastDiv::make((uint32_t)m);
    ++l;
    if (!(m / 2 >= 4 && ((m / 2) % 2) == 0) || l >= kMaxLev) break;
    m /= 2;
  }
  ctx->nlev = l;
  int f = ctx->nlev;
  for (int q = 1; q < ctx->nlev; ++q)
    if (ctx->L[q].n <= kFuseN) {
      f = q;
      break;
    }
  if (f > ctx->nlev - 1) f = ctx->nlev - 1;  // the coarsest level is always solved
  // Level 0 never runs in the single-block kernels (they expect the coarse
  // levels' buffers); a grid that cannot be coarsened is relaxed by the
  // level-0 smoother instead (single_level_sweeps).
  if (f < 1) f = ctx->nlev;
  if (ctx->nlev - f > kMaxFused) f = ctx->nlev - kMaxFused;
  ctx->fused_from = f;
  ctx->part_cap = nblk((int64_t)n * n * n) + 16;
  int rc = dalloc(ctx, &ctx->part, ctx->part_cap);
  if (rc == MG_OK) rc = dalloc(ctx, &ctx->part2, 256);
  if (rc == MG_OK) rc = dalloc(ctx, &ctx->part3, ctx->part_cap);
  if (rc == MG_OK) rc = dalloc(ctx, &ctx->part4, ctx->part_cap);
  if (rc == MG_OK) rc = dalloc(ctx, &ctx->scal, 16);
  if (rc == MG_OK) {
    void* h = nullptr;
    if (hipHostMalloc(&h, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess) rc = MG_EHIP;
    ctx->hscal = (double*)h;
  }
  if (rc != MG_OK) {
    mg_ctx_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return MG_OK;
}

void mg_ctx_destroy(mg_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  if (ctx->bpool) (void)hipFree(ctx->bpool);
  if (ctx->bdev) (void)hipFree(ctx->bdev);
  if (ctx->bout) (void)hipFree(ctx->bout);
  for (void* p : {(void*)ctx->border, (void*)ctx->bteams, (void*)ctx->bwg, (void*)ctx->bctr,
                  (void*)ctx->bparts, (void*)ctx->babort, (void*)ctx->gtab, (void*)ctx->gctl,
                  (void*)ctx->gpart, (void*)ctx->gsum})
    if (p) (void)hipFree(p);
  if (ctx->ghsum) (void)hipHostFree(ctx->ghsum);
  for (int i = 0; i < mg_ctx::kGStreams; ++i) {
    if (ctx->gst[i]) (void)hipStreamDestroy(ctx->gst[i]);
    if (ctx->gjoin[i]) (void)hipEventDestroy(ctx->gjoin[i]);
  }
  if (ctx->gfork) (void)hipEventDestroy(ctx->gfork);
  for (void* p : ctx->allocs) (void)hipFree(p);
  if (ctx->hscal) (void)hipHostFree(ctx->hscal);
  if (ctx->fft_ready) {
    std::string e;
    if (const RocfftApi* F = rocfft_api(&e)) {
      if (ctx->fft_fwd) F->plan_destroy(ctx->fft_fwd);
      if (ctx->fft_inv) F->plan_destroy(ctx->fft_inv);
      if (ctx->fft_info) F->info_destroy(ctx->fft_info);
    }
  }
  if (ctx->fft_work) (void)hipFree(ctx->fft_work);
  delete ctx;
}

const char* mg_last_error(const mg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int mg_ctx_levels(const mg_ctx* ctx) { return ctx ? ctx->nlev : 0; }

int cic_assign(mg_ctx* ctx, const float* pos, int64_t np, float* delta_out) {
  if (!ctx) return MG_EINVAL;
  if (!pos || !delta_out || np <= 0) return fail(ctx, MG_EINVAL, "cic_assign: bad arguments");
  int n = ctx->n;
  int64_t m = (int64_t)n * n * n;
  double scale = double(m) / double(np) / 4294967296.0;
  const int nt = n / kT;
  const int64_t ntiles = (int64_t)nt * nt * nt;
  if (n % kT == 0 && np < (int64_t)0xffffffffLL - kCicRegion &&
      8 * ntiles < ((int64_t)1 << kCicBinBits) && !ctx->cic_direct) {
    // binned path: runs of equal bins counted and recorded, scan, runs
    // placed in bin order, per-tile LDS deposit
    const unsigned nbp = (unsigned)((np + kCicRegion - 1) / kCicRegion);
    if (ctx->cic_np < np) {
      ACHK(dalloc(ctx, &ctx->cic_rec, (int64_t)nbp * kCicRegion));
      ACHK(dalloc(ctx, &ctx->cic_nrec, (int64_t)nbp));
      ACHK(dalloc(ctx, &ctx->cic_runs, np));
      ctx->cic_np = np;
    }
    if (!ctx->cic_cnt) ACHK(dalloc(ctx, &ctx->cic_cnt, 3 * 8 * ntiles));
    uint32_t* cnt = ctx->cic_cnt;
    uint32_t* boff = cnt + 8 * ntiles;
    uint32_t* cur = boff + 8 * ntiles;
    k_fill<uint32_t><<<nblk(8 * ntiles), kBlock, 0, ctx->stream>>>(cnt, 8 * ntiles, 0u);
    k_cic_runs<<<nbp, kCicCB, 0, ctx->stream>>>(n, nt, np, pos, cnt, ctx->cic_rec, ctx->cic_nrec);
    k_cic_scan<<<1, 1024, 0, ctx->stream>>>(cnt, ntiles, boff, cur);
    k_cic_place<<<nbp, kCicCB, 0, ctx->stream>>>(ctx->cic_rec, ctx->cic_nrec, cur, ctx->cic_runs);
    k_cic_tile<<<(unsigned)ntiles, kCicTB, 0, ctx->stream>>>(n, nt, pos, ctx->cic_runs, boff, cnt,
                                                             scale, delta_out);
    LAUNCHCHK();
    return MG_OK;
  }
  if (!ctx->cic) ACHK(dalloc(ctx, &ctx->cic, m));
  unsigned long long* acc = (unsigned long long*)ctx->cic;
  k_fill<unsigned long long><<<nblk(m), kBlock, 0, ctx->stream>>>(acc, m, 0ull);
  k_cic<<<nblk(np), kBlock, 0, ctx->stream>>>(n, np, pos, acc);
  k_cic_finish<<<nblk(m), kBlock, 0, ctx->stream>>>(m, acc, scale, delta_out);
  LAUNCHCHK();
  return MG_OK;
}

int mg_solve(mg_ctx* ctx, int model, const mg_model_params* params, const mg_solver_opts* opts,
             const float* delta, const double* field_in, double* field_out, double tol,
             mg_stats* stats) {
  if (!ctx) return MG_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  Consts C;
  ACHK(make_consts(ctx, model, params, ctx->n, &C));
  ACHK(check_opts(ctx, opts));
  if (!delta || !field_out) return fail(ctx, MG_EINVAL, "mg_solve: NULL array");
  if (!(tol > 0.0)) return fail(ctx, MG_EINVAL, "mg_solve: tol must be > 0");
  if (stats) memset(stats, 0, sizeof *stats);
  int rc;
  if (model == MG_FR) rc = dispatch_solve<FR>(ctx, C, opts, delta, field_in, field_out, tol, stats);
  else if (model == MG_SYMMETRON)
    rc = dispatch_solve<SYM>(ctx, C, opts, delta, field_in, field_out, tol, stats);
  else rc = dispatch_solve<CQ>(ctx, C, opts, delta, field_in, field_out, tol, stats);
  if (stats) {
    (void)hipStreamSynchronize(ctx->stream);
    stats->status = rc;
    stats->ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return rc;
}

int mg_solve_noalloc(mg_ctx* ctx, int model, const mg_model_params* params,
                     const mg_solver_opts* opts, const float* delta, const double* field_in,
                     double* field_out, double tol, mg_stats* stats) {
  if (!ctx) return MG_EINVAL;
  ACHK(check_opts(ctx, opts));
  NoallocWork W;
  const size_t need = noalloc_layout(ctx, nullptr, &W);
  if (need > kScratchBytes)
    return fail(ctx, MG_EINVAL, "mg_solve_noalloc: an n^3 solve needs " + std::to_string(need) +
                                    " bytes of workspace; the scratch array holds " +
                                    std::to_string(kScratchBytes) + " (n <= 64)");
  char* base = nullptr;
  ACHK(scratch_base(ctx, &base));
  noalloc_layout(ctx, base, &W);
  NoallocScope scope(ctx, W);
  return mg_solve(ctx, model, params, opts, delta, field_in, field_out, tol, stats);
}

int mg_residual(mg_ctx* ctx, int model, const mg_model_params* params, const float* delta,
                const double* field, double* d_out, double* rel) {
  if (!ctx) return MG_EINVAL;
  Consts C;
  ACHK(make_consts(ctx, model, params, ctx->n, &C));
  if (!delta || !field) return fail(ctx, MG_EINVAL, "mg_residual: NULL array");
  ACHK(ensure64(ctx));
  ACHK(setup64(ctx, C, delta, field));
  double eps_bg, r;
  ACHK(bg_rms(ctx, C, delta, &eps_bg));
  if (model == MG_FR) ACHK(resid64<FR>(ctx, C, eps_bg, &r, d_out));
  else if (model == MG_SYMMETRON) ACHK(resid64<SYM>(ctx, C, eps_bg, &r, d_out));
  else ACHK(resid64<CQ>(ctx, C, eps_bg, &r, d_out));
  if (rel) *rel = r;
  return MG_OK;
}

}  // extern "C"

namespace {

// CIC interpolation to particles (same cells and weights as the assignment)
template <typename TG, typename TO, int NC>
__global__ __launch_bounds__(kBlock) void k_interp(int n, int64_t np,
                                                   const float* __restrict__ pos,
                                                   const TG* __restrict__ grid,
                                                   TO* __restrict__ out) {
  int64_t p = gid();
  if (p >= np) return;
  const CicCell c = cic_cell(n, pos, p);
  const int64_t m = (int64_t)n * n * n;
  double w[8];
  int64_t cell[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int di = q & 1, dj = (q >> 1) & 1, dk = (q >> 2) & 1;
    w[q] = (di ? c.t[0] : 1.0 - c.t[0]) * (dj ? c.t[1] : 1.0 - c.t[1]) *
           (dk ? c.t[2] : 1.0 - c.t[2]);
    const int ii = c.i0[0] + di == n ? 0 : c.i0[0] + di;
    const int jj = c.i0[1] + dj == n ? 0 : c.i0[1] + dj;
    const int kk = c.i0[2] + dk == n ? 0 : c.i0[2] + dk;
    cell[q] = ((int64_t)kk * n + jj) * n + ii;
  }
  // all 8 NC loads are independent: issue them together.  Corners q and q+1
  // are x-neighbours; unless the pair wraps the periodic seam they are
  // adjacent in memory and are read as one 2-element load.
  TG v[NC][8];
  const bool pair = c.i0[0] + 1 < n;
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      const TG* src = grid + a * m + cell[q];
      if (pair) {
        typedef TG two_t __attribute__((ext_vector_type(2), aligned(sizeof(TG))));
        const two_t two = *reinterpret_cast<const two_t*>(src);
        v[a][q] = two.x;
        v[a][q + 1] = two.y;
      } else {
        v[a][q] = src[0];
        v[a][q + 1] = grid[a * m + cell[q + 1]];
      }
    }
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += w[q] * double(v[a][q]);
    out[p * NC + a] = TO(acc);
  }
}

// symmetron friction term per particle: coef u(x_p) p_p
__global__ __launch_bounds__(kBlock) void k_sym_friction(int n, int64_t np,
                                                         const float* __restrict__ pos,
                                                         const double* __restrict__ u,
                                                         const float* __restrict__ mom,
                                                         double coef, float* __restrict__ out) {
  int64_t p = gid();
  if (p >= np) return;
  const CicCell c = cic_cell(n, pos, p);
  double up = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int di = q & 1, dj = (q >> 1) & 1, dk = (q >> 2) & 1;
    const double w = (di ? c.t[0] : 1.0 - c.t[0]) * (dj ? c.t[1] : 1.0 - c.t[1]) *
                     (dk ? c.t[2] : 1.0 - c.t[2]);
    const int ii = c.i0[0] + di == n ? 0 : c.i0[0] + di;
    const int jj = c.i0[1] + dj == n ? 0 : c.i0[1] + dj;
    const int kk = c.i0[2] + dk == n ? 0 : c.i0[2] + dk;
    up += w * u[((int64_t)kk * n + jj) * n + ii];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) out[3 * p + a] = float(coef * up * double(mom[3 * p + a]));
}

__global__ __launch_bounds__(kBlock) void k_f2d(int64_t m, const float* __restrict__ x,
                                                double* __restrict__ y) {
  int64_t g = gid();
  if (g < m) y[g] = double(x[g]);
}
// 4 values per thread (16-byte aligned arrays, m % 4 == 0)
__global__ __launch_bounds__(kBlock) void k_f2d4(int64_t m4, const float4* __restrict__ x,
                                                 double2* __restrict__ y) {
  int64_t g = gid();
  if (g >= m4) return;
  const float4 v = x[g];
  y[2 * g] = make_double2(double(v.x), double(v.y));
  y[2 * g + 1] = make_double2(double(v.z), double(v.w));
}

// sin^2(pi m / n) for m in [0, n): the 7-point Laplacian symbol per axis
__global__ __launch_bounds__(kBlock) void k_sin2(int n, double* __restrict__ s2) {
  int64_t g = gid();
  if (g < n) {
    const double v = sinpi(double(g) / n);
    s2[g] = v * v;
  }
}

// multiply the half spectrum (n x n x (n/2+1), fastest last) by the inverse of
// the 7-point discrete Laplacian symbol -4 sum sin^2(pi m_i / n) times coef,
// including the 1/n^3 of the unnormalised inverse transform; zero mode -> 0
__global__ __launch_bounds__(kBlock) void k_poisson_green(int n, double2* __restrict__ c,
                                                          double coef, FastDiv dnx, FastDiv dn,
                                                          const double* __restrict__ s2) {
  const uint32_t nx = (uint32_t)(n / 2 + 1);
  const uint32_t g = (uint32_t)gid();
  const uint32_t mc = (uint32_t)n * (uint32_t)n * nx;
  if (g >= mc) return;
  const uint32_t r = dnx.div(g), kx = g - r * nx;
  const uint32_t kz = dn.div(r), ky = r - kz * (uint32_t)n;
  const double k2 = 4.0 * (s2[kx] + s2[ky] + s2[kz]);
  const double f = (g == 0) ? 0.0 : -coef / (k2 * (double(n) * n * n));
  double2 v = c[g];
  v.x *= f;
  v.y *= f;
  c[g] = v;
}

// -grad of Phi5(f) (+ pn): z-marching kernel when n % 4 == 0
void launch_force(mg_ctx* ctx, const Consts& C, const double* f, const double* pn, double sn,
                  float* out) {
  const int n = ctx->n;
  const int64_t m = (int64_t)n * n * n;
  if (n % (4 * kFTX) == 0 && al16(f, out) && al16(pn)) {
    static_assert(kFTX * kFTY == kBlock, "one thread per 4-cell group of the tile");
    const unsigned tiles = (unsigned)((n / (4 * kFTX)) * (n / kFTY));
    const unsigned nb = tiles * (unsigned)((n + kMarchKT - 1) / kMarchKT);
    if (pn)
      k_force_tile<true><<<nb, kBlock, 0, ctx->stream>>>(ctx->L[0], f, pn, sn, C, out, kMarchKT);
    else
      k_force_tile<false><<<nb, kBlock, 0, ctx->stream>>>(ctx->L[0], f, nullptr, 0.0, C, out,
                                                          kMarchKT);
  } else if (n % 4 == 0 && al16(f, out) && al16(pn)) {
    unsigned nchunk = (unsigned)(((int64_t)n * n / 4 + kBlock - 1) / kBlock);
    unsigned nb = nchunk * (unsigned)((n + kMarchKT - 1) / kMarchKT);
    if (pn) k_force_kv<true><<<nb, kBlock, 0, ctx->stream>>>(ctx->L[0], f, pn, sn, C, out, kMarchKT);
    else k_force_kv<false><<<nb, kBlock, 0, ctx->stream>>>(ctx->L[0], f, nullptr, 0.0, C, out,
                                                           kMarchKT);
  } else {
    if (pn) k_force<true><<<nblk(m), kBlock, 0, ctx->stream>>>(ctx->L[0], f, pn, sn, C, out);
    else k_force<false><<<nblk(m), kBlock, 0, ctx->stream>>>(ctx->L[0], f, nullptr, 0.0, C, out);
  }
}

int ensure_fft(mg_ctx* ctx) {
  if (ctx->fft_ready) return MG_OK;
  std::string e;
  const RocfftApi* F = rocfft_api(&e);
  if (!F) return fail(ctx, MG_EHIP, "rocFFT unavailable: " + e);
  const size_t n = (size_t)ctx->n;
  const size_t len[3] = {n, n, n};
  if (F->plan_create(&ctx->fft_fwd, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                     rocfft_precision_double, 3, len, 1, nullptr) != rocfft_status_success ||
      F->plan_create(&ctx->fft_inv, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                     rocfft_precision_double, 3, len, 1, nullptr) != rocfft_status_success)
    return fail(ctx, MG_EHIP, "rocFFT plan creation failed");
  size_t w1 = 0, w2 = 0;
  F->work_size(ctx->fft_fwd, &w1);
  F->work_size(ctx->fft_inv, &w2);
  ctx->fft_work_bytes = std::max(w1, w2);
  if (ctx->fft_work_bytes) HIPCHK(hipMalloc(&ctx->fft_work, ctx->fft_work_bytes));
  if (F->info_create(&ctx->fft_info) != rocfft_status_success)
    return fail(ctx, MG_EHIP, "rocFFT execution info failed");
  if (ctx->fft_work_bytes) F->info_set_work(ctx->fft_info, ctx->fft_work, ctx->fft_work_bytes);
  F->info_set_stream(ctx->fft_info, ctx->stream);
  ACHK(dalloc(ctx, &ctx->fft_c, (int64_t)n * n * (n / 2 + 1)));
  ACHK(dalloc(ctx, &ctx->fft_s2, (int64_t)n));
  k_sin2<<<nblk(n), kBlock, 0, ctx->stream>>>(n, ctx->fft_s2);
  LAUNCHCHK();
  ctx->fft_ready = true;
  return MG_OK;
}

}  // namespace

extern "C" {

int mg_interp_to_particles(mg_ctx* ctx, const float* grid, int ncomp, const float* pos,
                           int64_t np, float* out) {
  if (!ctx) return MG_EINVAL;
  if (np == 0 && ncomp >= 1 && ncomp <= 3) return MG_OK;  // no particles: nothing to do
  if (!grid || !pos || !out || np < 0 || ncomp < 1 || ncomp > 3)
    return fail(ctx, MG_EINVAL, "mg_interp_to_particles: bad arguments");
  if (ncomp == 3)
    k_interp<float, float, 3><<<nblk(np), kBlock, 0, ctx->stream>>>(ctx->n, np, pos, grid, out);
  else if (ncomp == 2)
    k_interp<float, float, 2><<<nblk(np), kBlock, 0, ctx->stream>>>(ctx->n, np, pos, grid, out);
  else
    k_interp<float, float, 1><<<nblk(np), kBlock, 0, ctx->stream>>>(ctx->n, np, pos, grid, out);
  LAUNCHCHK();
  return MG_OK;
}

int mg_interp_field_to_particles(mg_ctx* ctx, const double* field, const float* pos, int64_t np,
                                 double* out) {
  if (!ctx) return MG_EINVAL;
  if (np == 0) return MG_OK;
  if (!field || !pos || !out || np < 0)
    return fail(ctx, MG_EINVAL, "mg_interp_field_to_particles: bad arguments");
  k_interp<double, double, 1><<<nblk(np), kBlock, 0, ctx->stream>>>(ctx->n, np, pos, field, out);
  LAUNCHCHK();
  return MG_OK;
}

int mg_poisson_newton(mg_ctx* ctx, const mg_model_params* params, const float* delta,
                      double* phi_out) {
  if (!ctx) return MG_EINVAL;
  if (!params || !delta || !phi_out) return fail(ctx, MG_EINVAL, "mg_poisson_newton: NULL");
  if (!(params->a > 0.0) || !(params->omega_m > 0.0))
    return fail(ctx, MG_EINVAL, "mg_poisson_newton: need a > 0 and omega_m > 0");
  ACHK(ensure_fft(ctx));
  std::string e;
  const RocfftApi* F = rocfft_api(&e);
  const int n = ctx->n;
  const int64_t m = (int64_t)n * n * n;
  const int64_t mc = (int64_t)n * n * (n / 2 + 1);
  if (m % 4 == 0 && al16(delta, phi_out))
    k_f2d4<<<nblk(m / 4), kBlock, 0, ctx->stream>>>(m / 4, reinterpret_cast<const float4*>(delta),
                                                     reinterpret_cast<double2*>(phi_out));
  else
    k_f2d<<<nblk(m), kBlock, 0, ctx->stream>>>(m, delta, phi_out);
  LAUNCHCHK();
  void* in[1] = {phi_out};
  void* cout[1] = {ctx->fft_c};
  if (F->execute(ctx->fft_fwd, in, cout, ctx->fft_info) != rocfft_status_success)
    return fail(ctx, MG_EHIP, "rocFFT forward transform failed");
  k_poisson_green<<<nblk(mc), kBlock, 0, ctx->stream>>>(
      n, ctx->fft_c, 1.5 * params->omega_m / params->a, FastDiv::make((uint32_t)(n / 2 + 1)),
      FastDiv::make((uint32_t)n), ctx->fft_s2);
  LAUNCHCHK();
  void* cin[1] = {ctx->fft_c};
  void* out[1] = {phi_out};
  if (F->execute(ctx->fft_inv, cin, out, ctx->fft_info) != rocfft_status_success)
    return fail(ctx, MG_EHIP, "rocFFT inverse transform failed");
  return MG_OK;
}

int mg_gradient(mg_ctx* ctx, const double* phi, float* force_out) {
  if (!ctx) return MG_EINVAL;
  if (!phi || !force_out) return fail(ctx, MG_EINVAL, "mg_gradient: NULL array");
  Consts C;
  memset(&C, 0, sizeof C);
  C.model = CQ;  // Phi5 = phi5 * f with phi5 = 1: the plain potential
  C.phi5 = 1.0;
  launch_force(ctx, C, phi, nullptr, 0.0, force_out);
  LAUNCHCHK();
  return MG_OK;
}

int mg_total_force(mg_ctx* ctx, int model, const mg_model_params* params, const double* phi_n,
                   const double* field, float* force_out) {
  if (!ctx) return MG_EINVAL;
  Consts C;
  ACHK(make_consts(ctx, model, params, ctx->n, &C));
  if (!phi_n || !field || !force_out) return fail(ctx, MG_EINVAL, "mg_total_force: NULL array");
  // coupled quintessence: the standard potential carries exp(beta phibar)
  const double sn = model == MG_CQ ? exp(params->cq_beta * params->cq_phibar) : 1.0;
  launch_force(ctx, C, field, phi_n, sn, force_out);
  LAUNCHCHK();
  return MG_OK;
}

int mg_symmetron_friction(mg_ctx* ctx, const mg_model_params* params, const double* u_field,
                          const float* pos, const float* mom, int64_t np, float* out) {
  if (!ctx) return MG_EINVAL;
  if (!params || np < 0 || (np > 0 && (!u_field || !pos || !mom || !out)))
    return fail(ctx, MG_EINVAL, "mg_symmetron_friction: bad arguments");
  const double a = params->a, as = params->sym_a_star;
  if (!(a > 0.0) || !(as > 0.0) || !(as < a))
    return fail(ctx, MG_EINVAL, "mg_symmetron_friction: need 0 < a_* < a");
  // -(dA/dphi)(d phi-bar/da) of eq:csf_particle_geodesic_qsa with A of
  // eq:sym_coupling_function, phi_* of eq:varphi_ast and phi-bar(a) of
  // eq:varphi_min_symm: 9 Om beta*^2 xi^2 a^-4 u / u-bar (eq:F_x_codeunit
  // prints u-bar in place of 1/u-bar)
  const double coef = -9.0 * params->omega_m * params->sym_beta_star * params->sym_beta_star *
                      params->sym_xi * params->sym_xi /
                      (sqrt(1.0 - pow(as / a, 3.0)) * pow(a, 4.0));
  if (np == 0) return MG_OK;
  k_sym_friction<<<nblk(np), kBlock, 0, ctx->stream>>>(ctx->n, np, pos, u_field, mom, coef, out);
  LAUNCHCHK();
  return MG_OK;
}

int mg_force(mg_ctx* ctx, int model, const mg_model_params* params, const double* field,
             float* force_out) {
  if (!ctx) return MG_EINVAL;
  Consts C;
  ACHK(make_consts(ctx, model, params, ctx->n, &C));
  if (!field || !force_out) return fail(ctx, MG_EINVAL, "mg_force: NULL array");
  launch_force(ctx, C, field, nullptr, 0.0, force_out);
  LAUNCHCHK();
  return MG_OK;
}

int mg_force_adjoint(mg_ctx* ctx, int model, const mg_model_params* params, const double* field,
                     const float* grad_force, double* grad_field_out) {
  if (!ctx) return MG_EINVAL;
  Consts C;
  ACHK(make_consts(ctx, model, params, ctx->n, &C));
  if (!field || !grad_force || !grad_field_out)
    return fail(ctx, MG_EINVAL, "mg_force_adjoint: NULL array");
  const int n = ctx->n;
  int64_t m = (int64_t)n * n * n;
  if (n % (4 * kFTX) == 0 && al16(field, grad_force) && al16(grad_field_out)) {
    const unsigned tiles = (unsigned)((n / (4 * kFTX)) * (n / kFTY));
    const unsigned nb = tiles * (unsigned)((n + kMarchKT - 1) / kMarchKT);
    k_force_adjoint_tile<<<nb, kBlock, 0, ctx->stream>>>(ctx->L[0], field, grad_force, C,
                                                         grad_field_out, kMarchKT);
  } else {
    k_force_adjoint<<<nblk(m), kBlock, 0, ctx->stream>>>(ctx->L[0], field, grad_force, C,
                                                         grad_field_out);
  }
  LAUNCHCHK();
  return MG_OK;
}

int mg_solve_adjoint(mg_ctx* ctx, int model, const mg_model_params* params,
                     const mg_solver_opts* opts, const float* delta, const double* field,
                     const double* grad_field, double* grad_delta_out, double tol,
                     mg_stats* stats) {
  if (!ctx) return MG_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  Consts C;
  ACHK(make_consts(ctx, model, params, ctx->n, &C));
  ACHK(check_opts(ctx, opts));
  if (!delta || !field || !grad_field || !grad_delta_out)
    return fail(ctx, MG_EINVAL, "mg_solve_adjoint: NULL array");
  if (!(tol > 0.0)) return fail(ctx, MG_EINVAL, "mg_solve_adjoint: tol must be > 0");
  if (stats) memset(stats, 0, sizeof *stats);
  int rc;
  if (model == MG_FR)
    rc = adjoint_impl<FR>(ctx, C, opts, delta, field, grad_field, grad_delta_out, tol, stats);
  else if (model == MG_SYMMETRON)
    rc = adjoint_impl<SYM>(ctx, C, opts, delta, field, grad_field, grad_delta_out, tol, stats);
  else rc = adjoint_impl<CQ>(ctx, C, opts, delta, field, grad_field, grad_delta_out, tol, stats);
  if (stats) {
    (void)hipStreamSynchronize(ctx->stream);
    stats->status = rc;
    stats->ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return rc;
}

int mg_loss_force_sq(mg_ctx* ctx, const float* force, const int64_t* cellsv, int64_t n_cells,
                     float* grad_force_out, double* loss_out) {
  if (!ctx) return MG_EINVAL;
  if (!force || !cellsv || !grad_force_out || !loss_out || n_cells <= 0)
    return fail(ctx, MG_EINVAL, "mg_loss_force_sq: bad arguments");
  int64_t m = (int64_t)ctx->n * ctx->n * ctx->n;
  if (nblk(n_cells) > (unsigned)ctx->part_cap)
    return fail(ctx, MG_EINVAL, "mg_loss_force_sq: too many cells");
  if ((3 * m) % 4 == 0 && ((uintptr_t)grad_force_out & 15) == 0)
    k_fill4<<<nblk(3 * m / 4), kBlock, 0, ctx->stream>>>((float4*)grad_force_out, 3 * m / 4, 0.0f);
  else
    k_fill<float><<<nblk(3 * m), kBlock, 0, ctx->stream>>>(grad_force_out, 3 * m, 0.0f);
  k_loss_sq<<<nblk(n_cells), kBlock, 0, ctx->stream>>>(m, force, cellsv, n_cells, grad_force_out,
                                                       ctx->part);
  ACHK(sum_on_device(ctx, nblk(n_cells), loss_out));
  return MG_OK;
}

int mg_relax_halfsweep(mg_ctx* ctx, int model, const mg_model_params* params, const float* delta,
                       double* field, int colour) {
  if (!ctx) return MG_EINVAL;
  Consts C;
  ACHK(make_consts(ctx, model, params, ctx->n, &C));
  if (!delta || !field || (colour != 0 && colour != 1))
    return fail(ctx, MG_EINVAL, "mg_relax_halfsweep: bad arguments");
  ACHK(ensure64(ctx));
  ACHK(setup64(ctx, C, delta, field));
  const Lev& L = ctx->L[0];
  if (L.nh % Vec<double>::V == 0) {
    int64_t nv = L.half / Vec<double>::V;
    if (model == MG_FR)
      k_smooth_direct_v<FR, float><<<nblk(nv), kBlock, 0, ctx->stream>>>(
          L, ctx->w64.v[0], ctx->w64.dens0, (const double*)nullptr, colour, 1.0, C);
    else if (model == MG_SYMMETRON)
      k_smooth_direct_v<SYM, float><<<nblk(nv), kBlock, 0, ctx->stream>>>(
          L, ctx->w64.v[0], ctx->w64.dens0, (const double*)nullptr, colour, 1.0, C);
    else
      k_smooth_direct_v<CQ, float><<<nblk(nv), kBlock, 0, ctx->stream>>>(
          L, ctx->w64.v[0], ctx->w64.dens0, (const double*)nullptr, colour, 1.0, C);
  } else if (model == MG_FR) {
    k_smooth_direct<FR, double, float><<<nblk(L.half), kBlock, 0, ctx->stream>>>(
        L, ctx->w64.v[0], ctx->w64.dens0, (const double*)nullptr, colour, 1.0, C);
  } else if (model == MG_SYMMETRON) {
    k_smooth_direct<SYM, double, float><<<nblk(L.half), kBlock, 0, ctx->stream>>>(
        L, ctx->w64.v[0], ctx->w64.dens0, (const double*)nullptr, colour, 1.0, C);
  } else {
    k_smooth_direct<CQ, double, float><<<nblk(L.half), kBlock, 0, ctx->stream>>>(
        L, ctx->w64.v[0], ctx->w64.dens0, (const double*)nullptr, colour, 1.0, C);
  }
  double sgn = (model == MG_FR) ? -1.0 : 1.0;
  launch_unpack<double, double>(ctx, L, ctx->w64.v[0], field,
                                                                         sgn);
  LAUNCHCHK();
  return MG_OK;
}

int mg_restrict(mg_ctx* ctx, const double* fine, double* coarse) {
  if (!ctx) return MG_EINVAL;
  if (!fine || !coarse || ctx->nlev < 2) return fail(ctx, MG_EINVAL, "mg_restrict: bad arguments");
  ACHK(ensure64(ctx));
  const Lev& Lf = ctx->L[0];
  const Lev& Lc = ctx->L[1];
  launch_pack<double, double>(ctx, Lf, fine, ctx->w64.v[0], 1.0);
  k_restrict<double, double><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(Lf, Lc, ctx->w64.v[0],
                                                                          ctx->w64.v[1]);
  launch_unpack<double, double>(ctx, Lc, ctx->w64.v[1], coarse,
                                                                         1.0);
  LAUNCHCHK();
  return MG_OK;
}

int mg_prolong_add(mg_ctx* ctx, const double* coarse, double* fine) {
  if (!ctx) return MG_EINVAL;
  if (!fine || !coarse || ctx->nlev < 2)
    return fail(ctx, MG_EINVAL, "mg_prolong_add: bad arguments");
  ACHK(ensure64(ctx));
  const Lev& Lf = ctx->L[0];
  const Lev& Lc = ctx->L[1];
  launch_pack<double, double>(ctx, Lf, fine, ctx->w64.v[0], 1.0);
  launch_pack<double, double>(ctx, Lc, coarse, ctx->w64.v[1], 1.0);
  if (Lc.n % Vec<double>::V == 0)
    launch_prolong<double, 0>(ctx, Lf, Lc, ctx->w64.v[0], ctx->w64.v[1], (const double*)nullptr);
  else
    k_prolong_block<double><<<nblk(cells(Lc)), kBlock, 0, ctx->stream>>>(Lf, Lc, ctx->w64.v[0],
                                                                           ctx->w64.v[1]);
  launch_unpack<double, double>(ctx, Lf, ctx->w64.v[0], fine,
                                                                         1.0);
  LAUNCHCHK();
  return MG_OK;
}

int mg_prof_enable(mg_ctx* ctx, int on) {
  if (!ctx) return MG_EINVAL;
  if (on && ctx->ev.empty()) {
    ctx->ev.resize(2 * kEvPairs);
    ctx->ev_cls.resize(kEvPairs);
    for (auto& e : ctx->ev) HIPCHK(hipEventCreate(&e));
  }
  prof_flush(ctx);
  ctx->prof = on != 0;
  for (int c = 0; c < 4; ++c) {
    ctx->prof_ms[c] = 0.0;
    ctx->prof_n[c] = 0;
  }
  return MG_OK;
}

int mg_prof_read(mg_ctx* ctx, int cls, double* total_ms, int64_t* launches) {
  if (!ctx) return MG_EINVAL;
  if (cls < 0 || cls > 3 || !total_ms || !launches)
    return fail(ctx, MG_EINVAL, "mg_prof_read: bad arguments");
  prof_flush(ctx);
  *total_ms = ctx->prof_ms[cls];
  *launches = ctx->prof_n[cls];
  return MG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched solves: descriptors, workspace, tile-shape tuning
// ---------------------------------------------------------------------------
namespace {

constexpr int kTileBlocks[3] = {256, 512, 1024};

// level pyramid of one box (same rule as the context's)
int box_levels(int n, Lev* L) {
  int m = n, l = 0;
  for (;;) {
    L[l].n = m;
    L[l].nh = m / 2;
    L[l].half = (int64_t)m * m * m / 2;
    L[l].dnh = FastDiv::make((uint32_t)(m / 2));
    L[l].dn = FastDiv::make((uint32_t)m);
    ++l;
    if (!(m / 2 >= 4 && ((m / 2) % 2) == 0) || l >= kMaxLevB) break;
    m /= 2;
  }
  return l;
}

size_t box_bytes(const Lev* L, int nlev) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t t = up(8 * (size_t)(2 * L[0].half));
  for (int l = 0; l < nlev; ++l) t += (l > 0 ? 5 : 4) * up(4 * (size_t)(2 * L[l].half));
  return t;
}

// Builds and uploads the descriptors; allocates the workspace pool.
int batch_setup(mg_ctx* ctx, int nb, const mg_box_desc* boxes, const mg_solver_opts* o, double tol,
                bool trial, int vec, std::vector<BoxDev>& host) {
  host.assign(nb, BoxDev());
  size_t total = 0;
  for (int b = 0; b < nb; ++b) {
    BoxDev& B = host[b];
    memset(&B, 0, sizeof B);
    const mg_box_desc& D = boxes[b];
    if (D.n < 8 || (D.n & 1) || D.n > 1024 || !D.delta || !D.field)
      return fail(ctx, MG_EINVAL, "mg_solve_batched: box " + std::to_string(b) +
                                      " needs even 8 <= n <= 1024 and delta/field");
    ACHK(make_consts(ctx, D.model, &D.params, D.n, &B.C));
    B.model = D.model;
    B.nlev = box_levels(D.n, B.L);
    for (int l = 0; l < B.nlev; ++l) B.h2[l] = float(lev_h2(l));
    OpList ops;
    gen_prog(ops, 0, B.nlev - 1, o->cycle, o->nu_pre, o->nu_post);
    if (ops.over || ops.n > kMaxOpsB) return fail(ctx, MG_EINVAL, "cycle program too long");
    B.nops = ops.n;
    for (int q = 0; q < ops.n; ++q) B.op[q] = ops.op[q];
    B.vec = vec;
    B.nu1 = o->nu_pre;
    B.nu2 = o->nu_post;
    B.fixed_inner = trial ? 2 : o->inner_cycles;
    B.max_outer = trial ? 1 : o->max_cycles;
    B.coarse_sweeps =
        o->coarse_sweeps > 0 ? o->coarse_sweeps : default_coarse_sweeps(B.L[B.nlev - 1].n, B.nlev);
    B.use_field_in = D.field_in ? 1 : 0;
    B.trial = trial ? 1 : 0;
    B.tol = trial ? 1e-300 : tol;
    B.delta = D.delta;
    B.field = D.field;
    B.force = D.force;
    total += box_bytes(B.L, B.nlev);
  }
  if (total > ctx->bpool_bytes) {
    if (ctx->bpool) (void)hipFree(ctx->bpool);
    ctx->bpool = nullptr;
    ctx->bpool_bytes = 0;
    HIPCHK(hipMalloc(&ctx->bpool, total));
    ctx->bpool_bytes = total;
  }
  if (nb > ctx->bcap) {
    if (ctx->bdev) (void)hipFree(ctx->bdev);
    if (ctx->bout) (void)hipFree(ctx->bout);
    ctx->bdev = nullptr;
    ctx->bout = nullptr;
    HIPCHK(hipMalloc((void**)&ctx->bdev, sizeof(BoxDev) * nb));
    HIPCHK(hipMalloc((void**)&ctx->bout, sizeof(BoxOut) * nb));
    ctx->bcap = nb;
  }
  char* base = (char*)ctx->bpool;
  auto take = [&](size_t bytes) {
    char* p = base;
    base += (bytes + 255) & ~(size_t)255;
    return p;
  };
  for (int b = 0; b < nb; ++b) {
    BoxDev& B = host[b];
    B.w = (double*)take(8 * (size_t)(2 * B.L[0].half));
    for (int l = 0; l < B.nlev; ++l) {
      size_t bytes = 4 * (size_t)(2 * B.L[l].half);
      B.e[l] = (float*)take(bytes);
      B.X[l] = (float*)take(bytes);
      B.rho[l] = (float*)take(bytes);
      B.dens[l] = (float*)take(bytes);
      if (l > 0) B.eR[l] = (float*)take(bytes);
    }
  }
  HIPCHK(hipMemcpyAsync(ctx->bdev, host.data(), sizeof(BoxDev) * nb, hipMemcpyHostToDevice,
                        ctx->stream));
  return MG_OK;
}

// Team plan for a grid of G resident workgroups.  team_mode 1: one team per
// box (when boxes <= G) with sizes that balance cells per workgroup, capped
// so that a workgroup keeps at least 32768 fine cells; team_mode 0 (or more
// boxes than workgroups): single-workgroup teams with a longest-first static
// list of boxes each.
struct BatchPlan {
  std::vector<int> order;
  std::vector<TeamDev> teams;
  std::vector<int2> wg;
  int parts = 0;
};

void plan_teams(const std::vector<BoxDev>& host, int G, int team_mode, BatchPlan& P) {
  const int nb = (int)host.size();
  std::vector<double> cost(nb);
  for (int b = 0; b < nb; ++b) cost[b] = double(host[b].L[0].half) * 2.0;
  P.order.clear();
  P.teams.clear();
  P.wg.clear();
  if (team_mode == 1 && nb <= G) {
    std::vector<int> t(nb, 1), cap(nb);
    for (int b = 0; b < nb; ++b) cap[b] = (int)std::max<double>(1.0, std::floor(cost[b] / 32768.0));
    int left = G - nb;
    while (left > 0) {
      int best = -1;
      double bc = 0.0;
      for (int b = 0; b < nb; ++b)
        if (t[b] < cap[b] && cost[b] / t[b] > bc) {
          bc = cost[b] / t[b];
          best = b;
        }
      if (best < 0) break;
      ++t[best];
      --left;
    }
    for (int b = 0; b < nb; ++b) {
      P.order.push_back(b);
      P.teams.push_back(TeamDev{t[b], b, 1, 0});
    }
  } else {
    const int nt = std::min(nb, G);
    std::vector<int> idx(nb);
    for (int b = 0; b < nb; ++b) idx[b] = b;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<double> load(nt, 0.0);
    std::vector<std::vector<int>> lists(nt);
    for (int b : idx) {
      int best = 0;
      for (int q = 1; q < nt; ++q)
        if (load[q] < load[best]) best = q;
      load[best] += cost[b];
      lists[best].push_back(b);
    }
    for (int q = 0; q < nt; ++q) {
      P.teams.push_back(TeamDev{1, (int)P.order.size(), (int)lists[q].size(), 0});
      for (int b : lists[q]) P.order.push_back(b);
    }
  }
  P.parts = 0;
  for (int q = 0; q < (int)P.teams.size(); ++q) {
    P.teams[q].part_off = P.parts;
    P.parts += 2 * P.teams[q].size;
    for (int r = 0; r < P.teams[q].size; ++r) P.wg.push_back(make_int2(q, r));
  }
}

template <int BS>
int batch_launch_bs(mg_ctx* ctx, const std::vector<BoxDev>& host, int team_mode, int* grid_out) {
  const int nb = (int)host.size();
  if (ctx->bdev_coop < 0) {
    int dev = 0, coop = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    ctx->bdev_coop = coop;
    ctx->bdev_cus = cus;
  }
  if (!ctx->bdev_coop) return fail(ctx, MG_EHIP, "batched solve needs cooperative launch support");
  const int oi = BS == 256 ? 0 : (BS == 512 ? 1 : 2);
  if (ctx->bocc[oi] == 0) {
    int per_cu = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched<BS>, BS, 0));
    if (per_cu < 1) return fail(ctx, MG_EHIP, "batched kernel cannot be resident");
    ctx->bocc[oi] = per_cu;
  }
  const int G = ctx->bocc[oi] * ctx->bdev_cus;
  BatchPlan P;
  plan_teams(host, G, team_mode, P);
  const int grid = (int)P.wg.size();
  if (grid < 1 || grid > G) return fail(ctx, MG_EHIP, "batched plan does not fit the device");
  const int need = std::max(std::max((int)P.order.size(), (int)P.teams.size()), grid);
  if (need > ctx->bplan_cap || P.parts > 2 * ctx->bplan_cap) {
    for (void** p : {(void**)&ctx->border, (void**)&ctx->bteams, (void**)&ctx->bwg,
                     (void**)&ctx->bctr, (void**)&ctx->bparts}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    ctx->bplan_cap = 0;
    const int cap = std::max(need, (P.parts + 1) / 2);
    HIPCHK(hipMalloc((void**)&ctx->border, sizeof(int) * cap));
    HIPCHK(hipMalloc((void**)&ctx->bteams, sizeof(TeamDev) * cap));
    HIPCHK(hipMalloc((void**)&ctx->bwg, sizeof(int2) * cap));
    HIPCHK(hipMalloc((void**)&ctx->bctr, sizeof(unsigned) * cap));
    HIPCHK(hipMalloc((void**)&ctx->bparts, sizeof(double) * 2 * cap));
    ctx->bplan_cap = cap;
  }
  if (!ctx->babort) HIPCHK(hipMalloc((void**)&ctx->babort, 256));
  HIPCHK(hipMemcpyAsync(ctx->border, P.order.data(), sizeof(int) * P.order.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->bteams, P.teams.data(), sizeof(TeamDev) * P.teams.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->bwg, P.wg.data(), sizeof(int2) * P.wg.size(), hipMemcpyHostToDevice,
                        ctx->stream));
  k_fill<unsigned><<<nblk((int64_t)P.teams.size()), kBlock, 0, ctx->stream>>>(
      ctx->bctr, (int64_t)P.teams.size(), 0u);
  k_fill<int><<<1, kBlock, 0, ctx->stream>>>(ctx->babort, 1, 0);
  LAUNCHCHK();
  // the host copies of the plan must outlive the asynchronous uploads
  HIPCHK(hipStreamSynchronize(ctx->stream));
  const BoxDev* a0 = ctx->bdev;
  const int* a1 = ctx->border;
  const TeamDev* a2 = ctx->bteams;
  const int2* a3 = ctx->bwg;
  BoxOut* a4 = ctx->bout;
  unsigned* a5 = ctx->bctr;
  double* a6 = ctx->bparts;
  int* a7 = ctx->babort;
  void* args[] = {(void*)&a0, (void*)&a1, (void*)&a2, (void*)&a3,
                  (void*)&a4, (void*)&a5, (void*)&a6, (void*)&a7};
  HIPCHK(hipLaunchCooperativeKernel((const void*)k_batched<BS>, dim3(grid), dim3(BS), args, 0,
                                    ctx->stream));
  if (grid_out) *grid_out = grid;
  (void)nb;
  return MG_OK;
}

// ---------------------------------------------------------------------------
// Grouped level launches (teams == 2): boxes of one (n, model) form a class,
// every level operation is one launch per class with the box in blockIdx.y.
// The outer FP64 steps of all boxes share one synchronisation; each box plans
// its own cycles and a control word switches it off when it is done.
// ---------------------------------------------------------------------------
struct GClass {
  int n, model, nlev, f;
  int first, count;  // range of the class-ordered table
};
// 4 packed cells per thread on level l (its rows hold a multiple of 4)
inline bool g_vec_rows(const Lev& L) { return L.nh % 4 == 0; }
// 4 coarse cells per thread between l and l + 1 (coarse side a multiple of 4)
inline bool g_vec_coarse(const Lev& Lc) { return Lc.n % 4 == 0; }

// first level run by the single-workgroup program (as mg_ctx_create does)
int fused_level(const Lev* L, int nlev) {
  int f = nlev;
  for (int q = 1; q < nlev; ++q)
    if (L[q].n <= kFuseN) {
      f = q;
      break;
    }
  if (f > nlev - 1) f = nlev - 1;
  if (f < 1) f = nlev;
  if (nlev - f > kMaxFused) f = nlev - kMaxFused;
  return f;
}

int g_grow(mg_ctx* ctx, int nb, int pstride) {
  if (nb > ctx->gcap || (int64_t)nb * pstride > ctx->gpart_cap) {
    for (void** p : {(void**)&ctx->gtab, (void**)&ctx->gctl, (void**)&ctx->gpart,
                     (void**)&ctx->gsum}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    if (ctx->ghsum) (void)hipHostFree(ctx->ghsum);
    ctx->ghsum = nullptr;
    ctx->gcap = 0;
    ctx->gpart_cap = 0;
    HIPCHK(hipMalloc((void**)&ctx->gtab, sizeof(GBox) * nb));
    HIPCHK(hipMalloc((void**)&ctx->gctl, sizeof(GCtl) * nb));
    HIPCHK(hipMalloc((void**)&ctx->gpart, sizeof(double) * (size_t)nb * pstride));
    HIPCHK(hipMalloc((void**)&ctx->gsum, sizeof(double) * nb));
    void* h = nullptr;
    HIPCHK(hipHostMalloc(&h, sizeof(double) * nb, hipHostMallocDefault));
    ctx->ghsum = (double*)h;
    ctx->gcap = nb;
    ctx->gpart_cap = (int64_t)nb * pstride;
  }
  if (!ctx->gfork) {
    for (int i = 0; i < mg_ctx::kGStreams; ++i) {
      HIPCHK(hipStreamCreateWithFlags(&ctx->gst[i], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&ctx->gjoin[i], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&ctx->gfork, hipEventDisableTiming));
  }
  return MG_OK;
}

// the class streams wait for the context's stream, and it for them
int g_fork(mg_ctx* ctx, int ns) {
  HIPCHK(hipEventRecord(ctx->gfork, ctx->stream));
  for (int i = 0; i < ns; ++i) HIPCHK(hipStreamWaitEvent(ctx->gst[i], ctx->gfork, 0));
  return MG_OK;
}
int g_join(mg_ctx* ctx, int ns) {
  for (int i = 0; i < ns; ++i) {
    HIPCHK(hipEventRecord(ctx->gjoin[i], ctx->gst[i]));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->gjoin[i], 0));
  }
  return MG_OK;
}

template <int M>
void g_smooth(mg_ctx* ctx, hipStream_t st, const GClass& K, const Lev& L, int it, int l,
              int sweeps) {
  const GBox* tab = ctx->gtab + K.first;
  const GCtl* ctl = ctx->gctl + K.first;
  const bool vec = g_vec_rows(L);
  // z-marching when the class's launch still has enough workgroups
  const int kt = ctx->smooth_march_kt;
  if (vec && kt > 0 && march_blocks(L, kt, 4) * (unsigned)K.count >= ctx->march_min_blocks) {
    for (int s = 0; s < sweeps; ++s)
      for (int colour = 0; colour < 2; ++colour)
        kg_smooth_kv<M><<<dim3(march_blocks(L, kt, 4), K.count), kBlock, 0, st>>>(tab, ctl, it, l,
                                                                                 colour, kt);
    return;
  }
  const unsigned bx = vec ? nblk(L.half / 4) : nblk(L.half);
  for (int s = 0; s < sweeps; ++s)
    for (int colour = 0; colour < 2; ++colour)
      kg_smooth<M><<<dim3(bx, K.count), kBlock, 0, st>>>(tab, ctl, it, l, colour,
                                                                  vec ? 1 : 0);
}

// one cycle of a class from level l down (the recursion of cycle32)
template <int M>
int g_cycle(mg_ctx* ctx, hipStream_t st, const GClass& K, const Lev* L,
            const mg_solver_opts* o, int it, int l, int type, bool rx) {
  const GBox* tab = ctx->gtab + K.first;
  const GCtl* ctl = ctx->gctl + K.first;
  if (l >= K.f) {
    OpList ops;
    gen_prog(ops, l - K.f, K.nlev - 1 - K.f, type, o->nu_pre, o->nu_post);
    if (ops.over || ops.n > kMaxOps) return fail(ctx, MG_EINVAL, "fused cycle program too long");
    FusedProg P;
    P.nops = ops.n;
    P.coarse_sweeps = o->coarse_sweeps > 0 ? o->coarse_sweeps
                                           : default_coarse_sweeps(L[K.nlev - 1].n, K.nlev);
    P.rx = rx ? 1 : 0;
    for (int q = 0; q < ops.n; ++q) P.op[q] = ops.op[q];
    kg_fused<M><<<K.count, kFusedThreads, 0, st>>>(tab, ctl, it, P);
    LAUNCHCHK();
    return MG_OK;
  }
  if (l == K.nlev - 1) {  // a grid that cannot be coarsened
    const int cap = o->coarse_sweeps > 0 ? o->coarse_sweeps : default_coarse_sweeps(L[0].n, 1);
    const int nu = o->nu_pre + o->nu_post;
    g_smooth<M>(ctx, st, K, L[l], it, l, cap > nu ? cap : nu);
    LAUNCHCHK();
    return MG_OK;
  }
  const Lev& Lc = L[l + 1];
  g_smooth<M>(ctx, st, K, L[l], it, l, o->nu_pre);
  const int skip1 = (M != CQ && o->nu_pre > 0) ? 1 : 0;
  const bool rvec = g_vec_coarse(Lc) && g_vec_rows(L[l]);
  // shifted coarse form (as in cycle32): the coarse correction starts at
  // zero, written by the restriction; the coarse level's linearisation
  // point changes, so its first visit forms R X again
  kg_down<M><<<dim3(rvec ? nblk(2 * Lc.half / 4) : nblk(2 * Lc.half), K.count), kBlock, 0,
               st>>>(tab, ctl, it, l, rx ? 1 : 0, skip1, rvec ? 1 : 0);
  LAUNCHCHK();
  if (type == MG_CYCLE_V) {
    ACHK(g_cycle<M>(ctx, st, K, L, o, it, l + 1, MG_CYCLE_V, true));
  } else if (type == MG_CYCLE_W) {
    ACHK(g_cycle<M>(ctx, st, K, L, o, it, l + 1, MG_CYCLE_W, true));
    ACHK(g_cycle<M>(ctx, st, K, L, o, it, l + 1, MG_CYCLE_W, false));
  } else {
    ACHK(g_cycle<M>(ctx, st, K, L, o, it, l + 1, MG_CYCLE_F, true));
    ACHK(g_cycle<M>(ctx, st, K, L, o, it, l + 1, MG_CYCLE_V, false));
  }
  if (g_vec_coarse(Lc)) {
    kg_up<M == CQ ? 0 : 1><<<dim3(nblk(2 * Lc.half / 4), K.count), kBlock, 0, st>>>(
        tab, ctl, it, l);
  } else {
    kg_up_block<<<dim3(nblk(2 * Lc.half), K.count), kBlock, 0, st>>>(tab, ctl, it, l);
  }
  g_smooth<M>(ctx, st, K, L[l], it, l, o->nu_post);
  LAUNCHCHK();
  return MG_OK;
}

template <int M>
int g_class_cycle(mg_ctx* ctx, hipStream_t st, const GClass& K, const Lev* L,
                  const mg_solver_opts* o, int it) {
  return g_cycle<M>(ctx, st, K, L, o, it, 0, o->cycle, it == 0);
}

// The whole batch: trial = one outer step of two cycles, no outputs (tuning).
int grouped_solve(mg_ctx* ctx, int nb, const mg_box_desc* boxes, const mg_solver_opts* o,
                  double tol, bool trial, std::vector<BoxOut>& outs) {
  // classes by (n, model), table in class order
  std::map<std::pair<int, int>, std::vector<int>> byc;
  for (int b = 0; b < nb; ++b) {
    const mg_box_desc& D = boxes[b];
    if (D.n < 8 || (D.n & 1) || D.n > 1024 || !D.delta || !D.field)
      return fail(ctx, MG_EINVAL, "mg_solve_batched: box " + std::to_string(b) +
                                      " needs even 8 <= n <= 1024 and delta/field");
    if (D.model < MG_FR || D.model > MG_CQ)
      return fail(ctx, MG_EINVAL, "mg_solve_batched: unknown model");
    byc[{D.n, D.model}].push_back(b);
  }
  std::vector<GClass> cls;
  std::vector<int> order;
  std::vector<GBox> host(nb);
  std::vector<Lev> levs;  // levels of each class (kMaxLevB per class)
  size_t total = 0;
  int pstride = 1;
  for (auto& kv : byc) {
    GClass K;
    memset(&K, 0, sizeof K);
    K.n = kv.first.first;
    K.model = kv.first.second;
    Lev L[kMaxLevB];
    K.nlev = box_levels(K.n, L);
    K.f = fused_level(L, K.nlev);
    K.first = (int)order.size();
    K.count = (int)kv.second.size();
    for (int b : kv.second) order.push_back(b);
    for (int l = 0; l < kMaxLevB; ++l) levs.push_back(L[l]);
    cls.push_back(K);
    total += (size_t)K.count * box_bytes(L, K.nlev);
    pstride = std::max(pstride, (int)nblk(2 * L[0].half));
  }
  if (total > ctx->bpool_bytes) {
    if (ctx->bpool) (void)hipFree(ctx->bpool);
    ctx->bpool = nullptr;
    ctx->bpool_bytes = 0;
    HIPCHK(hipMalloc(&ctx->bpool, total));
    ctx->bpool_bytes = total;
  }
  ACHK(g_grow(ctx, nb, pstride));
  const int ns = std::min((int)cls.size(), (int)mg_ctx::kGStreams);
  auto cst = [&](size_t c) { return ctx->gst[c % ns]; };
  // whatever path leaves this function, the context's stream ends up waiting
  // for the class streams (after a normal end they are already idle)
  struct JoinAtExit {
    mg_ctx* c;
    int ns;
    ~JoinAtExit() { (void)g_join(c, ns); }
  } join_at_exit{ctx, ns};
  char* base = (char*)ctx->bpool;
  auto take = [&](size_t bytes) {
    char* p = base;
    base += (bytes + 255) & ~(size_t)255;
    return p;
  };
  for (size_t c = 0; c < cls.size(); ++c) {
    const GClass& K = cls[c];
    const Lev* L = &levs[c * kMaxLevB];
    for (int q = 0; q < K.count; ++q) {
      const int b = order[K.first + q];
      const mg_box_desc& D = boxes[b];
      GBox& B = host[K.first + q];
      memset(&B, 0, sizeof B);
      ACHK(make_consts(ctx, D.model, &D.params, D.n, &B.C));
      B.nlev = K.nlev;
      B.fused_from = K.f;
      B.use_field_in = (D.field_in && !trial) ? 1 : 0;
      for (int l = 0; l < K.nlev; ++l) {
        B.L[l] = L[l];
        B.h2[l] = float(lev_h2(l));
      }
      B.delta = D.delta;
      B.field = D.field;
      B.force = trial ? nullptr : D.force;
      B.w = (double*)take(8 * (size_t)(2 * L[0].half));
      for (int l = 0; l < K.nlev; ++l) {
        const size_t bytes = 4 * (size_t)(2 * L[l].half);
        B.e[l] = (float*)take(bytes);
        B.X[l] = (float*)take(bytes);
        B.rho[l] = (float*)take(bytes);
        B.dens[l] = (float*)take(bytes);
        if (l > 0) B.eR[l] = (float*)take(bytes);
      }
      if (K.f < K.nlev) {
        B.F.nlev = K.nlev - K.f;
        for (int q2 = 0; q2 < B.F.nlev; ++q2) {
          const int l = K.f + q2;
          B.F.L[q2] = L[l];
          B.F.h2[q2] = B.h2[l];
          B.F.e[q2] = B.e[l];
          B.F.X[q2] = B.X[l];
          B.F.dens[q2] = B.dens[l];
          B.F.rho[q2] = B.rho[l];
          B.F.eR[q2] = B.eR[l];
        }
      }
    }
  }
  HIPCHK(hipMemcpyAsync(ctx->gtab, host.data(), sizeof(GBox) * nb, hipMemcpyHostToDevice,
                        ctx->stream));
  // inputs packed, density pyramids, background norms
  ACHK(g_fork(ctx, ns));
  for (size_t c = 0; c < cls.size(); ++c) {
    const GClass& K = cls[c];
    const Lev* L = &levs[c * kMaxLevB];
    const GBox* tab = ctx->gtab + K.first;
    double* part = ctx->gpart + (int64_t)K.first * pstride;
    const dim3 g0(nblk(2 * L[0].half), K.count);
    hipStream_t st = cst(c);
    if (K.model == MG_FR) kg_pack<FR><<<g0, kBlock, 0, st>>>(tab, part, pstride);
    else if (K.model == MG_SYMMETRON) kg_pack<SYM><<<g0, kBlock, 0, st>>>(tab, part, pstride);
    else kg_pack<CQ><<<g0, kBlock, 0, st>>>(tab, part, pstride);
    if (K.model != MG_FR)
      for (int l = 0; l + 1 < K.nlev; ++l)
        kg_restrict_dens<<<dim3(nblk(2 * L[l + 1].half), K.count), kBlock, 0, st>>>(tab, l);
    LAUNCHCHK();
  }
  // per-box sums of the partials (class streams), then joined and copied out
  auto box_sums = [&](std::vector<double>& s) -> int {
    for (size_t c = 0; c < cls.size(); ++c) {
      const GClass& K = cls[c];
      const Lev* L = &levs[c * kMaxLevB];
      kg_sum_box<<<K.count, 256, 0, cst(c)>>>(ctx->gpart + (int64_t)K.first * pstride, pstride,
                                               (int)nblk(2 * L[0].half), ctx->gsum + K.first);
    }
    LAUNCHCHK();
    ACHK(g_join(ctx, ns));
    HIPCHK(hipMemcpyAsync(ctx->ghsum, ctx->gsum, sizeof(double) * nb, hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    s.assign(ctx->ghsum, ctx->ghsum + nb);
    return MG_OK;
  };
  std::vector<double> sums;
  ACHK(box_sums(sums));
  std::vector<double> eps(nb), rel(nb, 0.0), rel_prev(nb, -1.0), mcell(nb);
  std::vector<int> k_prev(nb, 0), outer(nb, 0), vc(nb, 0), status(nb, 0), done(nb, 0);
  for (int i = 0; i < nb; ++i) {
    const GBox& B = host[i];
    mcell[i] = 2.0 * double(B.L[0].half);
    eps[i] = bg_norm_of(B.C, sqrt(sums[i] / mcell[i]));
  }
  const int max_outer = trial ? 1 : o->max_cycles;
  std::vector<GCtl> ctl(nb);
  for (int i = 0; i < nb; ++i) ctl[i] = GCtl{1, 0, 0, 0};
  for (;;) {
    HIPCHK(hipMemcpyAsync(ctx->gctl, ctl.data(), sizeof(GCtl) * nb, hipMemcpyHostToDevice,
                          ctx->stream));
    ACHK(g_fork(ctx, ns));
    for (size_t c = 0; c < cls.size(); ++c) {
      const GClass& K = cls[c];
      const Lev* L = &levs[c * kMaxLevB];
      const GBox* tab = ctx->gtab + K.first;
      const GCtl* gc = ctx->gctl + K.first;
      double* part = ctx->gpart + (int64_t)K.first * pstride;
      const dim3 g0(nblk(2 * L[0].half), K.count);
      hipStream_t st = cst(c);
      kg_update<<<g0, kBlock, 0, st>>>(tab, gc);
      if (K.model == MG_FR) kg_outer<FR><<<g0, kBlock, 0, st>>>(tab, gc, part, pstride);
      else if (K.model == MG_SYMMETRON) kg_outer<SYM><<<g0, kBlock, 0, st>>>(tab, gc, part, pstride);
      else kg_outer<CQ><<<g0, kBlock, 0, st>>>(tab, gc, part, pstride);
    }
    LAUNCHCHK();
    ACHK(box_sums(sums));
    int kmax = 0;
    for (int i = 0; i < nb; ++i) {
      if (done[i]) {
        ctl[i] = GCtl{0, 0, 0, 0};
        continue;
      }
      rel[i] = sqrt(sums[i] / mcell[i]) / eps[i];
      int kb = 0;
      if (!std::isfinite(rel[i])) {
        status[i] = MG_ENAN;
        done[i] = 1;
      } else if (!trial && rel[i] <= tol) {
        done[i] = 1;
      } else if (outer[i] >= max_outer) {
        if (!trial) status[i] = MG_ENOCONV;
        done[i] = 1;
      } else {
        kb = trial ? 2
                   : plan_cycles(o->inner_cycles, rel[i], rel_prev[i], k_prev[i], tol,
                                 (int64_t)mcell[i]);
      }
      ctl[i] = GCtl{kb > 0 ? 1 : 0, kb, kb > 0 ? 1 : 0, 0};
      if (kb > 0) {
        vc[i] += kb;
        rel_prev[i] = rel[i];
        k_prev[i] = kb;
        ++outer[i];
      }
      kmax = std::max(kmax, kb);
    }
    if (kmax == 0) break;
    HIPCHK(hipMemcpyAsync(ctx->gctl, ctl.data(), sizeof(GCtl) * nb, hipMemcpyHostToDevice,
                          ctx->stream));
    ACHK(g_fork(ctx, ns));
    for (int it = 0; it < kmax; ++it)
      for (size_t c = 0; c < cls.size(); ++c) {
        const GClass& K = cls[c];
        const Lev* L = &levs[c * kMaxLevB];
        hipStream_t st = cst(c);
        if (K.model == MG_FR) ACHK(g_class_cycle<FR>(ctx, st, K, L, o, it));
        else if (K.model == MG_SYMMETRON) ACHK(g_class_cycle<SYM>(ctx, st, K, L, o, it));
        else ACHK(g_class_cycle<CQ>(ctx, st, K, L, o, it));
      }
    ACHK(g_join(ctx, ns));  // before the control words are rewritten
  }
  if (!trial) {
    ACHK(g_fork(ctx, ns));
    for (size_t c = 0; c < cls.size(); ++c) {
      const GClass& K = cls[c];
      const Lev* L = &levs[c * kMaxLevB];
      const GBox* tab = ctx->gtab + K.first;
      const dim3 g0(nblk(2 * L[0].half), K.count);
      hipStream_t st = cst(c);
      if (K.model == MG_FR) {
        kg_unpack<FR><<<g0, kBlock, 0, st>>>(tab);
        kg_force<FR><<<g0, kBlock, 0, st>>>(tab);
      } else if (K.model == MG_SYMMETRON) {
        kg_unpack<SYM><<<g0, kBlock, 0, st>>>(tab);
        kg_force<SYM><<<g0, kBlock, 0, st>>>(tab);
      } else {
        kg_unpack<CQ><<<g0, kBlock, 0, st>>>(tab);
        kg_force<CQ><<<g0, kBlock, 0, st>>>(tab);
      }
    }
    LAUNCHCHK();
    ACHK(g_join(ctx, ns));
  }
  // the host table must outlive its asynchronous upload
  HIPCHK(hipStreamSynchronize(ctx->stream));
  outs.assign(nb, BoxOut());
  for (int i = 0; i < nb; ++i) {
    BoxOut& O = outs[order[i]];
    O.outer = outer[i];
    O.vcycles = vc[i];
    O.status = status[i];
    O.rel = rel[i];
  }
  return MG_OK;
}

int batch_launch(mg_ctx* ctx, const std::vector<BoxDev>& host, int block, int team_mode) {
  if (block == 256) return batch_launch_bs<256>(ctx, host, team_mode, nullptr);
  if (block == 512) return batch_launch_bs<512>(ctx, host, team_mode, nullptr);
  return batch_launch_bs<1024>(ctx, host, team_mode, nullptr);
}

// outputs of the last launch; MG_EHIP if a team barrier timed out
int batch_collect(mg_ctx* ctx, int nb, std::vector<BoxOut>& outs) {
  outs.resize(nb);
  int abort_flag = 0;
  HIPCHK(hipMemcpyAsync(outs.data(), ctx->bout, sizeof(BoxOut) * nb, hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipMemcpyAsync(&abort_flag, ctx->babort, sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (abort_flag) return fail(ctx, MG_EHIP, "batched solve: a team barrier timed out");
  return MG_OK;
}

std::string batch_key(mg_ctx* ctx, int nb, const mg_box_desc* boxes, const mg_solver_opts* o) {
  std::vector<std::string> parts;
  for (int b = 0; b < nb; ++b)
    parts.push_back(std::to_string(boxes[b].n) + (boxes[b].model == MG_FR ? "f" :
                                                  boxes[b].model == MG_SYMMETRON ? "s" : "q"));
  std::sort(parts.begin(), parts.end());
  // the multiset of (n, model): counts matter for the team split
  std::string k = "batched2:";
  for (size_t q = 0; q < parts.size();) {
    size_t r = q;
    while (r < parts.size() && parts[r] == parts[q]) ++r;
    k += parts[q] + "x" + std::to_string(r - q) + ",";
    q = r;
  }
  if (ctx->arch.empty()) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      ctx->arch = prop.gcnArchName;
  }
  if (!ctx->arch.empty()) k += ":" + ctx->arch;
  k += ":V(" + std::to_string(o->nu_pre) + "," + std::to_string(o->nu_post) + ")c" +
       std::to_string(o->cycle);
  return k;
}

std::string cache_path() {
  const char* e = getenv("MGGPU_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = getenv("HOME");
  return std::string(h && *h ? h : "/tmp") + "/.mggpu_tune.json";
}

// cache file: one JSON object, "key": [block, vec, team, ms] per line
bool cache_lookup(const std::string& key, int* block, int* vec, int* team) {
  std::ifstream f(cache_path());
  if (!f) return false;
  std::string line;
  std::string q = "\"" + key + "\":";
  while (std::getline(f, line)) {
    size_t p = line.find(q);
    if (p == std::string::npos) continue;
    int b = 0, v = 0, t = 0;
    if (sscanf(line.c_str() + p + q.size(), " [%d, %d, %d", &b, &v, &t) == 3 &&
        (b == 256 || b == 512 || b == 1024) && (v == 0 || v == 1) && (t >= 0 && t <= 2)) {
      *block = b;
      *vec = v;
      *team = t;
      return true;
    }
  }
  return false;
}

void cache_store(const std::string& key, int block, int vec, int team, double ms) {
  std::map<std::string, std::string> ent;
  {
    std::ifstream f(cache_path());
    std::string line;
    while (f && std::getline(f, line)) {
      size_t a = line.find('"'), b = line.find("\":");
      if (a == std::string::npos || b == std::string::npos || b <= a) continue;
      size_t c = line.find('[', b), d = line.find(']', b);
      if (c == std::string::npos || d == std::string::npos) continue;
      ent[line.substr(a + 1, b - a - 1)] = line.substr(c, d - c + 1);
    }
  }
  std::ostringstream v;
  v << "[" << block << ", " << vec << ", " << team << ", " << ms << "]";
  ent[key] = v.str();
  std::string tmp = cache_path() + ".tmp";
  std::ofstream f(tmp);
  if (!f) return;
  f << "{\n";
  size_t i = 0;
  for (auto& kv : ent) f << "  \"" << kv.first << "\": " << kv.second << (++i < ent.size() ? ",\n" : "\n");
  f << "}\n";
  f.close();
  (void)rename(tmp.c_str(), cache_path().c_str());
}

}  // namespace

extern "C" {

int mg_batched_tune(mg_ctx* ctx, int n_box, const mg_box_desc* boxes, const mg_solver_opts* opts,
                    int* block_out, int* vec_out) {
  if (!ctx) return MG_EINVAL;
  ACHK(check_opts(ctx, opts));
  if (n_box < 1 || !boxes) return fail(ctx, MG_EINVAL, "mg_batched_tune: no boxes");
  // time one outer step (2 FP32 cycles) of the whole batch per candidate
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  double best = 1e300;
  int bb = 256, bv = 1, bt = 2;
  std::vector<BoxDev> host;
  std::vector<BoxOut> outs;
  // the grouped level launches (teams == 2)
  int rc = grouped_solve(ctx, n_box, boxes, opts, 1e-300, true, outs);  // warm-up
  {
    if (rc == MG_OK) {
      HIPCHK(hipEventRecord(t0, ctx->stream));
      rc = grouped_solve(ctx, n_box, boxes, opts, 1e-300, true, outs);
      HIPCHK(hipEventRecord(t1, ctx->stream));
      HIPCHK(hipEventSynchronize(t1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, t0, t1));
      if (rc == MG_OK && ms < best) {
        best = ms;
        bb = 256;
        bv = 1;
        bt = 2;
      }
    }
  }
  // The persistent launch is cooperative, and any cooperative launch slows
  // the grouped path for the rest of the process: the 64-box 64^3..128^3
  // batch then takes 16.6 instead of 11.8 ms, about its time with the class
  // streams serialised.  So it is only tried for batches too small to fill
  // the chip with level launches (below 8M cells in all), where it can win.
  int64_t batch_cells = 0;
  for (int b = 0; b < n_box; ++b) batch_cells += (int64_t)boxes[b].n * boxes[b].n * boxes[b].n;
  if (batch_cells < ((int64_t)8 << 20))
    for (int vec = 0; vec < 2 && rc == MG_OK; ++vec) {
      rc = batch_setup(ctx, n_box, boxes, opts, 1e-300, true, vec, host);
      for (int team = 0; team < 2 && rc == MG_OK; ++team)
        for (int ci = 0; ci < 3 && rc == MG_OK; ++ci) {
          const int blk = kTileBlocks[ci];
          rc = batch_launch(ctx, host, blk, team);  // warm-up
          if (rc == MG_OK) rc = batch_collect(ctx, n_box, outs);
          if (rc != MG_OK) break;
          HIPCHK(hipEventRecord(t0, ctx->stream));
          rc = batch_launch(ctx, host, blk, team);
          if (rc != MG_OK) break;
          HIPCHK(hipEventRecord(t1, ctx->stream));
          HIPCHK(hipEventSynchronize(t1));
          rc = batch_collect(ctx, n_box, outs);
          if (rc != MG_OK) break;
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, t0, t1));
          if (ms < best) {
            best = ms;
            bb = blk;
            bv = vec;
            bt = team;
          }
        }
    }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc != MG_OK) return rc;
  std::string key = batch_key(ctx, n_box, boxes, opts);
  cache_store(key, bb, bv, bt, best);
  ctx->bkey = key;
  ctx->bpinned = false;
  ctx->bblock = bb;
  ctx->bvec = bv;
  ctx->bteam = bt;
  if (block_out) *block_out = bb;
  if (vec_out) *vec_out = bv;
  return MG_OK;
}

int mg_solve_batched(mg_ctx* ctx, int n_box, const mg_box_desc* boxes, const mg_solver_opts* opts,
                     double tol, mg_stats* per_box) {
  if (!ctx) return MG_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  ACHK(check_opts(ctx, opts));
  if (n_box < 1 || !boxes) return fail(ctx, MG_EINVAL, "mg_solve_batched: no boxes");
  if (!(tol > 0.0)) return fail(ctx, MG_EINVAL, "mg_solve_batched: tol must be > 0");
  if (opts->precision != MG_FP32_REFINED)
    return fail(ctx, MG_EINVAL, "mg_solve_batched: runs the FP32-refined scheme");
  if (opts->fixed_cycles > 0)
    return fail(ctx, MG_EINVAL, "mg_solve_batched: iterates to tol (fixed_cycles must be 0)");
  // tile shape: this context's last tuning for the same batch shape, else the
  // cache file, else tune now
  std::string key = batch_key(ctx, n_box, boxes, opts);
  int blk = 0, vec = -1, team = -1;
  if (ctx->bpinned || (ctx->bkey == key && ctx->bblock > 0)) {
    blk = ctx->bblock;
    vec = ctx->bvec;
    team = ctx->bteam;
  } else if (cache_lookup(key, &blk, &vec, &team)) {
    ctx->bkey = key;
    ctx->bblock = blk;
    ctx->bvec = vec;
    ctx->bteam = team;
  } else {
    ACHK(mg_batched_tune(ctx, n_box, boxes, opts, &blk, &vec));
    team = ctx->bteam;
  }
  std::vector<BoxOut> outs;
  if (team == 2) {
    ACHK(grouped_solve(ctx, n_box, boxes, opts, tol, false, outs));
  } else {
    std::vector<BoxDev> host;
    ACHK(batch_setup(ctx, n_box, boxes, opts, tol, false, vec, host));
    ACHK(batch_launch(ctx, host, blk, team));
    ACHK(batch_collect(ctx, n_box, outs));
  }
  double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int rc = MG_OK;
  for (int b = 0; b < n_box; ++b) {
    if (outs[b].status == MG_ENAN) rc = MG_ENAN;
    else if (outs[b].status == MG_ENOCONV && rc == MG_OK) rc = MG_ENOCONV;
    if (per_box) {
      memset(&per_box[b], 0, sizeof(mg_stats));
      per_box[b].cycles = outs[b].outer;
      per_box[b].vcycles = outs[b].vcycles;
      per_box[b].status = outs[b].status;
      per_box[b].rel_resid = outs[b].rel;
      per_box[b].ms_total = ms;
    }
  }
  if (rc != MG_OK)
    ctx->err = rc == MG_ENAN ? "mg_solve_batched: non-finite residual in a box"
                             : "mg_solve_batched: a box reached max_cycles";
  return rc;
}

int mg_batched_config(const mg_ctx* ctx, int* block, int* vec, int* teams) {
  if (!ctx || !block || !vec || !teams) return MG_EINVAL;
  *block = ctx->bblock;
  *vec = ctx->bvec;
  *teams = ctx->bteam;
  return MG_OK;
}

int mg_batched_set_config(mg_ctx* ctx, int block, int vec, int teams) {
  if (!ctx) return MG_EINVAL;
  if (block == 0) {
    ctx->bpinned = false;
    ctx->bkey.clear();
    ctx->bblock = 0;
    ctx->bvec = -1;
    ctx->bteam = -1;
    return MG_OK;
  }
  if ((block != 256 && block != 512 && block != 1024) || (vec != 0 && vec != 1) ||
      (teams < 0 || teams > 2))
    return fail(ctx, MG_EINVAL, "mg_batched_set_config: block 256/512/1024, vec 0/1, teams 0/1/2");
  ctx->bpinned = true;
  ctx->bblock = block;
  ctx->bvec = vec;
  ctx->bteam = teams;
  return MG_OK;
}

}  // extern "C"
