// mg_kernels.h -- generic HIP kernels of the multigrid hot path (gfx950).
//
// Data layout: every level-l grid of n^3 cells is stored red/black packed,
// colour c = (i+j+k)&1 holding the n^3/2 cells of that colour as
//   P_c[(k*n + j)*nh + ih],  i = 2*ih + ((j + k + c) & 1),  nh = n/2,
// colour 0 first, colour 1 at offset n^3/2.  A half-sweep then reads one
// contiguous array (the other colour) and writes another; the six
// neighbours of (ih,j,k) in colour c are, in the other colour's array,
// (ih-1+s, j, k), (ih+s, j, k), (ih, j+-1, k), (ih, j, k+-1), s = (j+k+c)&1.
// The 8 children of coarse cell (I,J,K) are ih = I in both colours of
// rows j = 2J+b, k = 2K+d, so restriction reads 8 coalesced streams.
#pragma once
#include "mg_device.h"

namespace mgg {

// Division by a run-time constant d (1 <= d < 2^31) as a multiply-high and
// a shift (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994): l = ceil(log2 d), m = floor(2^32 (2^l - d)/d) + 1,
// x / d = (mulhi(x, m) + x) >> l for every 32-bit x.
struct FastDiv {
  uint32_t m, s;
  __host__ static FastDiv make(uint32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    FastDiv f;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    f.s = l;
    return f;
  }
  __device__ __forceinline__ uint32_t div(uint32_t x) const {
    uint32_t t = __umulhi(x, m);
    return (uint32_t)(((uint64_t)t + x) >> s);
  }
};

// One level.  Cell counts stay below 2^32 (n <= 1600), so all index
// arithmetic is 32-bit.
struct Lev {
  int n;          // cells per side
  int nh;         // n / 2
  int64_t half;   // n^3 / 2: cells of one colour
  FastDiv dnh;    // division by nh
  FastDiv dn;     // division by n
};

constexpr int kBlock = 256;
constexpr int kMaxFused = 6;   // levels handled by the single-workgroup kernel
constexpr int kMaxOps = 96;    // operations in a fused cycle program

// Block index remapped so that each of the 8 XCDs (blocks are dealt to XCDs
// round-robin) works on one contiguous slab of rows: stencil neighbours in
// j and k then hit the same XCD's L2.
__device__ __forceinline__ int64_t xcd_block() {
  uint32_t b = blockIdx.x, nb = gridDim.x;
  uint32_t per = nb >> 3;
  if (b < (per << 3)) b = (b & 7u) * per + (b >> 3);
  return (int64_t)b;
}
__device__ __forceinline__ int64_t gid() { return xcd_block() * blockDim.x + threadIdx.x; }

__device__ __forceinline__ void dec(int64_t g64, const Lev& L, int& ih, int& j, int& k) {
  uint32_t g = (uint32_t)g64;
  uint32_t r = L.dnh.div(g);
  ih = (int)(g - r * (uint32_t)L.nh);
  uint32_t kk = L.dn.div(r);
  j = (int)(r - kk * (uint32_t)L.n);
  k = (int)kk;
}
// natural (i, j, k) of a natural linear index
__device__ __forceinline__ void dec_nat(int64_t g64, const Lev& L, int& i, int& j, int& k) {
  uint32_t g = (uint32_t)g64;
  uint32_t r = L.dn.div(g);
  i = (int)(g - r * (uint32_t)L.n);
  uint32_t kk = L.dn.div(r);
  j = (int)(r - kk * (uint32_t)L.n);
  k = (int)kk;
}
__device__ __forceinline__ uint32_t prow(const Lev& L, int j, int k) {
  return ((uint32_t)k * (uint32_t)L.n + (uint32_t)j) * (uint32_t)L.nh;
}
// packed index (including the colour offset) of natural cell (i,j,k)
__device__ __forceinline__ uint32_t pk_of(const Lev& L, int i, int j, int k) {
  return (uint32_t)((i + j + k) & 1) * (uint32_t)L.half + prow(L, j, k) + (uint32_t)(i >> 1);
}

template <typename T>
__device__ __forceinline__ T nbsum(const Lev& L, const T* __restrict__ o, int ih, int j, int k,
                                   int s) {
  int xm = ih - 1 + s;
  if (xm < 0) xm += L.nh;
  int xp = ih + s;
  if (xp >= L.nh) xp -= L.nh;
  int jm = (j == 0) ? L.n - 1 : j - 1, jp = (j == L.n - 1) ? 0 : j + 1;
  int km = (k == 0) ? L.n - 1 : k - 1, kp = (k == L.n - 1) ? 0 : k + 1;
  uint32_t r = prow(L, j, k);
  return (o[r + xm] + o[r + xp]) + (o[prow(L, jm, k) + ih] + o[prow(L, jp, k) + ih]) +
         (o[prow(L, j, km) + ih] + o[prow(L, j, kp) + ih]);
}

// ---------------------------------------------------------------------------
// Vector access: V consecutive packed cells of one row per thread (16-byte
// loads: 4 floats or 2 doubles), so each wave keeps more bytes in flight.
// Requires nh % V == 0 (rows then start on V-aligned offsets).
// ---------------------------------------------------------------------------
template <typename T>
struct Vec;
template <>
struct Vec<float> {
  static constexpr int V = 4;
  using type = float4;
};
template <>
struct Vec<double> {
  static constexpr int V = 2;
  using type = double2;
};
// N consecutive elements in 16-byte (or, for 2 floats, 8-byte) accesses;
// p must be aligned to the access size.
template <typename T, int N>
__device__ __forceinline__ void ldn(const T* __restrict__ p, T* out) {
  if constexpr (N * sizeof(T) == 8 && sizeof(T) == 4) {
    float2 v = *reinterpret_cast<const float2*>(p);
    out[0] = v.x; out[1] = v.y;
  } else {
    using VT = typename Vec<T>::type;
    constexpr int P = Vec<T>::V;
    static_assert(N % P == 0, "whole 16-byte accesses");
#pragma unroll
    for (int c = 0; c < N / P; ++c) {
      VT v = *reinterpret_cast<const VT*>(p + c * P);
      if constexpr (P == 4) {
        out[4 * c] = v.x; out[4 * c + 1] = v.y; out[4 * c + 2] = v.z; out[4 * c + 3] = v.w;
      } else {
        out[2 * c] = v.x; out[2 * c + 1] = v.y;
      }
    }
  }
}
template <typename T, int N>
__device__ __forceinline__ void stn(T* __restrict__ p, const T* in) {
  if constexpr (N * sizeof(T) == 8 && sizeof(T) == 4) {
    float2 v;
    v.x = in[0]; v.y = in[1];
    *reinterpret_cast<float2*>(p) = v;
  } else {
    using VT = typename Vec<T>::type;
    constexpr int P = Vec<T>::V;
    static_assert(N % P == 0, "whole 16-byte accesses");
#pragma unroll
    for (int c = 0; c < N / P; ++c) {
      VT v;
      if constexpr (P == 4) {
        v.x = in[4 * c]; v.y = in[4 * c + 1]; v.z = in[4 * c + 2]; v.w = in[4 * c + 3];
      } else {
        v.x = in[2 * c]; v.y = in[2 * c + 1];
      }
      *reinterpret_cast<VT*>(p + c * P) = v;
    }
  }
}
template <typename T>
__device__ __forceinline__ void ldv(const T* __restrict__ p, T* out) {
  ldn<T, Vec<T>::V>(p, out);
}
template <typename T>
__device__ __forceinline__ void stv(T* __restrict__ p, const T* in) {
  stn<T, Vec<T>::V>(p, in);
}
template <typename T, int N>
__device__ __forceinline__ void ldn_nt(const T* __restrict__ p, T* out);
template <typename T, int N>
__device__ __forceinline__ void stn_nt(T* __restrict__ p, const T* in);
// Streaming (non-temporal) 16-byte accesses for data touched once per pass:
// the cache hint keeps them from displacing lines that neighbouring threads
// still reuse (the other colour's rows and planes).
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ void ldv_nt(const T* __restrict__ p, T* out) {
  if constexpr (sizeof(T) == 4) {
    nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
  } else {
    nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    out[0] = v[0]; out[1] = v[1];
  }
}
template <typename T>
__device__ __forceinline__ void stv_nt(T* __restrict__ p, const T* in) {
  if constexpr (sizeof(T) == 4) {
    nt_f4 v = {in[0], in[1], in[2], in[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_f4*>(p));
  } else {
    nt_d2 v = {in[0], in[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_d2*>(p));
  }
}
typedef float nt_f2 __attribute__((ext_vector_type(2)));
template <typename T, int N>
__device__ __forceinline__ void ldn_nt(const T* __restrict__ p, T* out) {
  if constexpr (N * sizeof(T) == 8 && sizeof(T) == 4) {
    nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
    out[0] = v[0];
    out[1] = v[1];
  } else {
    constexpr int P = Vec<T>::V;
    static_assert(N % P == 0, "whole 16-byte accesses");
#pragma unroll
    for (int c = 0; c < N / P; ++c) ldv_nt<T>(p + c * P, out + c * P);
  }
}
template <typename T, int N>
__device__ __forceinline__ void stn_nt(T* __restrict__ p, const T* in) {
  if constexpr (N * sizeof(T) == 8 && sizeof(T) == 4) {
    nt_f2 v = {in[0], in[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_f2*>(p));
  } else {
    constexpr int P = Vec<T>::V;
    static_assert(N % P == 0, "whole 16-byte accesses");
#pragma unroll
    for (int c = 0; c < N / P; ++c) stv_nt<T>(p + c * P, in + c * P);
  }
}
// ---------------------------------------------------------------------------
// Storage of the finest level's per-cell data of the correction problem (the
// linearisation point X and the right-hand side rho): FP32, or 16-bit floats
// with a power-of-two scale (enc on the way in, dec = 1/enc on the way out).
// The kernels that read them decode identically, so the FP32 inner problem
// is exactly the correction equation at the decoded X; the FP64 outer
// residual is computed from the FP64 field and does not see the rounding.
// ---------------------------------------------------------------------------
typedef _Float16 h16;
typedef _Float16 nt_h4 __attribute__((ext_vector_type(4)));
struct Store {
  float x_enc, x_dec;  // X: f(R) 1024/wbar, symmetron 1024 (unused for FP32)
  float r_enc, r_dec;  // rho: 2^s chosen per outer step (unused for FP32)
};
// 4 consecutive stored cells -> float (streaming load)
template <typename TS>
__device__ __forceinline__ void ld4s(const TS* __restrict__ p, float dec, float* out) {
  if constexpr (sizeof(TS) == 4) {
    ldv_nt<float>(reinterpret_cast<const float*>(p), out);
  } else {
    const nt_h4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_h4*>(p));
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = float(v[q]) * dec;
  }
}
// float -> 4 consecutive stored cells (streaming store)
template <typename TS>
__device__ __forceinline__ void st4s(TS* __restrict__ p, const float* in, float enc) {
  if constexpr (sizeof(TS) == 4) {
    stv_nt<float>(reinterpret_cast<float*>(p), in);
  } else {
    const nt_h4 v = {h16(in[0] * enc), h16(in[1] * enc), h16(in[2] * enc), h16(in[3] * enc)};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_h4*>(p));
  }
}
// N (= 4, or Vec<T>::V) consecutive stored cells -> T: float arithmetic reads
// FP32 or 16-bit storage, FP64 arithmetic FP64 storage
template <typename T, typename TS, int N>
__device__ __forceinline__ void ldNs(const TS* __restrict__ p, float dec, T* out) {
  if constexpr (sizeof(T) == 4) {
    static_assert(N == 4, "float cells come in fours");
    ld4s<TS>(p, dec, out);
  } else {
    ldn_nt<T, N>(p, out);
  }
}

// Neighbour sums of the V cells (ih0 .. ih0+V-1, j, k) of colour c from the
// other colour's array o; s = (j + k + c) & 1.  Same summation order as nbsum.
template <typename T, int V = Vec<T>::V>
__device__ __forceinline__ void nbsum_vec(const Lev& L, const T* __restrict__ o, int ih0, int j,
                                          int k, int s, T* sum) {
  int jm = (j == 0) ? L.n - 1 : j - 1, jp = (j == L.n - 1) ? 0 : j + 1;
  int km = (k == 0) ? L.n - 1 : k - 1, kp = (k == L.n - 1) ? 0 : k + 1;
  uint32_t r = prow(L, j, k);
  T xv[V + 1], ym[V], yp[V], zm[V], zp[V];
  if (s) {
    ldn<T, V>(o + r + ih0, xv);
    xv[V] = o[r + (ih0 + V == L.nh ? 0 : ih0 + V)];
  } else {
    ldn<T, V>(o + r + ih0, xv + 1);
    xv[0] = o[r + (ih0 == 0 ? L.nh - 1 : ih0 - 1)];
  }
  ldn<T, V>(o + prow(L, jm, k) + ih0, ym);
  ldn<T, V>(o + prow(L, jp, k) + ih0, yp);
  ldn<T, V>(o + prow(L, j, km) + ih0, zm);
  ldn<T, V>(o + prow(L, j, kp) + ih0, zp);
#pragma unroll
  for (int q = 0; q < V; ++q) sum[q] = (xv[q] + xv[q + 1]) + (ym[q] + yp[q]) + (zm[q] + zp[q]);
}

// ---------------------------------------------------------------------------
// Reductions (deterministic: fixed per-block order, then one block)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
// Sum over the block; result valid in thread 0.  blockDim.x <= 1024.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; ++q) t += sh[q];
  }
  return t;
}
// Sum over the block, result broadcast to every thread.
__device__ __forceinline__ double block_sum_all(double v, double* sh) {
  double t = block_sum(v, sh);
  __syncthreads();
  if (threadIdx.x == 0) sh[16] = t;
  __syncthreads();
  return sh[16];
}
// Maximum over the block (v >= 0); result valid in thread 0.
__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int q = 1; q < nw; ++q) v = fmax(v, sh[q]);
  }
  return v;
}
// dst = 16-bit (src * enc), four cells per thread (m % 4 == 0)
__global__ __launch_bounds__(kBlock) void k_to_h16(int64_t m4, const float* __restrict__ src,
                                                   h16* __restrict__ dst, float enc) {
  const int64_t g = gid();
  if (g >= m4) return;
  float v[4];
  ld4s<float>(src + 4 * g, 1.0f, v);
  st4s<h16>(dst + 4 * g, v, enc);
}
// block maxima of |x| over m floats
// block partial maxima of |x| (exact in float), four values per load over
// a grid-stride loop of kAbsmaxBlocks blocks; x 16-byte aligned
constexpr int kAbsmaxBlocks = 2048;
__global__ __launch_bounds__(kBlock) void k_absmax_f32(int64_t m, const float* __restrict__ x,
                                                       double* __restrict__ part) {
  __shared__ double sh[32];
  const int64_t m4 = m >> 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  float v = 0.0f;
  for (int64_t q = gid(); q < m4; q += stride) {
    const float4 a = reinterpret_cast<const float4*>(x)[q];
    v = fmaxf(v, fmaxf(fmaxf(fabsf(a.x), fabsf(a.y)), fmaxf(fabsf(a.z), fabsf(a.w))));
  }
  for (int64_t q = 4 * m4 + gid(); q < m; q += stride) v = fmaxf(v, fabsf(x[q]));
  const double t = block_max(double(v), sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
// Maxima of fixed chunks of m partial maxima, one block per chunk
__global__ void k_max_chunks(const double* __restrict__ part, int64_t m, int64_t chunk,
                             double* __restrict__ out) {
  __shared__ double sh[32];
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < m ? lo + chunk : m;
  double v = 0.0;
  for (int64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) v = fmax(v, part[q]);
  v = block_max(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}
// Maximum of m partial maxima (one block)
__global__ void k_max_partials(const double* __restrict__ part, int64_t m, double* out) {
  __shared__ double sh[32];
  double v = 0.0;
  for (int64_t q = threadIdx.x; q < m; q += blockDim.x) v = fmax(v, part[q]);
  v = block_max(v, sh);
  if (threadIdx.x == 0) *out = v;
}

// stage 1: block b sums the contiguous chunk [b*chunk, (b+1)*chunk)
__global__ void k_sum_chunks(const double* __restrict__ part, int64_t m, int64_t chunk,
                             double* __restrict__ out) {
  __shared__ double sh[32];
  int64_t lo = (int64_t)blockIdx.x * chunk;
  int64_t hi = lo + chunk < m ? lo + chunk : m;
  double s = 0.0;
  for (int64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) s += part[q];
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}
__global__ void k_sum_partials(const double* __restrict__ part, int64_t m, double* out, int slot) {
  __shared__ double sh[32];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < m; q += blockDim.x) s += part[q];
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) out[slot] = t;
}

// ---------------------------------------------------------------------------
// Layout conversion
// ---------------------------------------------------------------------------
// packed[pk] = scale * natural[nat]; one thread per natural cell.
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_pack(Lev L, const TI* __restrict__ nat,
                                                 TO* __restrict__ pk, double scale) {
  int64_t g = gid();
  if (g >= 2 * L.half) return;
  int i, j, k;
  dec_nat(g, L, i, j, k);
  pk[pk_of(L, i, j, k)] = TO(scale * double(nat[g]));
}
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_unpack(Lev L, const TI* __restrict__ pk,
                                                   TO* __restrict__ nat, double scale) {
  int64_t g = gid();
  if (g >= 2 * L.half) return;
  int i, j, k;
  dec_nat(g, L, i, j, k);
  nat[g] = TO(scale * double(pk[pk_of(L, i, j, k)]));
}
// The same transposes on 8 natural cells of a row per thread (n % 8 == 0):
// the row's even cells are 4 consecutive packed cells of one colour, its odd
// cells 4 of the other.
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_pack8(Lev L, const TI* __restrict__ nat,
                                                  TO* __restrict__ pk, double scale) {
  const int64_t g8 = gid();
  if (g8 >= 2 * L.half / 8) return;
  const uint32_t g = (uint32_t)g8 * 8u;
  int i0, j, k;
  dec_nat(g, L, i0, j, k);
  TI v[8];
  ldn<TI, 8>(nat + g, v);
  TO ev[4], od[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ev[q] = TO(scale * double(v[2 * q]));
    od[q] = TO(scale * double(v[2 * q + 1]));
  }
  const int p = (j + k) & 1;  // colour of the row's even cells
  const uint32_t row = prow(L, j, k) + (uint32_t)(i0 >> 1);
  stn<TO, 4>(pk + (uint32_t)p * (uint32_t)L.half + row, ev);
  stn<TO, 4>(pk + (uint32_t)(1 - p) * (uint32_t)L.half + row, od);
}
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_unpack8(Lev L, const TI* __restrict__ pk,
                                                    TO* __restrict__ nat, double scale) {
  const int64_t g8 = gid();
  if (g8 >= 2 * L.half / 8) return;
  const uint32_t g = (uint32_t)g8 * 8u;
  int i0, j, k;
  dec_nat(g, L, i0, j, k);
  const int p = (j + k) & 1;
  const uint32_t row = prow(L, j, k) + (uint32_t)(i0 >> 1);
  TI ev[4], od[4];
  ldn<TI, 4>(pk + (uint32_t)p * (uint32_t)L.half + row, ev);
  ldn<TI, 4>(pk + (uint32_t)(1 - p) * (uint32_t)L.half + row, od);
  TO v[8];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[2 * q] = TO(scale * double(ev[q]));
    v[2 * q + 1] = TO(scale * double(od[q]));
  }
  stn<TO, 8>(nat + g, v);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* __restrict__ p, int64_t m, T v) {
  int64_t g = gid();
  if (g < m) p[g] = v;
}
// 16-byte stores: p 16-byte aligned, m4 = count / 4 for floats
__global__ __launch_bounds__(kBlock) void k_fill4(float4* __restrict__ p, int64_t m4, float v) {
  int64_t g = gid();
  if (g < m4) p[g] = make_float4(v, v, v, v);
}

// ---------------------------------------------------------------------------
// Per-level operations written once, called from grid kernels (one cell per
// thread) and from the fused single-workgroup kernel (strided loops).
// ---------------------------------------------------------------------------
// Direct form.  dens/S packed like v; S may be null (finest level).
template <int M, typename T, typename TD>
__device__ __forceinline__ void op_smooth_direct(const Lev& L, T* __restrict__ v,
                                                 const TD* __restrict__ dens,
                                                 const T* __restrict__ S, int colour, T h2,
                                                 const Consts& C, int64_t g) {
  int ih, j, k;
  dec(g, L, ih, j, k);
  int s = (j + k + colour) & 1;
  T* own = v + colour * L.half;
  const T* oth = v + (1 - colour) * L.half;
  T sum = nbsum<T>(L, oth, ih, j, k, s);
  T dc = T(dens[colour * L.half + g]);
  T sc = S ? S[colour * L.half + g] : T(0);
  T vc = (M == CQ) ? own[g] : T(0);
  own[g] = direct_update<M, T>(C, h2, vc, sum, dc, sc);
}

// residual of packed cell g (both colours: g in [0, n^3))
template <int M, typename T, typename TD>
__device__ __forceinline__ T cell_resid_direct(const Lev& L, const T* __restrict__ v,
                                               const TD* __restrict__ dens,
                                               const T* __restrict__ S, T h2, const Consts& C,
                                               int64_t g) {
  int colour = g >= L.half ? 1 : 0;
  int64_t gg = g - colour * L.half;
  int ih, j, k;
  dec(gg, L, ih, j, k);
  int s = (j + k + colour) & 1;
  T sum = nbsum<T>(L, v + (1 - colour) * L.half, ih, j, k, s);
  T sc = S ? S[g] : T(0);
  return direct_resid<M, T>(C, h2, v[g], sum, T(dens[g]), sc);
}

// Coarse cell gc (natural index over nc^3): restrict v and the residual.
// Writes Rv (packed coarse) into Rv and vinit, R d into Sd.
template <int M, typename T, typename TD>
__device__ __forceinline__ void op_resid_restrict_direct(const Lev& Lf, const Lev& Lc,
                                                         const T* __restrict__ v,
                                                         const TD* __restrict__ dens,
                                                         const T* __restrict__ S, T h2,
                                                         T* __restrict__ Rv, T* __restrict__ vinit,
                                                         T* __restrict__ Sd, const Consts& C,
                                                         int64_t gc) {
  int I, J, K;
  dec_nat(gc, Lc, I, J, K);
  T sv = T(0), sd = T(0);
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int j = 2 * J + b, k = 2 * K + d;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uint32_t g = (uint32_t)c * (uint32_t)Lf.half + prow(Lf, j, k) + I;
        int s = (j + k + c) & 1;
        T vc = v[g];
        T sum = nbsum<T>(Lf, v + (1 - c) * Lf.half, I, j, k, s);
        T sc = S ? S[g] : T(0);
        sv += vc;
        sd += direct_resid<M, T>(C, h2, vc, sum, T(dens[g]), sc);
      }
    }
  uint32_t pc = pk_of(Lc, I, J, K);
  T rv = sv * T(0.125);
  Rv[pc] = rv;
  vinit[pc] = rv;
  Sd[pc] = sd * T(0.125);
}

// S^H = L^H(R v) - R d  (in place on S, which holds R d); g over nc^3 packed
template <int M, typename T, typename TD>
__device__ __forceinline__ void op_coarse_src_direct(const Lev& L, const T* __restrict__ Rv,
                                                     const TD* __restrict__ dens,
                                                     T* __restrict__ S, T h2, const Consts& C,
                                                     int64_t g) {
  T F = cell_resid_direct<M, T, TD>(L, Rv, dens, (const T*)nullptr, h2, C, g);
  S[g] = F - S[g];
}

// v^h += P(vH - RvH) with 27/9/3/1 weights (RvH may be null); g over n^3 packed
template <typename T>
__device__ __forceinline__ void op_prolong_add(const Lev& Lf, const Lev& Lc, T* __restrict__ v,
                                               const T* __restrict__ vH,
                                               const T* __restrict__ RvH, int64_t g) {
  int colour = g >= Lf.half ? 1 : 0;
  int64_t gg = g - colour * Lf.half;
  int ih, j, k;
  dec(gg, Lf, ih, j, k);
  int s = (j + k + colour) & 1;
  int I = ih, J = j >> 1, K = k >> 1;
  int nc = Lc.n;
  int I1 = s ? (I + 1 == nc ? 0 : I + 1) : (I == 0 ? nc - 1 : I - 1);
  int J1 = (j & 1) ? (J + 1 == nc ? 0 : J + 1) : (J == 0 ? nc - 1 : J - 1);
  int K1 = (k & 1) ? (K + 1 == nc ? 0 : K + 1) : (K == 0 ? nc - 1 : K - 1);
  const int Is[2] = {I, I1}, Js[2] = {J, J1}, Ks[2] = {K, K1};
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        uint32_t pc = pk_of(Lc, Is[a], Js[b], Ks[d]);
        T c = RvH ? (vH[pc] - RvH[pc]) : vH[pc];
        T w = T((a ? 1 : 3) * (b ? 1 : 3) * (d ? 1 : 3)) * T(1.0 / 64.0);
        acc += w * c;
      }
  v[g] += acc;
}

// Prolongation weight pair: 3/4 on the nearer coarse value, 1/4 on the
// farther, as one explicit multiply and one fused multiply-add, so every
// kernel that forms P (fused into a smoother or not) rounds identically.
template <typename T>
__device__ __forceinline__ T p34(T near, T far) {
  if constexpr (sizeof(T) == 4) return __fmaf_rn(0.75f, near, __fmul_rn(0.25f, far));
  else return __fma_rn(0.75, near, __dmul_rn(0.25, far));
}

// v^h += P c for the 8 children of coarse cell gc (natural index over nc^3):
// c is the packed coarse correction; trilinear 3/4-1/4 per axis applied
// separably over the 3x3x3 coarse neighbourhood (27/9/3/1 in total).
template <typename T>
__device__ __forceinline__ void op_prolong_block(const Lev& Lf, const Lev& Lc, T* __restrict__ v,
                                                 const T* __restrict__ c, int64_t gc) {
  const int nc = Lc.n;
  int I, J, K;
  dec_nat(gc, Lc, I, J, K);
  const int Is[3] = {I == 0 ? nc - 1 : I - 1, I, I + 1 == nc ? 0 : I + 1};
  const int Js[3] = {J == 0 ? nc - 1 : J - 1, J, J + 1 == nc ? 0 : J + 1};
  const int Ks[3] = {K == 0 ? nc - 1 : K - 1, K, K + 1 == nc ? 0 : K + 1};
  T ax[3][3][2];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      T c0 = c[pk_of(Lc, Is[0], Js[b], Ks[d])];
      T c1 = c[pk_of(Lc, Is[1], Js[b], Ks[d])];
      T c2 = c[pk_of(Lc, Is[2], Js[b], Ks[d])];
      ax[d][b][0] = p34<T>(c1, c0);
      ax[d][b][1] = p34<T>(c1, c2);
    }
  T ay[3][2][2];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      ay[d][0][x] = p34<T>(ax[d][1][x], ax[d][0][x]);
      ay[d][1][x] = p34<T>(ax[d][1][x], ax[d][2][x]);
    }
#pragma unroll
  for (int z = 0; z < 2; ++z)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int j = 2 * J + y, k = 2 * K + z;
      const uint32_t row = prow(Lf, j, k) + I;
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        T val = p34<T>(ay[1][y][x], ay[z ? 2 : 0][y][x]);
        const int colour = (2 * I + x + j + k) & 1;
        v[colour * Lf.half + row] += val;
      }
    }
}

// plain 8-mean restriction, natural coarse index gc, packed in/out
template <typename TI, typename TO>
__device__ __forceinline__ void op_restrict(const Lev& Lf, const Lev& Lc, const TI* __restrict__ f,
                                            TO* __restrict__ c, int64_t gc) {
  int I, J, K;
  dec_nat(gc, Lc, I, J, K);
  double s = 0.0;
  for (int d = 0; d < 2; ++d)
    for (int b = 0; b < 2; ++b) {
      uint32_t row = prow(Lf, 2 * J + b, 2 * K + d) + I;
      s += double(f[row]) + double(f[Lf.half + row]);
    }
  c[pk_of(Lc, I, J, K)] = TO(s * 0.125);
}

// Correction form (FP32)
template <int M>
__device__ __forceinline__ void op_smooth_corr(const Lev& L, float* __restrict__ e,
                                               const float* __restrict__ X,
                                               const float* __restrict__ dens,
                                               const float* __restrict__ rho, int colour, float h2,
                                               const Consts& C, int64_t g) {
  int ih, j, k;
  dec(g, L, ih, j, k);
  int s = (j + k + colour) & 1;
  float* own = e + colour * L.half;
  float sum = nbsum<float>(L, e + (1 - colour) * L.half, ih, j, k, s);
  int64_t q = colour * L.half + g;
  float dc = (M == FR) ? 0.0f : dens[q];
  float eo = (M == CQ) ? own[g] : 0.0f;
  own[g] = corr_update<M>(C, h2, eo, sum, X[q], dc, rho[q]);
}

template <int M>
__device__ __forceinline__ float cell_resid_corr(const Lev& L, const float* __restrict__ e,
                                                 const float* __restrict__ X,
                                                 const float* __restrict__ dens,
                                                 const float* __restrict__ rho, float h2,
                                                 const Consts& C, int64_t g) {
  int colour = g >= L.half ? 1 : 0;
  int64_t gg = g - colour * L.half;
  int ih, j, k;
  dec(gg, L, ih, j, k);
  int s = (j + k + colour) & 1;
  float sum = nbsum<float>(L, e + (1 - colour) * L.half, ih, j, k, s);
  float dc = (M == FR) ? 0.0f : dens[g];
  float r = rho ? rho[g] : 0.0f;
  return corr_G<M>(C, h2, e[g], sum, X[g], dc) - r;
}

// Coarse outputs of a correction-form restriction at packed coarse index pc
// from the fine sums se (of e), sd (of the residual G(e) - rho) and sx (of
// X, when formed).
// Plain form (Xf null): eH = eR = R e, rhoH = R(G(e) - rho), XH = R X when
// XH is given; the coarse-source pass then sets rhoH = G_H(R e) - rhoH, and
// the coarse correction is e_H - R e.
// Shifted form (Xf given): the coarse problem is posed around the
// restricted current approximation, XH = R X + R e (R X formed, and with rx
// stored in Xf, or read from Xf).  Since G_H(R e + d; R X) - G_H(R e; R X)
// = G_H(d; R X + R e), the same coarse equation for d = e_H - R e reads
// G_H(d; XH) = R(rho - G(e)), so rhoH = -R(G(e) - rho), d starts at zero
// (eH = 0 when given, else the coarse smoother takes it as zero) and is
// itself the coarse correction: no coarse source and no eR.
__device__ __forceinline__ void store_coarse_corr(uint32_t pc, float se, float sd, float sx,
                                                  float* eH, float* eR, float* rhoH, float* XH,
                                                  float* Xf, int rx) {
  const float re = se * 0.125f;
  rhoH[pc] = Xf ? -(sd * 0.125f) : sd * 0.125f;
  if (Xf) {
    float xf;
    if (rx) {
      xf = sx * 0.125f;
      Xf[pc] = xf;
    } else {
      xf = Xf[pc];
    }
    XH[pc] = xf + re;
    if (eH) eH[pc] = 0.0f;
  } else {
    eH[pc] = re;
    eR[pc] = re;
    if (XH) XH[pc] = sx * 0.125f;
  }
}
// coarse cell gc: restriction in the plain or shifted form (store_coarse_corr)
template <int M>
__device__ __forceinline__ void op_resid_restrict_corr(
    const Lev& Lf, const Lev& Lc, const float* __restrict__ e, const float* __restrict__ X,
    const float* __restrict__ dens, const float* __restrict__ rho, float h2,
    float* __restrict__ eH, float* __restrict__ eR, float* __restrict__ rhoH,
    float* __restrict__ XH, const Consts& C, int64_t gc, float* Xf = nullptr, int rx = 0) {
  int I, J, K;
  dec_nat(gc, Lc, I, J, K);
  const bool want_x = XH && (!Xf || rx);
  float se = 0.0f, sd = 0.0f, sx = 0.0f;
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int j = 2 * J + b, k = 2 * K + d;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uint32_t g = (uint32_t)c * (uint32_t)Lf.half + prow(Lf, j, k) + I;
        int s = (j + k + c) & 1;
        float ec = e[g];
        float sum = nbsum<float>(Lf, e + (1 - c) * Lf.half, I, j, k, s);
        float x = X[g];
        float dc = (M == FR) ? 0.0f : dens[g];
        se += ec;
        if (want_x) sx += x;
        sd += corr_G<M>(C, h2, ec, sum, x, dc) - rho[g];
      }
    }
  store_coarse_corr(pk_of(Lc, I, J, K), se, sd, sx, eH, eR, rhoH, XH, Xf, rx);
}

template <int M>
__device__ __forceinline__ void op_coarse_src_corr(const Lev& L, const float* __restrict__ eR,
                                                   const float* __restrict__ X,
                                                   const float* __restrict__ dens,
                                                   float* __restrict__ rho, float h2,
                                                   const Consts& C, int64_t g) {
  float G = cell_resid_corr<M>(L, eR, X, dens, (const float*)nullptr, h2, C, g);
  rho[g] = G - rho[g];
}

// Exact FP32 update of one cell of the linear operator below, (r + kh2 sum)
// / (6 kh2 + dg), with every rounding explicit: a loop-invariant 6 kh2 may
// otherwise be fused into the add in one kernel and not in another.
__device__ __forceinline__ float lin_cell_f(float r, float sum, float dg, float kh2) {
  return __fmul_rn(__fmaf_rn(kh2, sum, r), f_rcp(__fmaf_rn(6.0f, kh2, dg)));
}
// Linear (adjoint) operator A v = kap (6v - sum)/h^2 + dg v; kh2 = kap/h^2
template <typename T>
__device__ __forceinline__ void op_smooth_lin(const Lev& L, T* __restrict__ e,
                                              const T* __restrict__ dg, const T* __restrict__ r,
                                              int colour, T kh2, int64_t g) {
  int ih, j, k;
  dec(g, L, ih, j, k);
  int s = (j + k + colour) & 1;
  T sum = nbsum<T>(L, e + (1 - colour) * L.half, ih, j, k, s);
  int64_t q = colour * L.half + g;
  e[q] = (r[q] + kh2 * sum) / (T(6) * kh2 + dg[q]);
}
template <typename T>
__device__ __forceinline__ T cell_lin_resid(const Lev& L, const T* __restrict__ e,
                                            const T* __restrict__ dg, const T* __restrict__ r,
                                            T kh2, int64_t g) {
  int colour = g >= L.half ? 1 : 0;
  int64_t gg = g - colour * L.half;
  int ih, j, k;
  dec(gg, L, ih, j, k);
  int s = (j + k + colour) & 1;
  T sum = nbsum<T>(L, e + (1 - colour) * L.half, ih, j, k, s);
  return r[g] - (kh2 * (T(6) * e[g] - sum) + dg[g] * e[g]);
}
// coarse cell gc: rH = R(r - A e), eH = 0
template <typename T>
__device__ __forceinline__ void op_lin_resid_restrict(const Lev& Lf, const Lev& Lc,
                                                      const T* __restrict__ e,
                                                      const T* __restrict__ dg,
                                                      const T* __restrict__ r, T kh2,
                                                      T* __restrict__ rH, T* __restrict__ eH,
                                                      int64_t gc) {
  int I, J, K;
  dec_nat(gc, Lc, I, J, K);
  T sd = T(0);
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int j = 2 * J + b, k = 2 * K + d;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uint32_t g = (uint32_t)c * (uint32_t)Lf.half + prow(Lf, j, k) + I;
        sd += cell_lin_resid<T>(Lf, e, dg, r, kh2, g);
      }
    }
  uint32_t pc = pk_of(Lc, I, J, K);
  rH[pc] = sd * T(0.125);
  eH[pc] = T(0);
}

// ---------------------------------------------------------------------------
// Vectorised grid kernels: V cells of one colour per thread (smoothers) or V
// cells of each colour (residual kernels, so a row's two colours are read by
// the same thread and the other colour's rows stay in L2).  g4 indexes
// groups of V packed cells; nh % V == 0.
// ---------------------------------------------------------------------------
template <int M, typename TD>
__global__ __launch_bounds__(kBlock) void k_smooth_direct_v(Lev L, double* v, const TD* dens,
                                                            const double* S, int colour,
                                                            double h2, Consts C) {
  constexpr int V = Vec<double>::V;
  uint32_t g4 = (uint32_t)gid();
  if (g4 >= (uint32_t)(L.half / V)) return;
  uint32_t g = g4 * V;
  int ih0, j, k;
  dec(g, L, ih0, j, k);
  int s = (j + k + colour) & 1;
  double* own = v + colour * L.half;
  double sum[V], vo[V] = {0.0, 0.0}, sc[V] = {0.0, 0.0}, out[V];
  nbsum_vec<double>(L, v + (1 - colour) * L.half, ih0, j, k, s, sum);
  if (M == CQ) ldv<double>(own + g, vo);
  if (S) ldv<double>(S + colour * L.half + g, sc);
  const TD* dp = dens + colour * L.half + g;
#pragma unroll
  for (int q = 0; q < V; ++q)
    out[q] = direct_update<M, double>(C, h2, vo[q], sum[q], double(dp[q]), sc[q]);
  stv<double>(own + g, out);
}

// fresh: first half-sweeps after an outer step, whose correction starts at
// zero: the buffer is not cleared, the old values are taken as 0 instead
// (colour 0: neighbours and own value; colour 1: own value).
template <int M, typename TX = float, typename TR = float>
__device__ __forceinline__ void op_smooth_corr_v(const Lev& L, float* __restrict__ e,
                                                 const TX* __restrict__ X,
                                                 const float* __restrict__ dens,
                                                 const TR* __restrict__ rho, int colour,
                                                 float h2, const Consts& C, uint32_t g4,
                                                 int fresh = 0, Store S = Store{1, 1, 1, 1}) {
  constexpr int V = Vec<float>::V;
  uint32_t g = g4 * V;
  int ih0, j, k;
  dec(g, L, ih0, j, k);
  int s = (j + k + colour) & 1;
  float* own = e + colour * L.half;
  uint32_t q0 = (uint32_t)colour * (uint32_t)L.half + g;
  float sum[V] = {0, 0, 0, 0}, x[V], r[V], dc[V] = {0, 0, 0, 0}, eo[V] = {0, 0, 0, 0}, out[V];
  if (!(fresh && colour == 0)) nbsum_vec<float>(L, e + (1 - colour) * L.half, ih0, j, k, s, sum);
  ld4s<TX>(X + q0, S.x_dec, x);
  ld4s<TR>(rho + q0, S.r_dec, r);
  if (M != FR) ldv_nt<float>(dens + q0, dc);
  if (M == CQ && !fresh) ldv<float>(own + g, eo);
  corr_update4<M>(C, h2, eo, sum, x, dc, r, out);
  stv_nt<float>(own + g, out);
}
template <int M, typename TX = float, typename TR = float>
__global__ __launch_bounds__(kBlock) void k_smooth_corr_v(Lev L, float* e, const TX* X,
                                                          const float* dens, const TR* rho,
                                                          int colour, float h2, Consts C,
                                                          int fresh, Store S = Store{1, 1, 1, 1}) {
  uint32_t g4 = (uint32_t)gid();
  if (g4 < (uint32_t)(L.half / Vec<float>::V))
    op_smooth_corr_v<M, TX, TR>(L, e, X, dens, rho, colour, h2, C, g4, fresh, S);
}

// fresh (colour 0 only): the correction starts at zero, neighbours are 0.
// TD, TR: storage of dg and r (16-bit on the finest level of an FP32 solve;
// S.x_dec decodes dg, S.r_dec decodes r)
template <typename T, typename TD = T, typename TR = T>
__global__ __launch_bounds__(kBlock) void k_smooth_lin_v(Lev L, T* e, const TD* dg, const TR* r,
                                                         int colour, T kh2, int fresh,
                                                         Store S = Store{1, 1, 1, 1}) {
  constexpr int V = Vec<T>::V;
  uint32_t g4 = (uint32_t)gid();
  if (g4 >= (uint32_t)(L.half / V)) return;
  uint32_t g = g4 * V;
  int ih0, j, k;
  dec(g, L, ih0, j, k);
  int s = (j + k + colour) & 1;
  uint32_t q0 = (uint32_t)colour * (uint32_t)L.half + g;
  T sum[V], d[V], rr[V], out[V];
  if (fresh && colour == 0) {
#pragma unroll
    for (int q = 0; q < V; ++q) sum[q] = T(0);
  } else {
    nbsum_vec<T>(L, e + (1 - colour) * L.half, ih0, j, k, s, sum);
  }
  ldNs<T, TD, V>(dg + q0, S.x_dec, d);
  ldNs<T, TR, V>(r + q0, S.r_dec, rr);
#pragma unroll
  for (int q = 0; q < V; ++q) {
    if constexpr (sizeof(T) == 4) out[q] = lin_cell_f(rr[q], sum[q], d[q], kh2);
    else out[q] = (rr[q] + kh2 * sum[q]) / (T(6) * kh2 + d[q]);
  }
  stv_nt<T>(e + q0, out);
}


// Fused FP64 outer step of the refined mode: w_new = w + e (e may be null:
// no update), d = F(w_new), rho = -d, X = w_new, e_zero = 0 (a different
// buffer from e); per-block sum of d^2.
constexpr int kVOuter = 4;  // cells per colour per thread in the outer kernels (nh % 4 == 0)

// ---------------------------------------------------------------------------
// k-marching versions of the FP64 outer steps.  A block owns kBlock groups of
// V consecutive packed cells of one plane (both colours) and walks kt planes
// upwards, keeping its own columns of planes k-1, k, k+1 in registers, so the
// z-neighbours are read from HBM once; the in-plane neighbours (rows j +- 1,
// the row's edge cell) are recent lines of the neighbouring threads and come
// from L1/L2.  Consecutive blocks take neighbouring chunks of the same planes.
// Same per-cell arithmetic and neighbour summation order as the kernels above.
// ---------------------------------------------------------------------------
constexpr int kMarchKT = 16;

struct MarchPos {
  int j, jm, jp, ih0, k0, k1;
  bool ok;
};
__device__ __forceinline__ MarchPos march_pos(const Lev& L, int kt, int V) {
  MarchPos P;
  const uint32_t ngrp = (uint32_t)L.n * (uint32_t)L.nh / (uint32_t)V;
  const uint32_t nchunk = (ngrp + kBlock - 1) / kBlock;
  const uint32_t b = (uint32_t)xcd_block();
  const uint32_t kb = b / nchunk, chunk = b - kb * nchunk;
  const uint32_t grp = chunk * kBlock + threadIdx.x;
  P.k0 = (int)kb * kt;
  P.ok = grp < ngrp && P.k0 < L.n;
  const uint32_t p = grp * (uint32_t)V;
  const uint32_t jj = L.dnh.div(p);
  P.j = (int)jj;
  P.ih0 = (int)(p - jj * (uint32_t)L.nh);
  P.jm = P.j == 0 ? L.n - 1 : P.j - 1;
  P.jp = P.j == L.n - 1 ? 0 : P.j + 1;
  P.k1 = P.k0 + kt < L.n ? P.k0 + kt : L.n;
  return P;
}
// blocks of a march over a level
__host__ __device__ inline unsigned march_blocks(const Lev& L, int kt, int V) {
  unsigned ngrp = (unsigned)((uint64_t)L.n * (uint64_t)L.nh / (uint64_t)V);
  unsigned nchunk = (ngrp + kBlock - 1) / kBlock;
  return nchunk * (unsigned)((L.n + kt - 1) / kt);
}
// The same half-sweep marching in z: a thread owns 4 packed cells of its
// colour in row j and walks kt planes, keeping the other colour's rows
// (j, k-1), (j, k), (j, k+1) in registers, so each plane reads one new
// other-colour row plus the rows j +- 1.  Per-cell arithmetic and the
// neighbour summation order are those of op_smooth_corr_v (bit-identical).
template <int M, typename TX, typename TR>
__device__ __forceinline__ void op_smooth_corr_kv(const Lev& L, float* e, const TX* X,
                                                  const float* dens, const TR* rho, int colour,
                                                  float h2, const Consts& C, int fresh, int kt,
                                                  const Store& S) {
  constexpr int V = Vec<float>::V;
  const MarchPos P = march_pos(L, kt, V);
  if (!P.ok) return;
  const float* o = e + (1 - colour) * L.half;
  float* own = e + colour * L.half;
  const int j = P.j, ih0 = P.ih0, n = L.n;
  const bool zero_nb = fresh && colour == 0;  // the other colour still holds no correction
  float zm[V] = {0, 0, 0, 0}, zc[V] = {0, 0, 0, 0}, zp[V] = {0, 0, 0, 0};
  if (!zero_nb) {
    ldn<float, V>(o + prow(L, j, P.k0 == 0 ? n - 1 : P.k0 - 1) + ih0, zm);
    ldn<float, V>(o + prow(L, j, P.k0) + ih0, zc);
  }
  for (int k = P.k0; k < P.k1; ++k) {
    const uint32_t r = prow(L, j, k);
    float sum[V] = {0, 0, 0, 0};
    if (!zero_nb) {
      ldn<float, V>(o + prow(L, j, k + 1 == n ? 0 : k + 1) + ih0, zp);
      const int s = (j + k + colour) & 1;
      float xv[V + 1], ym[V], yp[V];
      if (s) {
#pragma unroll
        for (int q = 0; q < V; ++q) xv[q] = zc[q];
        xv[V] = o[r + (ih0 + V == L.nh ? 0 : ih0 + V)];
      } else {
#pragma unroll
        for (int q = 0; q < V; ++q) xv[q + 1] = zc[q];
        xv[0] = o[r + (ih0 == 0 ? L.nh - 1 : ih0 - 1)];
      }
      ldn<float, V>(o + prow(L, P.jm, k) + ih0, ym);
      ldn<float, V>(o + prow(L, P.jp, k) + ih0, yp);
#pragma unroll
      for (int q = 0; q < V; ++q)
        sum[q] = (xv[q] + xv[q + 1]) + (ym[q] + yp[q]) + (zm[q] + zp[q]);
    }
    const uint32_t q0 = (uint32_t)colour * (uint32_t)L.half + r + (uint32_t)ih0;
    float x[V], rr[V], dc[V] = {0, 0, 0, 0}, eo[V] = {0, 0, 0, 0}, out[V];
    ld4s<TX>(X + q0, S.x_dec, x);
    ld4s<TR>(rho + q0, S.r_dec, rr);
    if (M != FR) ldv_nt<float>(dens + q0, dc);
    if (M == CQ && !fresh) ldv<float>(own + r + ih0, eo);
    corr_update4<M>(C, h2, eo, sum, x, dc, rr, out);
    stv_nt<float>(own + r + ih0, out);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      zm[q] = zc[q];
      zc[q] = zp[q];
    }
  }
}
template <int M, typename TX = float, typename TR = float>
__global__ __launch_bounds__(kBlock) void k_smooth_corr_kv(Lev L, float* e, const TX* X,
                                                           const float* dens, const TR* rho,
                                                           int colour, float h2, Consts C,
                                                           int fresh, int kt,
                                                           Store S = Store{1, 1, 1, 1}) {
  op_smooth_corr_kv<M, TX, TR>(L, e, X, dens, rho, colour, h2, C, fresh, kt, S);
}
// Exact per-cell update of the linear (adjoint) operator for 4 consecutive
// packed cells at q0, given the sums of their 6 neighbours.
template <typename TD, typename TR>
__device__ __forceinline__ void lin_update4(const TD* __restrict__ dg, const TR* __restrict__ r,
                                            uint32_t q0, float kh2, const Store& S,
                                            const float* sum, float* out) {
  float d[4], rr[4];
  ld4s<TD>(dg + q0, S.x_dec, d);
  ld4s<TR>(r + q0, S.r_dec, rr);
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = lin_cell_f(rr[q], sum[q], d[q], kh2);
}
// The linear half-sweep marching in z (FP32): a thread owns 4 packed cells
// of its colour in row j and walks kt planes, keeping the other colour's
// rows (j, k-1), (j, k), (j, k+1) in registers.  Same per-cell arithmetic
// and neighbour summation order as k_smooth_lin_v (bit-identical).
template <typename TD, typename TR>
__global__ __launch_bounds__(kBlock) void k_smooth_lin_kv(Lev L, float* e, const TD* dg,
                                                          const TR* r, int colour, float kh2,
                                                          int fresh, int kt, Store S) {
  constexpr int V = 4;
  const MarchPos P = march_pos(L, kt, V);
  if (!P.ok) return;
  const float* o = e + (1 - colour) * L.half;
  float* own = e + colour * L.half;
  const int j = P.j, ih0 = P.ih0, n = L.n;
  const bool zero_nb = fresh && colour == 0;
  float zm[V] = {0, 0, 0, 0}, zc[V] = {0, 0, 0, 0}, zp[V] = {0, 0, 0, 0};
  if (!zero_nb) {
    ldn<float, V>(o + prow(L, j, P.k0 == 0 ? n - 1 : P.k0 - 1) + ih0, zm);
    ldn<float, V>(o + prow(L, j, P.k0) + ih0, zc);
  }
  for (int k = P.k0; k < P.k1; ++k) {
    const uint32_t rw = prow(L, j, k);
    float sum[V] = {0, 0, 0, 0};
    if (!zero_nb) {
      ldn<float, V>(o + prow(L, j, k + 1 == n ? 0 : k + 1) + ih0, zp);
      const int s = (j + k + colour) & 1;
      float xv[V + 1], ym[V], yp[V];
      if (s) {
#pragma unroll
        for (int q = 0; q < V; ++q) xv[q] = zc[q];
        xv[V] = o[rw + (ih0 + V == L.nh ? 0 : ih0 + V)];
      } else {
#pragma unroll
        for (int q = 0; q < V; ++q) xv[q + 1] = zc[q];
        xv[0] = o[rw + (ih0 == 0 ? L.nh - 1 : ih0 - 1)];
      }
      ldn<float, V>(o + prow(L, P.jm, k) + ih0, ym);
      ldn<float, V>(o + prow(L, P.jp, k) + ih0, yp);
#pragma unroll
      for (int q = 0; q < V; ++q)
        sum[q] = (xv[q] + xv[q + 1]) + (ym[q] + yp[q]) + (zm[q] + zp[q]);
    }
    const uint32_t q0 = (uint32_t)colour * (uint32_t)L.half + rw + (uint32_t)ih0;
    float out[V];
    lin_update4<TD, TR>(dg, r, q0, kh2, S, sum, out);
    stv_nt<float>(own + rw + ih0, out);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      zm[q] = zc[q];
      zc[q] = zp[q];
    }
  }
}


// v = w + e (e may be null; w null: the uniform value wu) of V packed cells
// of colour c in row (j, k)
template <typename TE, int V>
__device__ __forceinline__ void march_ld(const Lev& L, const double* __restrict__ w,
                                         const TE* __restrict__ e, int c, int j, int k, int ih0,
                                         double* out, double wu) {
  const uint32_t q0 = (uint32_t)c * (uint32_t)L.half + prow(L, j, k) + (uint32_t)ih0;
  if (w) {
    ldn<double, V>(w + q0, out);
  } else {
#pragma unroll
    for (int t = 0; t < V; ++t) out[t] = wu;
  }
  if (e) {
    TE ev[V];
    ldn<TE, V>(e + q0, ev);
#pragma unroll
    for (int t = 0; t < V; ++t) out[t] += double(ev[t]);
  }
}
// neighbour sums of the V cells of colour c at plane k from the window
// (planes k-1 and k+1 of the other colour) and the in-plane loads
template <typename TE, int V>
__device__ __forceinline__ void march_nbsum(const Lev& L, const double* __restrict__ w,
                                            const TE* __restrict__ e, const MarchPos& P, int c,
                                            int k, const double (*wo)[V], double* sum,
                                            double wu) {
  const int o = 1 - c;
  const int s = (P.j + k + c) & 1;
  double ym[V], yp[V];
  march_ld<TE, V>(L, w, e, o, P.jm, k, P.ih0, ym, wu);
  march_ld<TE, V>(L, w, e, o, P.jp, k, P.ih0, yp, wu);
  const uint32_t ro = (uint32_t)o * (uint32_t)L.half + prow(L, P.j, k);
  const uint32_t xi = s ? (P.ih0 + V == L.nh ? 0 : P.ih0 + V) : (P.ih0 == 0 ? L.nh - 1 : P.ih0 - 1);
  const double xe = (w ? w[ro + xi] : wu) + (e ? double(e[ro + xi]) : 0.0);
  double xv[V + 1];
#pragma unroll
  for (int t = 0; t < V; ++t) xv[s ? t : t + 1] = wo[1][t];
  xv[s ? V : 0] = xe;
#pragma unroll
  for (int q = 0; q < V; ++q)
    sum[q] = (xv[q] + xv[q + 1]) + (ym[q] + yp[q]) + (wo[0][q] + wo[2][q]);
}

template <int M, typename TX = float, typename TR = float>
__global__ __launch_bounds__(kBlock) void k_outer_fused_kv(Lev L, const double* __restrict__ w,
                                                           const float* __restrict__ e,
                                                           double* __restrict__ w_new,
                                                           const float* __restrict__ dens,
                                                           Consts C, TR* __restrict__ rho,
                                                           TX* __restrict__ X,
                                                           float* __restrict__ e_zero,
                                                           double* __restrict__ part,
                                                           double* __restrict__ part_bg, int kt,
                                                           Store S = Store{1, 1, 1, 1},
                                                           double* __restrict__ part_max = nullptr) {
  constexpr int V = kVOuter;
  static_assert(V == 4, "the stored 4-cell groups");
  __shared__ double sh[32];
  const MarchPos P = march_pos(L, kt, V);
  double acc = 0.0, accb = 0.0;  // sum d^2; sum (bg_coef delta)^2 when part_bg is given
  double amax = 0.0;             // max |d| when part_max is given
  if (P.ok) {
    double win[2][3][V];  // [colour][plane k-1, k, k+1][cell]
    const int km0 = P.k0 == 0 ? L.n - 1 : P.k0 - 1;
    const double wu = C.bg;  // w null: the master is the uniform background
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      march_ld<float, V>(L, w, e, c, P.j, km0, P.ih0, win[c][0], wu);
      march_ld<float, V>(L, w, e, c, P.j, P.k0, P.ih0, win[c][1], wu);
    }
    for (int k = P.k0; k < P.k1; ++k) {
      const int kp = k + 1 == L.n ? 0 : k + 1;
#pragma unroll
      for (int c = 0; c < 2; ++c) march_ld<float, V>(L, w, e, c, P.j, kp, P.ih0, win[c][2], wu);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double sum[V];
        march_nbsum<float, V>(L, w, e, P, c, k, win[1 - c], sum, wu);
        const uint32_t q0 = (uint32_t)c * (uint32_t)L.half + prow(L, P.j, k) + (uint32_t)P.ih0;
        if (e) stn_nt<double, V>(w_new + q0, win[c][1]);
        float dn[V], ro[V], xo[V], zo[V];
        ldn_nt<float, V>(dens + q0, dn);
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const double vc = win[c][1][q];
          double d = direct_resid<M, double>(C, 1.0, vc, sum[q], double(dn[q]), 0.0);
          acc += d * d;
          if (part_bg) {
            const double bd = C.bg_coef * double(dn[q]);
            accb += bd * bd;
          }
          amax = fmax(amax, fabs(d));
          ro[q] = float(-d);
          xo[q] = float(vc);
          zo[q] = 0.0f;
        }
        st4s<TR>(rho + q0, ro, S.r_enc);
        st4s<TX>(X + q0, xo, S.x_enc);
        if (e_zero) stn_nt<float, V>(e_zero + q0, zo);
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < V; ++q) {
          win[c][0][q] = win[c][1][q];
          win[c][1][q] = win[c][2][q];
        }
    }
  }
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
  if (part_bg) {  // uniform over the grid: every thread reaches block_sum's barriers
    const double tb = block_sum(accb, sh);
    if (threadIdx.x == 0) part_bg[blockIdx.x] = tb;
  }
  if (part_max) {  // uniform over the grid as well
    const double tm = block_max(amax, sh);
    if (threadIdx.x == 0) part_max[blockIdx.x] = tm;
  }
}

// adjoint: lam_new = lam + e + shift, r = b - A lam_new, e_zero = 0;
// partial sums of r^2 (and of r when part_sum is given)
// TR: storage of r (16-bit, scaled by S.r_enc, for an FP32 solve's finest
// level); part_max: block maxima of |r| when given
template <typename TO, typename TR = TO>
__global__ __launch_bounds__(kBlock) void k_lin_outer_fused_kv(
    Lev L, const double* __restrict__ lam, const TO* __restrict__ e, double* __restrict__ lam_new,
    const double* __restrict__ dg, const double* __restrict__ b, double kh2, TR* __restrict__ r,
    TO* __restrict__ e_zero, double* __restrict__ part, double shift, double* __restrict__ part_sum,
    int kt, Store S = Store{1, 1, 1, 1}, double* __restrict__ part_max = nullptr) {
  constexpr int V = kVOuter;
  __shared__ double sh[32];
  const MarchPos P = march_pos(L, kt, V);
  const bool zero_start = !lam && !e && shift == 0.0;
  double acc = 0.0, accs = 0.0, amax = 0.0;
  if (P.ok) {
    double win[2][3][V];
    const int km0 = P.k0 == 0 ? L.n - 1 : P.k0 - 1;
#pragma unroll
    for (int c = 0; c < 2; ++c) {  // lam null: lam = 0
      march_ld<TO, V>(L, lam, e, c, P.j, km0, P.ih0, win[c][0], 0.0);
      march_ld<TO, V>(L, lam, e, c, P.j, P.k0, P.ih0, win[c][1], 0.0);
    }
    for (int k = P.k0; k < P.k1; ++k) {
      const int kp = k + 1 == L.n ? 0 : k + 1;
#pragma unroll
      for (int c = 0; c < 2; ++c) march_ld<TO, V>(L, lam, e, c, P.j, kp, P.ih0, win[c][2], 0.0);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double sum[V], lc[V], dd[V], bb[V];
        march_nbsum<TO, V>(L, lam, e, P, c, k, win[1 - c], sum, 0.0);
        const uint32_t q0 = (uint32_t)c * (uint32_t)L.half + prow(L, P.j, k) + (uint32_t)P.ih0;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          lc[q] = win[c][1][q] + shift;
          sum[q] += 6.0 * shift;
        }
        if (e) stn<double, V>(lam_new + q0, lc);
        if (zero_start) {  // lam = 0: the residual is b, dg * 0 = 0 (dg finite)
#pragma unroll
          for (int q = 0; q < V; ++q) dd[q] = 0.0;
        } else {
          ldn<double, V>(dg + q0, dd);
        }
        ldn<double, V>(b + q0, bb);
        TO ro[V], zo[V];
#pragma unroll
        for (int q = 0; q < V; ++q) {
          double d = bb[q] - (kh2 * (6.0 * lc[q] - sum[q]) + dd[q] * lc[q]);
          acc += d * d;
          accs += d;
          amax = fmax(amax, fabs(d));
          ro[q] = TO(d);
          zo[q] = TO(0);
        }
        if constexpr (sizeof(TO) == 4) st4s<TR>(r + q0, ro, S.r_enc);
        else stn<TO, V>(r + q0, ro);
        if (e_zero) stn<TO, V>(e_zero + q0, zo);
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < V; ++q) {
          win[c][0][q] = win[c][1][q];
          win[c][1][q] = win[c][2][q];
        }
    }
  }
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
  if (part_sum) {
    t = block_sum(accs, sh);
    if (threadIdx.x == 0) part_sum[blockIdx.x] = t;
  }
  if (part_max) {  // uniform over the grid
    t = block_max(amax, sh);
    if (threadIdx.x == 0) part_max[blockIdx.x] = t;
  }
}

// residual norm of the finest level (FP64 direct form), both colours per thread
template <int M, typename TD>
__global__ __launch_bounds__(kBlock) void k_resid_norm_v(Lev L, const double* v, const TD* dens,
                                                         Consts C, double* part, double* d_nat) {
  constexpr int V = Vec<double>::V;
  __shared__ double sh[32];
  uint32_t g4 = (uint32_t)gid();
  double acc = 0.0;
  if (g4 < (uint32_t)(L.half / V)) {
    uint32_t g = g4 * V;
    int ih0, j, k;
    dec(g, L, ih0, j, k);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t q0 = (uint32_t)c * (uint32_t)L.half + g;
      int s = (j + k + c) & 1;
      double sum[V], vc[V];
      nbsum_vec<double>(L, v + (1 - c) * L.half, ih0, j, k, s, sum);
      ldv<double>(v + q0, vc);
#pragma unroll
      for (int q = 0; q < V; ++q) {
        double d = direct_resid<M, double>(C, 1.0, vc[q], sum[q], double(dens[q0 + q]), 0.0);
        acc += d * d;
        if (d_nat) d_nat[((int64_t)k * L.n + j) * L.n + 2 * (ih0 + q) + s] = d;
      }
    }
  }
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// Vectorised transfers: V consecutive coarse cells (I0 .. I0+V-1, J, K) per
// thread, I0 % V == 0 (requires the coarse side % V == 0).  Their children
// are the fine packed cells ih = I0 .. I0+V-1 of both colours in the four
// rows (2J+b, 2K+d), read and written with 16-byte accesses.
// ---------------------------------------------------------------------------
// v^h += P (c - c2) (27/9/3/1 trilinear, separable over the coarse
// neighbourhood; c2 may be null).  Only fine colours COL0..1 are written:
// before a smoother that solves each cell exactly (f(R), symmetron, the
// linear adjoint), the first post-smoothing half-sweep overwrites colour 0
// without reading its old value, so its prolongation is not needed.
template <typename T, int COL0>
__device__ __forceinline__ void op_prolong_v(const Lev& Lf, const Lev& Lc, T* __restrict__ v,
                                             const T* __restrict__ c, const T* __restrict__ c2,
                                             uint32_t g4) {
  constexpr int V = Vec<T>::V;
  int I0, J, K;
  dec_nat(g4 * V, Lc, I0, J, K);
  const int nc = Lc.n;
  const int Js[3] = {J == 0 ? nc - 1 : J - 1, J, J + 1 == nc ? 0 : J + 1};
  const int Ks[3] = {K == 0 ? nc - 1 : K - 1, K, K + 1 == nc ? 0 : K + 1};
  // x pass: ax[d][b][q][x] for coarse cell I0+q, child x
  T ax[3][3][V][2];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      T cx[V + 2];
      uint32_t pc[V + 2];
#pragma unroll
      for (int q = 0; q < V + 2; ++q) {
        int I = I0 - 1 + q;
        I = I < 0 ? I + nc : (I >= nc ? I - nc : I);
        pc[q] = pk_of(Lc, I, Js[b], Ks[d]);
        cx[q] = c[pc[q]];
      }
      if (c2) {
#pragma unroll
        for (int q = 0; q < V + 2; ++q) cx[q] -= c2[pc[q]];
      }
#pragma unroll
      for (int q = 0; q < V; ++q) {
        ax[d][b][q][0] = p34<T>(cx[q + 1], cx[q]);
        ax[d][b][q][1] = p34<T>(cx[q + 1], cx[q + 2]);
      }
    }
#pragma unroll
  for (int z = 0; z < 2; ++z)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int j = 2 * J + y, k = 2 * K + z;
      const uint32_t row = prow(Lf, j, k) + (uint32_t)I0;
#pragma unroll
      for (int col = COL0; col < 2; ++col) {
        const int x = (col + j + k) & 1;  // child parity of this colour in the row
        T* dst = v + (uint32_t)col * (uint32_t)Lf.half + row;
        T cur[V];
        ldv_nt<T>(dst, cur);
#pragma unroll
        for (int q = 0; q < V; ++q) {
          T ay[3];
#pragma unroll
          for (int d = 0; d < 3; ++d)
            ay[d] = p34<T>(ax[d][1][q][x], ax[d][y ? 2 : 0][q][x]);
          cur[q] += p34<T>(ay[1], ay[z ? 2 : 0]);
        }
        stv_nt<T>(dst, cur);
      }
    }
}
template <typename T, int COL0>
__global__ __launch_bounds__(kBlock) void k_prolong_v(Lev Lf, Lev Lc, T* __restrict__ v,
                                                      const T* __restrict__ c,
                                                      const T* __restrict__ c2) {
  uint32_t g4 = (uint32_t)gid();
  if (g4 < (uint32_t)(2 * Lc.half / Vec<T>::V)) op_prolong_v<T, COL0>(Lf, Lc, v, c, c2, g4);
}

// The same prolongation marching in z over coarse planes: a thread owns 4
// coarse cells of a row (natural I0..I0+3, J) and walks kt coarse planes,
// keeping the y-interpolated coarse difference of planes K-1, K, K+1 in
// registers; each new plane costs three coarse rows, each read as one
// 2-vector per colour plus its two edge cells.  Arithmetic and its order are
// those of op_prolong_v.  Requires nc % 4 == 0.
template <typename T>
struct Vec2Of;
template <>
struct Vec2Of<float> {
  typedef float2 type;
};
template <>
struct Vec2Of<double> {
  typedef double2 type;
};
// coarse row (J, K): cx[q] = (c - c2) at natural I0 - 1 + q, q = 0..5
template <typename T>
__device__ __forceinline__ void prolong_row(const Lev& Lc, const T* __restrict__ c,
                                            const T* __restrict__ c2, int I0, int J, int K,
                                            T* cx) {
  typedef typename Vec2Of<T>::type T2;
  const int p = (J + K) & 1;  // colour of the even cells of this row
  const uint32_t row = prow(Lc, J, K);
  const uint32_t he = (uint32_t)p * (uint32_t)Lc.half + row;       // even cells
  const uint32_t ho = (uint32_t)(1 - p) * (uint32_t)Lc.half + row; // odd cells
  const uint32_t o = (uint32_t)(I0 >> 1);
  const uint32_t om = I0 == 0 ? (uint32_t)Lc.nh - 1 : o - 1;       // cell I0 - 1 (odd)
  const uint32_t op = I0 + 4 == Lc.n ? 0u : o + 2;                 // cell I0 + 4 (even)
  T2 ev = *reinterpret_cast<const T2*>(c + he + o);
  T2 od = *reinterpret_cast<const T2*>(c + ho + o);
  cx[0] = c[ho + om];
  cx[1] = ev.x;
  cx[2] = od.x;
  cx[3] = ev.y;
  cx[4] = od.y;
  cx[5] = c[he + op];
  if (c2) {
    T2 ev2 = *reinterpret_cast<const T2*>(c2 + he + o);
    T2 od2 = *reinterpret_cast<const T2*>(c2 + ho + o);
    cx[0] -= c2[ho + om];
    cx[1] -= ev2.x;
    cx[2] -= od2.x;
    cx[3] -= ev2.y;
    cx[4] -= od2.y;
    cx[5] -= c2[he + op];
  }
}
// ay[y][q][x] of coarse plane K for the thread's row J (x, then y weights)
template <typename T>
__device__ __forceinline__ void prolong_plane(const Lev& Lc, const T* __restrict__ c,
                                              const T* __restrict__ c2, int I0, const int* Js,
                                              int K, T (*ay)[4][2]) {
  T ax[3][4][2];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    T cx[6];
    prolong_row<T>(Lc, c, c2, I0, Js[b], K, cx);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ax[b][q][0] = p34<T>(cx[q + 1], cx[q]);
      ax[b][q][1] = p34<T>(cx[q + 1], cx[q + 2]);
    }
  }
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int x = 0; x < 2; ++x)
        ay[y][q][x] = p34<T>(ax[1][q][x], ax[y ? 2 : 0][q][x]);
}
__host__ __device__ inline unsigned prolong_march_blocks(int nc, int kt) {
  const unsigned ngrp = (unsigned)nc * (unsigned)nc / 4u;
  return ((ngrp + kBlock - 1) / kBlock) * (unsigned)((nc + kt - 1) / kt);
}
template <typename T, int COL0>
__global__ __launch_bounds__(kBlock) void k_prolong_kv(Lev Lf, Lev Lc, T* __restrict__ v,
                                                       const T* __restrict__ c,
                                                       const T* __restrict__ c2, int kt) {
  const int nc = Lc.n;
  const uint32_t ngrp = (uint32_t)nc * (uint32_t)nc / 4u;
  const uint32_t nchunk = (ngrp + kBlock - 1) / kBlock;
  const uint32_t b = (uint32_t)xcd_block();
  const uint32_t kb = b / nchunk, chunk = b - kb * nchunk;
  const uint32_t grp = chunk * kBlock + threadIdx.x;
  const int K0 = (int)kb * kt;
  if (grp >= ngrp || K0 >= nc) return;
  const uint32_t gpr = (uint32_t)nc / 4u;  // groups per coarse row
  const int J = (int)(grp / gpr), I0 = (int)(grp - (uint32_t)J * gpr) * 4;
  const int K1 = K0 + kt < nc ? K0 + kt : nc;
  const int Js[3] = {J == 0 ? nc - 1 : J - 1, J, J + 1 == nc ? 0 : J + 1};
  T ay[3][2][4][2];  // planes K-1, K, K+1
  prolong_plane<T>(Lc, c, c2, I0, Js, K0 == 0 ? nc - 1 : K0 - 1, ay[0]);
  prolong_plane<T>(Lc, c, c2, I0, Js, K0, ay[1]);
  for (int K = K0; K < K1; ++K) {
    prolong_plane<T>(Lc, c, c2, I0, Js, K + 1 == nc ? 0 : K + 1, ay[2]);
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int j = 2 * J + y, k = 2 * K + z;
        const uint32_t row = prow(Lf, j, k) + (uint32_t)I0;
#pragma unroll
        for (int col = COL0; col < 2; ++col) {
          const int x = (col + j + k) & 1;
          T* dst = v + (uint32_t)col * (uint32_t)Lf.half + row;
          T cur[4];
          ldn_nt<T, 4>(dst, cur);
#pragma unroll
          for (int q = 0; q < 4; ++q)
            cur[q] += p34<T>(ay[1][y][q][x], ay[z ? 2 : 0][y][q][x]);
          stn_nt<T, 4>(dst, cur);
        }
      }
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          ay[0][y][q][x] = ay[1][y][q][x];
          ay[1][y][q][x] = ay[2][y][q][x];
        }
  }
}

// ---------------------------------------------------------------------------
// Prolongation fused into the first post-smoothing half-sweep of a smoother
// that solves each cell exactly (f(R), symmetron, the linear adjoint).
// There the prolonged colour-1 values e1 + P(c - c2) are read only as the
// neighbours of the colour-0 half-sweep: the colour-1 half-sweep after it
// overwrites e1 without reading it (and the colour-0 prolongation is not
// needed either).  So they are formed in registers and never stored, and
// the kernel writes colour 0 only: per fine cell it reads e1, the stored X
// and rho of colour 0 and 1/8 of the coarse data, instead of reading and
// writing e1 once more in a separate prolongation.
//
// A thread owns coarse cells I0..I0+3 of coarse row J (fine rows 2J, 2J+1,
// packed cells I0..I0+3 of both colours) and walks the coarse planes
// K0..K1-1, i.e. the fine planes 2K0..2K1-1.  A block holds the whole
// coarse rows J0..J0+R-1 (R >= 2, no tile of a single row); for each coarse
// plane its threads swap the colour-1 values of the two current fine
// planes through LDS (x and y neighbours), its first row also forms the
// outside fine row 2J0-1 and its last row 2(J0+R), from the coarse rows
// they load anyway.  z neighbours stay in registers.  The prolongation
// arithmetic is k_prolong_kv's, the neighbour sum and cell update those of
// the z-marching half-sweeps, so the result is bit-identical to the two
// kernels run one after the other.
// ---------------------------------------------------------------------------
// 4 stored cells as loaded, decoded later exactly as ld4s decodes them (so
// the loads can be issued before the LDS exchange and wait behind it)
template <typename TS>
struct Raw4 {
  nt_f4 v;
};
template <>
struct Raw4<h16> {
  nt_h4 v;
};
template <typename TS>
__device__ __forceinline__ Raw4<TS> ld4raw(const TS* __restrict__ p) {
  Raw4<TS> r;
  if constexpr (sizeof(TS) == 4) r.v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  else r.v = __builtin_nontemporal_load(reinterpret_cast<const nt_h4*>(p));
  return r;
}
template <typename TS>
__device__ __forceinline__ void dec4s(const Raw4<TS>& r, float dec, float* out) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if constexpr (sizeof(TS) == 4) out[q] = r.v[q];
    else out[q] = float(r.v[q]) * dec;
  }
}
// Cell update policies for four consecutive colour-0 cells at packed index
// q0: load() the cell data, apply() the update to the neighbour sums.
// kPreload: load a step's cell data before the LDS exchange (f(R), linear:
// 31.3 against 31.7 ms per 512^3 f(R) step); the symmetron's extra density
// operand would cost a wave per SIMD, so it loads after the exchange.
template <int M, typename TX, typename TR>
struct UpdCorr {
  static constexpr bool kPreload = M != SYM;
  const TX* X;
  const float* dens;
  const TR* rho;
  float h2;
  Store S;
  Consts C;
  struct In {
    Raw4<TX> x;
    Raw4<TR> r;
    Raw4<float> d;
  };
  __device__ __forceinline__ In load(uint32_t q0) const {
    In a;
    a.x = ld4raw<TX>(X + q0);
    a.r = ld4raw<TR>(rho + q0);
    if (M != FR) a.d = ld4raw<float>(dens + q0);
    return a;
  }
  __device__ __forceinline__ void apply(const In& a, const float* sum, float* out) const {
    float x[4], rr[4], dc[4] = {0, 0, 0, 0}, eo[4] = {0, 0, 0, 0};
    dec4s<TX>(a.x, S.x_dec, x);
    dec4s<TR>(a.r, S.r_dec, rr);
    if (M != FR) dec4s<float>(a.d, 1.0f, dc);
    corr_update4<M>(C, h2, eo, sum, x, dc, rr, out);
  }
};
template <typename TD, typename TR>
struct UpdLin {
  static constexpr bool kPreload = true;
  const TD* dg;
  const TR* r;
  float kh2;
  Store S;
  struct In {
    Raw4<TD> d;
    Raw4<TR> r;
  };
  __device__ __forceinline__ In load(uint32_t q0) const {
    In a;
    a.d = ld4raw<TD>(dg + q0);
    a.r = ld4raw<TR>(r + q0);
    return a;
  }
  __device__ __forceinline__ void apply(const In& a, const float* sum, float* out) const {
    float d[4], rr[4];
    dec4s<TD>(a.d, S.x_dec, d);
    dec4s<TR>(a.r, S.r_dec, rr);
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = lin_cell_f(rr[q], sum[q], d[q], kh2);
  }
};
// Coarse plane K interpolated in x and y for the fine rows 2J (a[0]) and
// 2J+1 (a[1]) of the thread's 4 coarse cells, both x children, and for one
// outside row h: 2J-1 (lo) or 2J+2 (!lo).  Same steps as prolong_plane.
__device__ __forceinline__ void prolong_plane_h(const Lev& Lc, const float* __restrict__ c,
                                                const float* __restrict__ c2, int I0,
                                                const int* Js, int K, bool lo,
                                                float (*a)[4][2], float (*h)[2]) {
  float ax[3][4][2];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    float cx[6];
    prolong_row<float>(Lc, c, c2, I0, Js[b], K, cx);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ax[b][q][0] = p34<float>(cx[q + 1], cx[q]);
      ax[b][q][1] = p34<float>(cx[q + 1], cx[q + 2]);
    }
  }
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int x = 0; x < 2; ++x) a[y][q][x] = p34<float>(ax[1][q][x], ax[y ? 2 : 0][q][x]);
  // row 2J-1 is child 1 of coarse row J-1, row 2J+2 child 0 of row J+1
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int x = 0; x < 2; ++x) h[q][x] = p34<float>(lo ? ax[0][q][x] : ax[2][q][x], ax[1][q][x]);
}
// LDS of one block: [buffer][fine plane of the pair][fine row of the block]
// [packed cell]; R rows of nc/4 threads fill at most kBlock threads, so
// 2R nc <= 8 kBlock.
constexpr int kPSRowCells = 8 * kBlock;
__host__ __device__ inline int prolong_smooth_rows(int nc) {
  if (nc % 4 != 0 || nc < 8 || nc / 4 > kBlock / 2) return 0;  // needs R >= 2
  int R = kBlock / (nc / 4);
  if (R > nc) R = nc;
  while (R > 2 && nc % R == 1) --R;  // no tile of a single coarse row
  return nc % R == 1 ? 0 : R;
}
template <class U>
__global__ __launch_bounds__(kBlock) void k_prolong_smooth0(Lev Lf, Lev Lc, float* __restrict__ e,
                                                            const float* __restrict__ c,
                                                            const float* __restrict__ c2, int kt,
                                                            U upd) {
  __shared__ __align__(16) float sh[2][2][kPSRowCells];
  const int nc = Lc.n, n = Lf.n, gpr = nc >> 2;
  const int R = (int)blockDim.x / gpr;
  const uint32_t ntile = ((uint32_t)nc + (uint32_t)R - 1) / (uint32_t)R;
  const uint32_t b = (uint32_t)xcd_block();
  const uint32_t kb = b / ntile, tile = b - kb * ntile;
  const int rl = (int)threadIdx.x / gpr, g = (int)threadIdx.x - rl * gpr;
  const int J0 = (int)tile * R, J = J0 + rl;
  const int Jend = J0 + R < nc ? J0 + R : nc;
  const bool act = J < nc;
  const int Jr = act ? J : nc - 1;  // rows past the last one compute a copy of it
  const bool first = J == J0, last = J == Jend - 1;
  const int I0 = 4 * g;
  const int K0 = (int)kb * kt, K1 = K0 + kt < nc ? K0 + kt : nc;
  const int Js[3] = {Jr == 0 ? nc - 1 : Jr - 1, Jr, Jr + 1 == nc ? 0 : Jr + 1};
  const int jh = first ? (Jr == 0 ? n - 1 : 2 * Jr - 1) : (Jr + 1 == nc ? 0 : 2 * Jr + 2);
  const bool need_h = act && (first || last);
  const float* e1 = e + Lf.half;
  // e1 + P on the fine plane k of own row y, from the interpolated coarse
  // planes `near` (weight 3/4) and `far`
  auto own_rows = [&](int k, const float (*near)[4][2], const float (*far)[4][2], float (*E)[4]) {
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int j = 2 * Jr + y, x = (1 + j + k) & 1;
      float old[4];
      ldn_nt<float, 4>(e1 + prow(Lf, j, k) + I0, old);
#pragma unroll
      for (int q = 0; q < 4; ++q) E[y][q] = old[q] + p34<float>(near[y][q][x], far[y][q][x]);
    }
  };
  auto out_row = [&](int k, const float (*near)[2], const float (*far)[2], float* E) {
    const int x = (1 + jh + k) & 1;
    float old[4] = {0, 0, 0, 0};
    if (need_h) ldn<float, 4>(e1 + prow(Lf, jh, k) + I0, old);
#pragma unroll
    for (int q = 0; q < 4; ++q) E[q] = old[q] + p34<float>(near[q][x], far[q][x]);
  };
  float aK[2][4][2], hK[4][2], aN[2][4][2], hN[4][2];
  float Eb[2][4];          // fine plane 2K-1, own rows
  float Ec[2][4], Ech[4];  // fine plane 2K: own rows, outside row
  {
    const int Kp = K0 == 0 ? nc - 1 : K0 - 1;
    prolong_plane_h(Lc, c, c2, I0, Js, Kp, first, aN, hN);
    prolong_plane_h(Lc, c, c2, I0, Js, K0, first, aK, hK);
    own_rows(K0 == 0 ? n - 1 : 2 * K0 - 1, aN, aK, Eb);  // child z = 1 of plane K0-1
    own_rows(2 * K0, aK, aN, Ec);                        // child z = 0 of plane K0
    out_row(2 * K0, hK, hN, Ech);
  }
  for (int K = K0; K < K1; ++K) {
    const int Kn = K + 1 == nc ? 0 : K + 1;
    const int k0 = 2 * K, k1 = 2 * K + 1, k2 = 2 * Kn;
    typename U::In in[2][2];  // cell data of the two planes' own rows
    if constexpr (U::kPreload) {
#pragma unroll
      for (int z = 0; z < 2; ++z)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          in[z][y] = upd.load(prow(Lf, 2 * Jr + y, k0 + z) + (uint32_t)I0);
    }
    prolong_plane_h(Lc, c, c2, I0, Js, Kn, first, aN, hN);
    float Ed[2][4], Edh[4], Ee[2][4], Eeh[4];
    own_rows(k1, aK, aN, Ed);  // child z = 1 of plane K
    out_row(k1, hK, hN, Edh);
    own_rows(k2, aN, aK, Ee);  // child z = 0 of plane K+1
    out_row(k2, hN, hK, Eeh);
    float* s0 = sh[K & 1][0];
    float* s1 = sh[K & 1][1];
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      stn<float, 4>(s0 + (2 * rl + y) * nc + I0, Ec[y]);
      stn<float, 4>(s1 + (2 * rl + y) * nc + I0, Ed[y]);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int z = 0; z < 2; ++z) {
        const float* s = z ? s1 : s0;
        const int k = z ? k1 : k0;
        const float(*cen)[4] = z ? Ed : Ec;
        const float(*zmv)[4] = z ? Ec : Eb;
        const float(*zpv)[4] = z ? Ee : Ed;
        const float* hv = z ? Edh : Ech;
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int j = 2 * Jr + y;
          const float* srow = s + (2 * rl + y) * nc;
          float xv[5], ym[4], yp[4], sum[4], out[4];
          if ((j + k) & 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[q] = cen[y][q];
            xv[4] = srow[I0 + 4 == nc ? 0 : I0 + 4];
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[q + 1] = cen[y][q];
            xv[0] = srow[I0 == 0 ? nc - 1 : I0 - 1];
          }
          if (y == 0) {
            if (first) {
#pragma unroll
              for (int q = 0; q < 4; ++q) ym[q] = hv[q];
            } else {
              ldn<float, 4>(srow - nc + I0, ym);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) yp[q] = cen[1][q];
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) ym[q] = cen[0][q];
            if (last) {
#pragma unroll
              for (int q = 0; q < 4; ++q) yp[q] = hv[q];
            } else {
              ldn<float, 4>(srow + nc + I0, yp);
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q)
            sum[q] = (xv[q] + xv[q + 1]) + (ym[q] + yp[q]) + (zmv[y][q] + zpv[y][q]);
          const uint32_t r = prow(Lf, j, k) + (uint32_t)I0;
          if constexpr (!U::kPreload) in[z][y] = upd.load(r);
          upd.apply(in[z][y], sum, out);
          stv_nt<float>(e + r, out);
        }
      }
    }
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Eb[y][q] = Ed[y][q];
        Ec[y][q] = Ee[y][q];
#pragma unroll
        for (int x = 0; x < 2; ++x) aK[y][q][x] = aN[y][q][x];
      }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Ech[q] = Eeh[q];
#pragma unroll
      for (int x = 0; x < 2; ++x) hK[q][x] = hN[q][x];
    }
  }
}

// correction form: Re -> eH and eR, R(G(e) - rho) -> rhoH, optionally R X -> XH.
// skip1: colour 1 was the last half-sweep of an exact per-cell smoother, so
// its residual vanishes (to rounding) and is not recomputed.
template <int M, typename TX = float, typename TR = float>
__device__ __forceinline__ void op_resid_restrict_corr_v(
    const Lev& Lf, const Lev& Lc, const float* __restrict__ e, const TX* __restrict__ X,
    const float* __restrict__ dens, const TR* __restrict__ rho, float h2, float* eH, float* eR,
    float* rhoH, float* XH, const Consts& C, int skip1, uint32_t g4,
    Store S = Store{1, 1, 1, 1}, float* Xf = nullptr, int rx = 0) {
  constexpr int V = Vec<float>::V;
  int I0, J, K;
  dec_nat(g4 * V, Lc, I0, J, K);
  const bool want_x = XH && (!Xf || rx);
  float se[V] = {0, 0, 0, 0}, sd[V] = {0, 0, 0, 0}, sx[V] = {0, 0, 0, 0};
#pragma unroll 1
  for (int d = 0; d < 2; ++d)
#pragma unroll 1
    for (int b = 0; b < 2; ++b) {
      const int j = 2 * J + b, k = 2 * K + d;
#pragma unroll 1
      for (int col = 0; col < 2; ++col) {
        const uint32_t q0 = (uint32_t)col * (uint32_t)Lf.half + prow(Lf, j, k) + (uint32_t)I0;
        float sum[V], ec[V], x[V], r[V], dc[V] = {0, 0, 0, 0};
        ldv<float>(e + q0, ec);
        if (col == 1 && skip1) {
#pragma unroll
          for (int q = 0; q < V; ++q) se[q] += ec[q];
          if (want_x) {
            ld4s<TX>(X + q0, S.x_dec, x);
#pragma unroll
            for (int q = 0; q < V; ++q) sx[q] += x[q];
          }
          continue;
        }
        nbsum_vec<float>(Lf, e + (1 - col) * Lf.half, I0, j, k, (j + k + col) & 1, sum);
        ld4s<TX>(X + q0, S.x_dec, x);
        ld4s<TR>(rho + q0, S.r_dec, r);
        if (M != FR) ldv_nt<float>(dens + q0, dc);
#pragma unroll
        for (int q = 0; q < V; ++q) {
          se[q] += ec[q];
          sx[q] += x[q];
          sd[q] += corr_G<M>(C, h2, ec[q], sum[q], x[q], dc[q]) - r[q];
        }
      }
    }
#pragma unroll
  for (int q = 0; q < V; ++q)
    store_coarse_corr(pk_of(Lc, I0 + q, J, K), se[q], sd[q], sx[q], eH, eR, rhoH, XH, Xf, rx);
}
template <int M, typename TX = float, typename TR = float>
__global__ __launch_bounds__(kBlock) void k_resid_restrict_corr_v(
    Lev Lf, Lev Lc, const float* __restrict__ e, const TX* __restrict__ X,
    const float* __restrict__ dens, const TR* __restrict__ rho, float h2, float* eH, float* eR,
    float* rhoH, float* XH, Consts C, int skip1, Store S = Store{1, 1, 1, 1},
    float* Xf = nullptr, int rx = 0) {
  uint32_t g4 = (uint32_t)gid();
  if (g4 < (uint32_t)(2 * Lc.half / Vec<float>::V))
    op_resid_restrict_corr_v<M, TX, TR>(Lf, Lc, e, X, dens, rho, h2, eH, eR, rhoH, XH, C, skip1,
                                        g4, S, Xf, rx);
}

// Residual and restriction marching in z, for exact per-cell smoothers
// (colour 1, swept last, has zero residual and is only restricted).  A
// thread owns 4 coarse cells (natural I0..I0+3, row J) and walks kt coarse
// planes; the colour-1 rows of fine planes 2K and 2K-1 around its two fine
// rows stay in registers, so each step reads the colour-1 rows of planes
// 2K+1 and 2K+2 once.  Per-cell arithmetic and every summation order are
// those of op_resid_restrict_corr_v and k_lin_resid_restrict_v; coarse
// results are written as one 2-vector per colour.  Requires nc % 4 == 0.
template <typename T>
struct RestrictWin {
  T zm[2][4];  // colour-1 rows (2J+b, 2K-1)
  T zc[2][4];  // colour-1 rows (2J+b, 2K)
};
// neighbour sum of the 4 colour-0 cells (I0.., j, k) from colour-1 rows:
// centre c (x neighbours), y- ym, y+ yp, z- zm, z+ zp; same order as nbsum_vec
template <typename T>
__device__ __forceinline__ void rr_nbsum(const Lev& Lf, const T* __restrict__ o1, int I0, int j,
                                         int k, const T* c, const T* ym, const T* yp,
                                         const T* zm, const T* zp, T* sum) {
  const uint32_t r = prow(Lf, j, k);
  T xv[5];
  if ((j + k) & 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) xv[q] = c[q];
    xv[4] = o1[r + (I0 + 4 == Lf.nh ? 0 : I0 + 4)];
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) xv[q + 1] = c[q];
    xv[0] = o1[r + (I0 == 0 ? Lf.nh - 1 : I0 - 1)];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) sum[q] = (xv[q] + xv[q + 1]) + (ym[q] + yp[q]) + (zm[q] + zp[q]);
}
// store 4 natural coarse values of row (J, K) from I0: even cells share one
// colour's 2-vector, odd cells the other's
template <typename T>
__device__ __forceinline__ void st_coarse4(const Lev& Lc, T* __restrict__ a, int I0, int J, int K,
                                           const T* v) {
  typedef typename Vec2Of<T>::type T2;
  const int p = (J + K) & 1;
  const uint32_t row = prow(Lc, J, K) + (uint32_t)(I0 >> 1);
  T2 ev, od;
  ev.x = v[0];
  ev.y = v[2];
  od.x = v[1];
  od.y = v[3];
  *reinterpret_cast<T2*>(a + (uint32_t)p * (uint32_t)Lc.half + row) = ev;
  *reinterpret_cast<T2*>(a + (uint32_t)(1 - p) * (uint32_t)Lc.half + row) = od;
}
// load 4 natural coarse values of row (J, K) from I0 (st_coarse4's layout)
template <typename T>
__device__ __forceinline__ void ld_coarse4(const Lev& Lc, const T* __restrict__ a, int I0, int J,
                                           int K, T* v) {
  typedef typename Vec2Of<T>::type T2;
  const int p = (J + K) & 1;
  const uint32_t row = prow(Lc, J, K) + (uint32_t)(I0 >> 1);
  const T2 ev = *reinterpret_cast<const T2*>(a + (uint32_t)p * (uint32_t)Lc.half + row);
  const T2 od = *reinterpret_cast<const T2*>(a + (uint32_t)(1 - p) * (uint32_t)Lc.half + row);
  v[0] = ev.x;
  v[2] = ev.y;
  v[1] = od.x;
  v[3] = od.y;
}
struct RRPos {
  int I0, J, Jm2, Jp2, K0, K1;  // Jm2 = fine row 2J-1, Jp2 = fine row 2J+2 (periodic)
  bool ok;
};
__device__ __forceinline__ RRPos rr_pos(const Lev& Lc, int kt) {
  RRPos P;
  const int nc = Lc.n;
  const uint32_t ngrp = (uint32_t)nc * (uint32_t)nc / 4u;
  const uint32_t nchunk = (ngrp + kBlock - 1) / kBlock;
  const uint32_t b = (uint32_t)xcd_block();
  const uint32_t kb = b / nchunk, chunk = b - kb * nchunk;
  const uint32_t grp = chunk * kBlock + threadIdx.x;
  P.K0 = (int)kb * kt;
  P.ok = grp < ngrp && P.K0 < nc;
  const uint32_t gpr = (uint32_t)nc / 4u;
  P.J = (int)(grp / gpr);
  P.I0 = (int)(grp - (uint32_t)P.J * gpr) * 4;
  const int n = 2 * nc;
  P.Jm2 = P.J == 0 ? n - 1 : 2 * P.J - 1;
  P.Jp2 = 2 * P.J + 2 == n ? 0 : 2 * P.J + 2;
  P.K1 = P.K0 + kt < nc ? P.K0 + kt : nc;
  return P;
}
template <int M, typename TX = float, typename TR = float>
__global__ __launch_bounds__(kBlock) void k_resid_restrict_corr_kv(
    Lev Lf, Lev Lc, const float* __restrict__ e, const TX* __restrict__ X,
    const float* __restrict__ dens, const TR* __restrict__ rho, float h2,
    float* __restrict__ eH, float* __restrict__ eR, float* __restrict__ rhoH,
    float* __restrict__ XH, Consts C, int kt, Store S = Store{1, 1, 1, 1}, float* Xf = nullptr,
    int rx = 0) {
  const RRPos P = rr_pos(Lc, kt);
  if (!P.ok) return;
  const int n = Lf.n, I0 = P.I0, J = P.J;
  const bool want_x = XH && (!Xf || rx);
  const float* o1 = e + Lf.half;
  auto row1 = [&](int j, int k, float* v) { ldn<float, 4>(o1 + prow(Lf, j, k) + I0, v); };
  RestrictWin<float> W;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    row1(2 * J + b, P.K0 == 0 ? n - 1 : 2 * P.K0 - 1, W.zm[b]);
    row1(2 * J + b, 2 * P.K0, W.zc[b]);
  }
  for (int K = P.K0; K < P.K1; ++K) {
    float c1[2][4], c2[2][4];  // colour-1 rows of planes 2K+1 and 2K+2
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      row1(2 * J + b, 2 * K + 1, c1[b]);
      row1(2 * J + b, 2 * K + 2 == n ? 0 : 2 * K + 2, c2[b]);
    }
    float se[4] = {0, 0, 0, 0}, sd[4] = {0, 0, 0, 0}, sx[4] = {0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int k = 2 * K + d;
      float ym[4], yp[4];
      row1(P.Jm2, k, ym);
      row1(P.Jp2, k, yp);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = 2 * J + b;
        const float* cen = d ? c1[b] : W.zc[b];
        const float* zmv = d ? W.zc[b] : W.zm[b];
        const float* zpv = d ? c2[b] : c1[b];
        const float* ymv = b ? (d ? c1[0] : W.zc[0]) : ym;
        const float* ypv = b ? yp : (d ? c1[1] : W.zc[1]);
        const uint32_t q0 = prow(Lf, j, k) + (uint32_t)I0;
        float sum[4], ec[4], x[4], r[4], dc[4] = {0, 0, 0, 0};
        rr_nbsum<float>(Lf, o1, I0, j, k, cen, ymv, ypv, zmv, zpv, sum);
        ldn<float, 4>(e + q0, ec);
        ld4s<TX>(X + q0, S.x_dec, x);
        ld4s<TR>(rho + q0, S.r_dec, r);
        if (M != FR) ldn_nt<float, 4>(dens + q0, dc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          se[q] += ec[q];
          sx[q] += x[q];
          sd[q] += corr_G<M>(C, h2, ec[q], sum[q], x[q], dc[q]) - r[q];
        }
        // colour 1: restricted only
#pragma unroll
        for (int q = 0; q < 4; ++q) se[q] += cen[q];
        if (want_x) {
          ld4s<TX>(X + Lf.half + q0, S.x_dec, x);
#pragma unroll
          for (int q = 0; q < 4; ++q) sx[q] += x[q];
        }
      }
    }
    // coarse outputs as in store_coarse_corr, 4 natural cells at a time
    float re[4], rd[4], rxv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      re[q] = se[q] * 0.125f;
      rd[q] = Xf ? -(sd[q] * 0.125f) : sd[q] * 0.125f;
      rxv[q] = sx[q] * 0.125f;
    }
    st_coarse4<float>(Lc, rhoH, I0, J, K, rd);
    if (Xf) {
      if (rx) st_coarse4<float>(Lc, Xf, I0, J, K, rxv);
      else ld_coarse4<float>(Lc, Xf, I0, J, K, rxv);
      float xn[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) xn[q] = rxv[q] + re[q];
      st_coarse4<float>(Lc, XH, I0, J, K, xn);
      if (eH) {
        const float zero[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        st_coarse4<float>(Lc, eH, I0, J, K, zero);
      }
    } else {
      st_coarse4<float>(Lc, eH, I0, J, K, re);
      st_coarse4<float>(Lc, eR, I0, J, K, re);
      if (XH) st_coarse4<float>(Lc, XH, I0, J, K, rxv);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        W.zm[b][q] = c1[b][q];
        W.zc[b][q] = c2[b][q];
      }
  }
}
template <typename T, typename TD = T, typename TR = T>
__global__ __launch_bounds__(kBlock) void k_lin_resid_restrict_kv(Lev Lf, Lev Lc,
                                                                  const T* __restrict__ e,
                                                                  const TD* __restrict__ dg,
                                                                  const TR* __restrict__ r, T kh2,
                                                                  T* __restrict__ rH,
                                                                  T* __restrict__ eH, int kt,
                                                                  Store S = Store{1, 1, 1, 1}) {
  const RRPos P = rr_pos(Lc, kt);
  if (!P.ok) return;
  const int n = Lf.n, I0 = P.I0, J = P.J;
  const T* o1 = e + Lf.half;
  auto row1 = [&](int j, int k, T* v) { ldn<T, 4>(o1 + prow(Lf, j, k) + I0, v); };
  RestrictWin<T> W;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    row1(2 * J + b, P.K0 == 0 ? n - 1 : 2 * P.K0 - 1, W.zm[b]);
    row1(2 * J + b, 2 * P.K0, W.zc[b]);
  }
  const T zero[4] = {T(0), T(0), T(0), T(0)};
  for (int K = P.K0; K < P.K1; ++K) {
    T c1[2][4], c2[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      row1(2 * J + b, 2 * K + 1, c1[b]);
      row1(2 * J + b, 2 * K + 2 == n ? 0 : 2 * K + 2, c2[b]);
    }
    T sd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) sd[q] = T(0);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int k = 2 * K + d;
      T ym[4], yp[4];
      row1(P.Jm2, k, ym);
      row1(P.Jp2, k, yp);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = 2 * J + b;
        const T* cen = d ? c1[b] : W.zc[b];
        const T* zmv = d ? W.zc[b] : W.zm[b];
        const T* zpv = d ? c2[b] : c1[b];
        const T* ymv = b ? (d ? c1[0] : W.zc[0]) : ym;
        const T* ypv = b ? yp : (d ? c1[1] : W.zc[1]);
        const uint32_t q0 = prow(Lf, j, k) + (uint32_t)I0;
        T sum[4], ec[4], dd[4], rr[4];
        rr_nbsum<T>(Lf, o1, I0, j, k, cen, ymv, ypv, zmv, zpv, sum);
        ldn<T, 4>(e + q0, ec);
        ldNs<T, TD, 4>(dg + q0, S.x_dec, dd);
        ldNs<T, TR, 4>(r + q0, S.r_dec, rr);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          sd[q] += rr[q] - (kh2 * (T(6) * ec[q] - sum[q]) + dd[q] * ec[q]);
      }
    }
    T rd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rd[q] = sd[q] * T(0.125);
    st_coarse4<T>(Lc, rH, I0, J, K, rd);
    st_coarse4<T>(Lc, eH, I0, J, K, zero);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        W.zm[b][q] = c1[b][q];
        W.zc[b][q] = c2[b][q];
      }
  }
}

// direct form: R v -> Rv and vinit, R(L(v) - S) -> Sd
template <int M, typename TD>
__global__ __launch_bounds__(kBlock) void k_resid_restrict_direct_v(
    Lev Lf, Lev Lc, const double* __restrict__ v, const TD* __restrict__ dens,
    const double* __restrict__ S, double h2, double* Rv, double* vinit, double* Sd, Consts C,
    int skip1) {
  constexpr int V = Vec<double>::V;
  uint32_t g4 = (uint32_t)gid();
  if (g4 >= (uint32_t)(2 * Lc.half / V)) return;
  int I0, J, K;
  dec_nat(g4 * V, Lc, I0, J, K);
  double sv[V] = {0, 0}, sd[V] = {0, 0};
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = 2 * J + b, k = 2 * K + d;
#pragma unroll
      for (int col = 0; col < 2; ++col) {
        const uint32_t q0 = (uint32_t)col * (uint32_t)Lf.half + prow(Lf, j, k) + (uint32_t)I0;
        double sum[V], vc[V], sc[V] = {0, 0};
        ldv<double>(v + q0, vc);
        if (col == 1 && skip1) {  // residual of the last exact half-sweep: zero
#pragma unroll
          for (int q = 0; q < V; ++q) sv[q] += vc[q];
          continue;
        }
        nbsum_vec<double>(Lf, v + (1 - col) * Lf.half, I0, j, k, (j + k + col) & 1, sum);
        if (S) ldv<double>(S + q0, sc);
#pragma unroll
        for (int q = 0; q < V; ++q) {
          sv[q] += vc[q];
          sd[q] += direct_resid<M, double>(C, h2, vc[q], sum[q], double(dens[q0 + q]), sc[q]);
        }
      }
    }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    uint32_t pc = pk_of(Lc, I0 + q, J, K);
    double rv = sv[q] * 0.125;
    Rv[pc] = rv;
    vinit[pc] = rv;
    Sd[pc] = sd[q] * 0.125;
  }
}

// linear: rH = R(r - A e), eH = 0
template <typename T, typename TD = T, typename TR = T>
__global__ __launch_bounds__(kBlock) void k_lin_resid_restrict_v(Lev Lf, Lev Lc,
                                                                 const T* __restrict__ e,
                                                                 const TD* __restrict__ dg,
                                                                 const TR* __restrict__ r, T kh2,
                                                                 T* rH, T* eH, int skip1,
                                                                 Store S = Store{1, 1, 1, 1}) {
  constexpr int V = Vec<T>::V;
  uint32_t g4 = (uint32_t)gid();
  if (g4 >= (uint32_t)(2 * Lc.half / V)) return;
  int I0, J, K;
  dec_nat(g4 * V, Lc, I0, J, K);
  T sd[V];
#pragma unroll
  for (int q = 0; q < V; ++q) sd[q] = T(0);
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = 2 * J + b, k = 2 * K + d;
      // skip1: colour 1 was the last (exact) half-sweep, its residual is zero
      for (int col = 0; col < 2 - skip1; ++col) {
        const uint32_t q0 = (uint32_t)col * (uint32_t)Lf.half + prow(Lf, j, k) + (uint32_t)I0;
        T sum[V], ec[V], dd[V], rr[V];
        nbsum_vec<T>(Lf, e + (1 - col) * Lf.half, I0, j, k, (j + k + col) & 1, sum);
        ldv<T>(e + q0, ec);
        ldNs<T, TD, V>(dg + q0, S.x_dec, dd);
        ldNs<T, TR, V>(r + q0, S.r_dec, rr);
#pragma unroll
        for (int q = 0; q < V; ++q) sd[q] += rr[q] - (kh2 * (T(6) * ec[q] - sum[q]) + dd[q] * ec[q]);
      }
    }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    uint32_t pc = pk_of(Lc, I0 + q, J, K);
    rH[pc] = sd[q] * T(0.125);
    eH[pc] = T(0);
  }
}

// ---------------------------------------------------------------------------
// Grid kernels (one cell per thread)
// ---------------------------------------------------------------------------
template <int M, typename T, typename TD>
__global__ __launch_bounds__(kBlock) void k_smooth_direct(Lev L, T* v, const TD* dens, const T* S,
                                                          int colour, T h2, Consts C) {
  int64_t g = gid();
  if (g < L.half) op_smooth_direct<M, T, TD>(L, v, dens, S, colour, h2, C, g);
}
template <int M, typename T, typename TD>
__global__ __launch_bounds__(kBlock) void k_resid_restrict_direct(Lev Lf, Lev Lc, const T* v,
                                                                  const TD* dens, const T* S,
                                                                  T h2, T* Rv, T* vinit, T* Sd,
                                                                  Consts C) {
  int64_t g = gid();
  if (g < 2 * Lc.half)
    op_resid_restrict_direct<M, T, TD>(Lf, Lc, v, dens, S, h2, Rv, vinit, Sd, C, g);
}
template <int M, typename T, typename TD>
__global__ __launch_bounds__(kBlock) void k_coarse_src_direct(Lev L, const T* Rv, const TD* dens,
                                                              T* S, T h2, Consts C) {
  int64_t g = gid();
  if (g < 2 * L.half) op_coarse_src_direct<M, T, TD>(L, Rv, dens, S, h2, C, g);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_block(Lev Lf, Lev Lc, T* v, const T* c) {
  int64_t g = gid();
  if (g < 2 * Lc.half) op_prolong_block<T>(Lf, Lc, v, c, g);
}
// c = vH - c (coarse correction formed in place of R v)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_diff(int64_t m, const T* vH, T* c) {
  int64_t g = gid();
  if (g < m) c[g] = vH[g] - c[g];
}
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_restrict(Lev Lf, Lev Lc, const TI* f, TO* c) {
  int64_t g = gid();
  if (g < 2 * Lc.half) op_restrict<TI, TO>(Lf, Lc, f, c, g);
}
// residual of the finest level: sum of d^2 per block (+ optional natural d)
template <int M, typename T, typename TD>
__global__ __launch_bounds__(kBlock) void k_resid_norm_direct(Lev L, const T* v, const TD* dens,
                                                              T h2, Consts C, double* part,
                                                              double* d_nat) {
  __shared__ double sh[32];
  int64_t g = gid();
  double d = 0.0;
  if (g < 2 * L.half) {
    d = double(cell_resid_direct<M, T, TD>(L, v, dens, (const T*)nullptr, h2, C, g));
    if (d_nat) {
      int colour = g >= L.half ? 1 : 0;
      int64_t gg = g - colour * L.half;
      int ih, j, k;
      dec(gg, L, ih, j, k);
      int i = 2 * ih + ((j + k + colour) & 1);
      d_nat[((int64_t)k * L.n + j) * L.n + i] = d;
    }
  }
  double t = block_sum(d * d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
// sum of (coef * delta)^2 per block: background residual
__global__ __launch_bounds__(kBlock) void k_bg_norm(int64_t m, const float* delta, double coef,
                                                   double* part) {
  __shared__ double sh[32];
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d = g < m ? coef * double(delta[g]) : 0.0;
  double t = block_sum(d * d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_smooth_corr(Lev L, float* e, const float* X,
                                                        const float* dens, const float* rho,
                                                        int colour, float h2, Consts C) {
  int64_t g = gid();
  if (g < L.half) op_smooth_corr<M>(L, e, X, dens, rho, colour, h2, C, g);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_resid_restrict_corr(Lev Lf, Lev Lc, const float* e,
                                                                const float* X, const float* dens,
                                                                const float* rho, float h2,
                                                                float* eH, float* eR, float* rhoH,
                                                                float* XH, Consts C,
                                                                float* Xf = nullptr, int rx = 0) {
  int64_t g = gid();
  if (g < 2 * Lc.half)
    op_resid_restrict_corr<M>(Lf, Lc, e, X, dens, rho, h2, eH, eR, rhoH, XH, C, g, Xf, rx);
}
// FP64 outer step of the refined mode: d = F(w64) (FP64), rho = -d, X = w64,
// e = 0; per-block sum of d^2.
template <int M>
__global__ __launch_bounds__(kBlock) void k_outer_residual(Lev L, const double* w, const float* dens,
                                                           Consts C, float* rho, float* X,
                                                           float* e, double* part) {
  __shared__ double sh[32];
  int64_t g = gid();
  double d = 0.0;
  if (g < 2 * L.half) {
    d = cell_resid_direct<M, double, float>(L, w, dens, (const double*)nullptr, 1.0, C, g);
    rho[g] = float(-d);
    X[g] = float(w[g]);
    e[g] = 0.0f;
  }
  double t = block_sum(d * d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
__global__ __launch_bounds__(kBlock) void k_outer_update(int64_t m, double* w, const float* e) {
  int64_t g = gid();
  if (g < m) w[g] += double(e[g]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_smooth_lin(Lev L, T* e, const T* dg, const T* r,
                                                       int colour, T kh2) {
  int64_t g = gid();
  if (g < L.half) op_smooth_lin<T>(L, e, dg, r, colour, kh2, g);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lin_resid_restrict(Lev Lf, Lev Lc, const T* e,
                                                               const T* dg, const T* r, T kh2,
                                                               T* rH, T* eH) {
  int64_t g = gid();
  if (g < 2 * Lc.half) op_lin_resid_restrict<T>(Lf, Lc, e, dg, r, kh2, rH, eH, g);
}
// FP64 outer step of the adjoint: r = b - A lam (FP64) -> r (inner
// precision), e = 0, per-block sum of r^2
template <typename TO>
__global__ __launch_bounds__(kBlock) void k_lin_outer(Lev L, const double* lam, const double* dg,
                                                      const double* b, double kh2, TO* r,
                                                      TO* e, double* part, double* part_sum) {
  __shared__ double sh[32];
  int64_t g = gid();
  double d = 0.0;
  if (g < 2 * L.half) {
    d = cell_lin_resid<double>(L, lam, dg, b, kh2, g);
    r[g] = TO(d);
    e[g] = TO(0);
  }
  double t = block_sum(d * d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
  if (part_sum) {
    t = block_sum(d, sh);
    if (threadIdx.x == 0) part_sum[blockIdx.x] = t;
  }
}
// partial sums of a[g] * b[g] (b null: of a[g])
template <typename TA>
__global__ __launch_bounds__(kBlock) void k_dot(int64_t m, const TA* a, const double* b,
                                                double* part) {
  __shared__ double sh[32];
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d = g < m ? double(a[g]) * (b ? b[g] : 1.0) : 0.0;
  double t = block_sum(d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
__global__ __launch_bounds__(kBlock) void k_add_const(int64_t m, double* y, double c) {
  int64_t g = gid();
  if (g < m) y[g] += c;
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy_to64(int64_t m, double* y, const T* x) {
  int64_t g = gid();
  if (g < m) y[g] += double(x[g]);
}
// ---------------------------------------------------------------------------
// Fused coarse cycle: one workgroup runs a precomputed program of level
// operations on the small levels (latency-bound as separate launches).
// ---------------------------------------------------------------------------
enum { OP_SMOOTH = 0, OP_DOWN = 1, OP_UP = 2, OP_COARSEST = 3 };
struct Op {
  uint8_t kind, lev, count, pad;
};
struct FusedProg {
  int nops;
  int coarse_sweeps;
  int rx;  // correction form: also restrict the linearisation point X on the way down
  Op op[kMaxOps];
};
// Level pointers of the fused part (index = level - first fused level).
template <typename T, typename TD>
struct FusedDirect {
  int nlev;
  Lev L[kMaxFused];
  T h2[kMaxFused];
  T* v[kMaxFused];
  const TD* dens[kMaxFused];
  T* S[kMaxFused];
  T* Rv[kMaxFused];
};
struct FusedCorr {
  int nlev;
  Lev L[kMaxFused];
  float h2[kMaxFused];
  float* e[kMaxFused];
  float* X[kMaxFused];
  const float* dens[kMaxFused];
  float* rho[kMaxFused];
  float* eR[kMaxFused];
};
template <typename T>
struct FusedLin {
  int nlev;
  Lev L[kMaxFused];
  T kh2[kMaxFused];
  T* e[kMaxFused];
  T* dg[kMaxFused];
  T* r[kMaxFused];
};

constexpr int kFusedThreads = 1024;

template <int M, typename T, typename TD>
__global__ __launch_bounds__(kFusedThreads) void k_fused_direct(FusedDirect<T, TD> F, FusedProg P,
                                                                Consts C) {
  __shared__ double sh[32];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int o = 0; o < P.nops; ++o) {
    const Op op = P.op[o];
    const int l = op.lev;
    const Lev L = F.L[l];
    if (op.kind == OP_SMOOTH) {
      for (int it = 0; it < op.count; ++it)
        for (int colour = 0; colour < 2; ++colour) {
          for (int64_t g = tid; g < L.half; g += nt)
            op_smooth_direct<M, T, TD>(L, F.v[l], F.dens[l], F.S[l], colour, F.h2[l], C, g);
          __syncthreads();
        }
    } else if (op.kind == OP_DOWN) {
      const Lev Lc = F.L[l + 1];
      for (int64_t g = tid; g < 2 * Lc.half; g += nt)
        op_resid_restrict_direct<M, T, TD>(L, Lc, F.v[l], F.dens[l], F.S[l], F.h2[l], F.Rv[l + 1],
                                           F.v[l + 1], F.S[l + 1], C, g);
      __syncthreads();
      for (int64_t g = tid; g < 2 * Lc.half; g += nt)
        op_coarse_src_direct<M, T, TD>(Lc, F.Rv[l + 1], F.dens[l + 1], F.S[l + 1], F.h2[l + 1], C,
                                       g);
      __syncthreads();
    } else if (op.kind == OP_UP) {
      const Lev Lc = F.L[l + 1];
      for (int64_t g = tid; g < 2 * L.half; g += nt)
        op_prolong_add<T>(L, Lc, F.v[l], F.v[l + 1], F.Rv[l + 1], g);
      __syncthreads();
    } else {  // coarsest: relax until RMS residual drops by 1e-10
      double r0 = -1.0;
      for (int it = 0; it < P.coarse_sweeps; ++it) {
        for (int colour = 0; colour < 2; ++colour) {
          for (int64_t g = tid; g < L.half; g += nt)
            op_smooth_direct<M, T, TD>(L, F.v[l], F.dens[l], F.S[l], colour, F.h2[l], C, g);
          __syncthreads();
        }
        if ((it & 3) != 3 && it + 1 < P.coarse_sweeps) continue;
        double s2 = 0.0, sd = 0.0, sj = 0.0;
        for (int64_t g = tid; g < 2 * L.half; g += nt) {
          double d = double(cell_resid_direct<M, T, TD>(L, F.v[l], F.dens[l], F.S[l], F.h2[l], C, g));
          s2 += d * d;
          if (M == CQ) {
            sd += d;
            sj += double(direct_diag<M, T>(C, F.h2[l], F.v[l][g], T(F.dens[l][g]))) + 6.0 / double(F.h2[l]);
          }
        }
        double tot = block_sum_all(s2, sh);
        if (M == CQ) {
          // uniform-mode Newton step: the Laplacian of a constant vanishes,
          // so sum_c F_c(v + mu) changes only through the per-cell terms
          double D = block_sum_all(sd, sh);
          double Jd = block_sum_all(sj, sh);
          if (Jd != 0.0) {
            T mu = T(-D / Jd);
            for (int64_t g = tid; g < 2 * L.half; g += nt) F.v[l][g] += mu;
          }
          __syncthreads();
        }
        if (r0 < 0.0) r0 = tot;
        if (tot <= 1e-16 * r0 || tot == 0.0) break;
      }
    }
  }
}

template <int M>
__device__ __forceinline__ void fused_corr_body(const FusedCorr& F, const FusedProg& P,
                                                const Consts& C, double* sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int o = 0; o < P.nops; ++o) {
    const Op op = P.op[o];
    const int l = op.lev;
    const Lev L = F.L[l];
    if (op.kind == OP_SMOOTH) {
      for (int it = 0; it < op.count; ++it)
        for (int colour = 0; colour < 2; ++colour) {
          for (int64_t g = tid; g < L.half; g += nt)
            op_smooth_corr<M>(L, F.e[l], F.X[l], F.dens[l], F.rho[l], colour, F.h2[l], C, g);
          __syncthreads();
        }
    } else if (op.kind == OP_DOWN) {
      const Lev Lc = F.L[l + 1];
      for (int64_t g = tid; g < 2 * Lc.half; g += nt)
        op_resid_restrict_corr<M>(L, Lc, F.e[l], F.X[l], F.dens[l], F.rho[l], F.h2[l], F.e[l + 1],
                                  F.eR[l + 1], F.rho[l + 1], P.rx ? F.X[l + 1] : (float*)nullptr,
                                  C, g);
      __syncthreads();
      for (int64_t g = tid; g < 2 * Lc.half; g += nt)
        op_coarse_src_corr<M>(Lc, F.eR[l + 1], F.X[l + 1], F.dens[l + 1], F.rho[l + 1], F.h2[l + 1],
                              C, g);
      __syncthreads();
    } else if (op.kind == OP_UP) {
      const Lev Lc = F.L[l + 1];
      for (int64_t g = tid; g < 2 * L.half; g += nt)
        op_prolong_add<float>(L, Lc, F.e[l], F.e[l + 1], F.eR[l + 1], g);
      __syncthreads();
    } else {
      double r0 = -1.0;
      for (int it = 0; it < P.coarse_sweeps; ++it) {
        for (int colour = 0; colour < 2; ++colour) {
          for (int64_t g = tid; g < L.half; g += nt)
            op_smooth_corr<M>(L, F.e[l], F.X[l], F.dens[l], F.rho[l], colour, F.h2[l], C, g);
          __syncthreads();
        }
        if ((it & 3) != 3 && it + 1 < P.coarse_sweeps) continue;
        double s2 = 0.0, sd = 0.0, sj = 0.0;
        for (int64_t g = tid; g < 2 * L.half; g += nt) {
          double d = double(cell_resid_corr<M>(L, F.e[l], F.X[l], F.dens[l], F.rho[l], F.h2[l], C, g));
          s2 += d * d;
          if (M == CQ) {
            sd += d;
            float dc = F.dens[l][g];
            sj += double(corr_diag<M>(C, F.h2[l], F.e[l][g], F.X[l][g], dc)) + 6.0 / double(F.h2[l]);
          }
        }
        double tot = block_sum_all(s2, sh);
        if (M == CQ) {
          double D = block_sum_all(sd, sh);
          double Jd = block_sum_all(sj, sh);
          if (Jd != 0.0) {
            float mu = float(-D / Jd);
            for (int64_t g = tid; g < 2 * L.half; g += nt) F.e[l][g] += mu;
          }
          __syncthreads();
        }
        if (r0 < 0.0) r0 = tot;
        if (tot <= 1e-16 * r0 || tot == 0.0) break;
      }
    }
  }
}
template <int M>
__global__ __launch_bounds__(kFusedThreads) void k_fused_corr(FusedCorr F, FusedProg P, Consts C) {
  __shared__ double sh[32];
  fused_corr_body<M>(F, P, C, sh);
}


template <typename T>
__global__ __launch_bounds__(kFusedThreads) void k_fused_lin(FusedLin<T> F, FusedProg P) {
  __shared__ double sh[32];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int o = 0; o < P.nops; ++o) {
    const Op op = P.op[o];
    const int l = op.lev;
    const Lev L = F.L[l];
    if (op.kind == OP_SMOOTH || op.kind == OP_COARSEST) {
      int count = op.kind == OP_SMOOTH ? op.count : P.coarse_sweeps;
      double r0 = -1.0;
      for (int it = 0; it < count; ++it) {
        for (int colour = 0; colour < 2; ++colour) {
          for (int64_t g = tid; g < L.half; g += nt)
            op_smooth_lin<T>(L, F.e[l], F.dg[l], F.r[l], colour, F.kh2[l], g);
          __syncthreads();
        }
        if (op.kind == OP_COARSEST && ((it & 3) == 3 || it + 1 == count)) {
          double s2 = 0.0, sd = 0.0, sj = 0.0;
          for (int64_t g = tid; g < 2 * L.half; g += nt) {
            double d = double(cell_lin_resid<T>(L, F.e[l], F.dg[l], F.r[l], F.kh2[l], g));
            s2 += d * d;
            sd += d;
            sj += double(F.dg[l][g]);
          }
          double tot = block_sum_all(s2, sh);
          double D = block_sum_all(sd, sh);
          double Jd = block_sum_all(sj, sh);
          if (Jd != 0.0) {  // uniform-mode correction (A 1 = dg)
            T mu = T(D / Jd);
            for (int64_t g = tid; g < 2 * L.half; g += nt) F.e[l][g] += mu;
          }
          __syncthreads();
          if (r0 < 0.0) r0 = tot;
          if (tot <= 1e-16 * r0 || tot == 0.0) break;
        }
      }
    } else if (op.kind == OP_DOWN) {
      const Lev Lc = F.L[l + 1];
      for (int64_t g = tid; g < 2 * Lc.half; g += nt)
        op_lin_resid_restrict<T>(L, Lc, F.e[l], F.dg[l], F.r[l], F.kh2[l], F.r[l + 1], F.e[l + 1], g);
      __syncthreads();
    } else {
      const Lev Lc = F.L[l + 1];
      for (int64_t g = tid; g < 2 * L.half; g += nt)
        op_prolong_add<T>(L, Lc, F.e[l], F.e[l + 1], (const T*)nullptr, g);
      __syncthreads();
    }
  }
}

}  // namespace mgg
