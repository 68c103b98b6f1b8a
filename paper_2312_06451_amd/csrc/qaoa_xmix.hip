// Mixers built from products of Pauli X (Sec. 2.1, Eq. (2)) and per-qubit multi-angle mixers
// (Sec. 3). A layer is the cost phase, a Walsh-Hadamard transform W (a Hadamard on every
// qubit), the mixer's diagonal e^{-i beta d(y)} and W again, since W e^{-i beta f(Z)} W =
// e^{-i beta f(X)}. Every step is unitary, so no scalar bookkeeping is needed.
//
// W runs as tile passes. For n >= 13 (complex64) or 12 (complex128) the passes hold tiles of
// 2^13 or 2^12 amplitudes in registers (k_wht, next to the other register-tile kernels); below that a workgroup loads the whole
// state into LDS (k_xwht below) and applies the n butterfly rounds there. Diagonals run
// elementwise; the index of the diagonal value comes from the cost table, from the popcount of y (symmetric k-body mixers), from the parities of y
// against up to 10 term masks (general term lists), or, per qubit, as a product of up to four
// 256-entry factor tables over 8-bit slices of y. Gradient sums are taken in the same sweep as
// the undoing of a diagonal, before it is undone: sum_y v(y) Im(conj(lam_y) phi_y), or for
// per-qubit angles the total and the sums over y with bit q set. Partial sums per workgroup in
// FP64, reduced in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qaoa_internal.h"

namespace qaoa {

namespace {

template <typename R> struct XC;
template <> struct XC<float> { using T2 = float2; };
template <> struct XC<double> { using T2 = double2; };

template <typename T2>
__device__ __forceinline__ T2 xmul(const T2 &a, const T2 &b) {
  T2 o;
  o.x = a.x * b.x - a.y * b.y;
  o.y = a.x * b.y + a.y * b.x;
  return o;
}

// ---------------------------------------------------------------- lookup tables

// out[s * len + c] = e^{-i sign theta_s vals[c]}, theta_s = angles[s * stride + off]
template <typename R>
__global__ void k_xlut(const double *__restrict__ vals, int len, const double *__restrict__ angles, int stride,
                       int off, double sign, typename XC<R>::T2 *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
  if (c >= len) return;
  double sn, co;
  sincos(-sign * angles[(size_t)s * stride + off] * vals[c], &sn, &co);
  out[(size_t)s * len + c] = typename XC<R>::T2{(R)co, (R)sn};
}

// Per-qubit factors: out[(s * 4 + h) * 256 + v] = e^{-i sign sum_q beta_q (1 - 2 v_{q - 8h})} over the
// qubits q = 8h .. 8h + 7 below n, beta_q = angles[s * stride + off + q].
template <typename R>
__global__ void k_xlut_q(int n, const double *__restrict__ angles, int stride, int off, double sign,
                         typename XC<R>::T2 *__restrict__ out) {
  const int v = threadIdx.x, h = blockIdx.x, s = blockIdx.y;
  const double *b = angles + (size_t)s * stride + off;
  double th = 0.0;
  for (int i = 0; i < 8; i++) {
    const int q = 8 * h + i;
    if (q < n) th += b[q] * (((v >> i) & 1) ? -1.0 : 1.0);
  }
  double sn, co;
  sincos(-sign * th, &sn, &co);
  out[((size_t)s * 4 + h) * 256 + v] = typename XC<R>::T2{(R)co, (R)sn};
}

// ---------------------------------------------------------------- block sums

// Adds each of the K per-thread values into partials[(o * nsets + s) * nblk + b], o < K.
template <int K>
__device__ __forceinline__ void block_partials(const double *v, double *red, double *partials, int nsets, int s,
                                               int nblk, int b) {
  const int t = threadIdx.x;
#pragma unroll
  for (int o = 0; o < K; o++) {
    double x = v[o];
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d);
    if ((t & 63) == 0) red[(t >> 6) * K + o] = x;
  }
  __syncthreads();
  if (t < K) {
    const double x = (red[t] + red[K + t]) + (red[2 * K + t] + red[3 * K + t]);
    partials[((size_t)t * nsets + s) * nblk + b] = x;
  }
}

// ---------------------------------------------------------------- diagonals

// v <- D v for NV vectors, D from the staged LUT (modes TABLE, POPCOUNT, TERMS) or the per-qubit
// factor tables (mode QUBIT). GS: first add sum_y g(y) Im(conj(lam) phi) into the partials, with
// g(y) = gv[index] - gshift, or (QUBIT) the total and the per-bit sums.
template <typename R, int NV, bool GS, bool QUBIT>
__global__ __launch_bounds__(256) void k_xdiag(typename XC<R>::T2 *__restrict__ phi, typename XC<R>::T2 *__restrict__ lam,
                                               uint64_t N, XDiag d, const typename XC<R>::T2 *__restrict__ luts,
                                               int lut_len, const double *__restrict__ gv, double gshift,
                                               double *__restrict__ partials, int nsets) {
  using T2 = typename XC<R>::T2;
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *lut = (T2 *)smem;
  const int L = QUBIT ? 4 * 256 : lut_len;
  double *lg = (double *)(lut + L);
  double *red = lg + (QUBIT ? 0 : lut_len);
  const int t = threadIdx.x, s = blockIdx.y;
  const T2 *src = luts + (size_t)s * L;
  for (int i = t; i < L; i += 256) lut[i] = src[i];
  if (GS && !QUBIT)
    for (int i = t; i < lut_len; i += 256) lg[i] = gv[i] - gshift;
  __syncthreads();
  T2 *ph = phi + (size_t)s * N;
  T2 *la = NV == 2 ? lam + (size_t)s * N : nullptr;
  constexpr int K = QUBIT ? 33 : 1;
  double acc[GS ? K : 1];
#pragma unroll
  for (int o = 0; o < (GS ? K : 1); o++) acc[o] = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t y = (uint64_t)blockIdx.x * 256 + t; y < N; y += stride) {
    T2 D;
    if constexpr (QUBIT) {
      D = lut[y & 255];
      if (N > 256) D = xmul(D, lut[256 + ((y >> 8) & 255)]);
      if (N > 65536) D = xmul(D, lut[512 + ((y >> 16) & 255)]);
      if (N > 16777216) D = xmul(D, lut[768 + ((y >> 24) & 255)]);
    }
    const uint32_t idx = QUBIT ? 0u : xdiag_index(d, y);
    if constexpr (!QUBIT) D = lut[idx];
    T2 a = ph[y];
    if constexpr (NV == 2) {
      T2 l = la[y];
      if constexpr (GS) {
        const double r = (double)l.x * a.y - (double)l.y * a.x;
        if constexpr (QUBIT) {
          acc[0] += r;
#pragma unroll
          for (int q = 0; q < 32; q++)
            if ((y >> q) & 1) acc[1 + q] += r;
        } else {
          acc[0] += r * lg[idx];
        }
      }
      la[y] = xmul(l, D);
    }
    ph[y] = xmul(a, D);
  }
  if constexpr (GS) {
    __syncthreads();
    block_partials<K>(acc, red, partials, nsets, s, gridDim.x, blockIdx.x);
  }
}

// End of the forward sweep: E = sum |phi|^2 C, Nrm = sum |phi|^2 and (LAM) lam = (C - c0) phi.
template <typename R, bool LAM>
__global__ __launch_bounds__(256) void k_xend(const typename XC<R>::T2 *__restrict__ phi,
                                              typename XC<R>::T2 *__restrict__ lam, uint64_t N, XDiag d,
                                              const double *__restrict__ vals, int lut_len, double c0,
                                              double *__restrict__ partials, int nsets) {
  using T2 = typename XC<R>::T2;
  extern __shared__ __align__(16) unsigned char smem[];
  double *lv = (double *)smem;
  double *red = lv + lut_len;
  const int t = threadIdx.x, s = blockIdx.y;
  for (int i = t; i < lut_len; i += 256) lv[i] = vals[i];
  __syncthreads();
  const T2 *ph = phi + (size_t)s * N;
  T2 *la = LAM ? lam + (size_t)s * N : nullptr;
  double acc[2] = {0.0, 0.0};
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t y = (uint64_t)blockIdx.x * 256 + t; y < N; y += stride) {
    const T2 a = ph[y];
    const double c = lv[xdiag_index(d, y)];
    const double pr = (double)a.x * a.x + (double)a.y * a.y;
    acc[0] += pr * c;
    acc[1] += pr;
    if constexpr (LAM) {
      const R k = (R)(c - c0);
      la[y] = T2{k * a.x, k * a.y};
    }
  }
  __syncthreads();
  block_partials<2>(acc, red, partials, nsets, s, gridDim.x, blockIdx.x);
}

template <typename R>
__global__ void k_xfill(typename XC<R>::T2 *__restrict__ v, uint64_t total, R u0) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    v[i] = typename XC<R>::T2{u0, (R)0};
}

// out[s * ostride + ooff + o] = sum over b < nblk of partials[(o * nsets + s) * nblk + b], fixed order.
__global__ __launch_bounds__(256) void k_xfinal(const double *__restrict__ partials, int nblk, int nsets,
                                                double *__restrict__ out, int ostride, int ooff) {
  __shared__ double red[256];
  const int o = blockIdx.x, s = blockIdx.y, t = threadIdx.x;
  const double *src = partials + ((size_t)o * nsets + s) * nblk;
  double x = 0.0;
  for (int b = t; b < nblk; b += 256) x += src[b];
  red[t] = x;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) out[(size_t)s * ostride + ooff + o] = red[0];
}

// ---------------------------------------------------------------- Walsh-Hadamard pass

// Hadamard on index bits [b0, b0 + B) of NV vectors; tile = 2^(B + c) amplitudes with the c
// contiguous low bits (c <= b0; c = 0 when b0 = 0).
template <typename R, int NV>
__global__ __launch_bounds__(256) void k_xwht(typename XC<R>::T2 *__restrict__ phi, typename XC<R>::T2 *__restrict__ lam,
                                              uint64_t N, int b0, int B, int c) {
  using T2 = typename XC<R>::T2;
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *tile = (T2 *)smem;
  const int t = threadIdx.x;
  const uint32_t TS = 1u << (B + c);
  const uint64_t r = blockIdx.x;
  const int lo_w = b0 - c;  // rest bits between the row bits and the transformed bits
  const uint64_t base = ((r & ((1ull << lo_w) - 1)) << c) | ((r >> lo_w) << (b0 + B));
  const uint32_t cmask = (1u << c) - 1;
  const R h = (R)0.70710678118654752440;
  for (int v = 0; v < NV; v++) {
    T2 *vec = (v == 0 ? phi : lam) + (size_t)blockIdx.y * N;
    if (v) __syncthreads();
    for (uint32_t l = t; l < TS; l += 256) tile[l] = vec[base | (l & cmask) | ((uint64_t)(l >> c) << b0)];
    for (int g = 0; g < B; g++) {
      __syncthreads();
      const int sh = c + g;
      for (uint32_t i = t; i < TS / 2; i += 256) {
        const uint32_t i0 = ((i >> sh) << (sh + 1)) | (i & ((1u << sh) - 1)), i1 = i0 | (1u << sh);
        const T2 a = tile[i0], b = tile[i1];
        tile[i0] = T2{(a.x + b.x) * h, (a.y + b.y) * h};
        tile[i1] = T2{(a.x - b.x) * h, (a.y - b.y) * h};
      }
    }
    __syncthreads();
    for (uint32_t l = t; l < TS; l += 256) vec[base | (l & cmask) | ((uint64_t)(l >> c) << b0)] = tile[l];
  }
}

template <typename F>
hipError_t set_lds(F *fn, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

// ---------------------------------------------------------------- launchers

unsigned xdiag_blocks(uint64_t N) {
  uint64_t b = (N + 255) / 256;
  return (unsigned)(b > 2048 ? 2048 : b);
}

hipError_t launch_xlut(int precision, const double *vals, int len, const double *angles, int stride, int off,
                       double sign, int nsets, void *out, hipStream_t s) {
  dim3 g((len + 255) / 256, nsets);
  if (precision == 0) k_xlut<float><<<g, 256, 0, s>>>(vals, len, angles, stride, off, sign, (float2 *)out);
  else k_xlut<double><<<g, 256, 0, s>>>(vals, len, angles, stride, off, sign, (double2 *)out);
  return hipGetLastError();
}

hipError_t launch_xlut_q(int precision, int n, const double *angles, int stride, int off, double sign, int nsets,
                         void *out, hipStream_t s) {
  dim3 g(4, nsets);
  if (precision == 0) k_xlut_q<float><<<g, 256, 0, s>>>(n, angles, stride, off, sign, (float2 *)out);
  else k_xlut_q<double><<<g, 256, 0, s>>>(n, angles, stride, off, sign, (double2 *)out);
  return hipGetLastError();
}

template <typename R, int NV, bool GS, bool Q>
static hipError_t xdiag_t(void *phi, void *lam, uint64_t N, const XDiag &d, const void *luts, int lut_len,
                          const double *gv, double gshift, double *partials, int nsets, hipStream_t s) {
  using T2 = typename XC<R>::T2;
  const int L = Q ? 1024 : lut_len;
  const size_t lds = (size_t)L * sizeof(T2) + (Q ? 0 : (size_t)lut_len * 8) + 4 * 33 * 8;
  hipError_t e = set_lds(k_xdiag<R, NV, GS, Q>, lds);
  if (e != hipSuccess) return e;
  dim3 g(xdiag_blocks(N), nsets);
  k_xdiag<R, NV, GS, Q><<<g, 256, lds, s>>>((T2 *)phi, (T2 *)lam, N, d, (const T2 *)luts, lut_len, gv, gshift,
                                            partials, nsets);
  return hipGetLastError();
}

hipError_t launch_xdiag(int precision, int nv, int gsums, void *phi, void *lam, uint64_t N, const XDiag &d,
                        const void *luts, int lut_len, const double *gv, double gshift, double *partials,
                        int nsets, hipStream_t s) {
  const bool q = d.mode == XD_QUBIT;
#define XD_CASE(R, NV, GS, Q) \
  if (nv == NV && (bool)gsums == GS && q == Q) \
    return xdiag_t<R, NV, GS, Q>(phi, lam, N, d, luts, lut_len, gv, gshift, partials, nsets, s);
  if (precision == 0) {
    XD_CASE(float, 1, false, false) XD_CASE(float, 1, false, true) XD_CASE(float, 2, false, false)
    XD_CASE(float, 2, false, true) XD_CASE(float, 2, true, false) XD_CASE(float, 2, true, true)
  } else {
    XD_CASE(double, 1, false, false) XD_CASE(double, 1, false, true) XD_CASE(double, 2, false, false)
    XD_CASE(double, 2, false, true) XD_CASE(double, 2, true, false) XD_CASE(double, 2, true, true)
  }
#undef XD_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_xend(int precision, const void *phi, void *lam, uint64_t N, const XDiag &d, const double *vals,
                       int lut_len, double c0, double *partials, int nsets, hipStream_t s) {
  const size_t lds = (size_t)lut_len * 8 + 4 * 2 * 8;
  dim3 g(xdiag_blocks(N), nsets);
  if (precision == 0) {
    if (lam) k_xend<float, true><<<g, 256, lds, s>>>((const float2 *)phi, (float2 *)lam, N, d, vals, lut_len, c0, partials, nsets);
    else k_xend<float, false><<<g, 256, lds, s>>>((const float2 *)phi, nullptr, N, d, vals, lut_len, c0, partials, nsets);
  } else {
    if (lam) k_xend<double, true><<<g, 256, lds, s>>>((const double2 *)phi, (double2 *)lam, N, d, vals, lut_len, c0, partials, nsets);
    else k_xend<double, false><<<g, 256, lds, s>>>((const double2 *)phi, nullptr, N, d, vals, lut_len, c0, partials, nsets);
  }
  return hipGetLastError();
}

hipError_t launch_xfill(int precision, void *v, uint64_t total, double u0, hipStream_t s) {
  uint64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (precision == 0) k_xfill<float><<<(unsigned)g, 256, 0, s>>>((float2 *)v, total, (float)u0);
  else k_xfill<double><<<(unsigned)g, 256, 0, s>>>((double2 *)v, total, u0);
  return hipGetLastError();
}

hipError_t launch_xfinal(const double *partials, int nblk, int nsums, int nsets, double *out, int ostride, int ooff,
                         hipStream_t s) {
  k_xfinal<<<dim3(nsums, nsets), 256, 0, s>>>(partials, nblk, nsets, out, ostride, ooff);
  return hipGetLastError();
}

hipError_t launch_xwht(int precision, int nv, void *phi, void *lam, int n, int nsets, hipStream_t s) {
  if (n >= wht_min_bits(precision)) return launch_wht_tiles(precision, nv, phi, lam, n, nsets, s);
  const uint64_t N = 1ull << n;
  int b = 0;
  while (b < n) {
    const int c = b == 0 ? 0 : (b < 5 ? b : 5);
    const int B = b == 0 ? (n < 12 ? n : 12) : ((n - b) < 12 - c ? (n - b) : 12 - c);
    const size_t lds = ((size_t)1 << (B + c)) * (precision == 0 ? 8 : 16);
    dim3 g((unsigned)(1ull << (n - B - c)), nsets);
    hipError_t e;
    if (precision == 0) {
      if (nv == 1) {
        e = set_lds(k_xwht<float, 1>, lds);
        if (e == hipSuccess) k_xwht<float, 1><<<g, 256, lds, s>>>((float2 *)phi, nullptr, N, b, B, c);
      } else {
        e = set_lds(k_xwht<float, 2>, lds);
        if (e == hipSuccess) k_xwht<float, 2><<<g, 256, lds, s>>>((float2 *)phi, (float2 *)lam, N, b, B, c);
      }
    } else {
      if (nv == 1) {
        e = set_lds(k_xwht<double, 1>, lds);
        if (e == hipSuccess) k_xwht<double, 1><<<g, 256, lds, s>>>((double2 *)phi, nullptr, N, b, B, c);
      } else {
        e = set_lds(k_xwht<double, 2>, lds);
        if (e == hipSuccess) k_xwht<double, 2><<<g, 256, lds, s>>>((double2 *)phi, (double2 *)lam, N, b, B, c);
      }
    }
    if (e != hipSuccess) return e;
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    b += B;
  }
  return hipSuccess;
}

hipError_t launch_xwht_pre(int precision, void *phi, int n, int nsets, const XDiag &d, const void *luts, int lut_len,
                           hipStream_t s) {
  if (n >= wht_min_bits(precision)) return launch_wht_tiles(precision, 1, phi, nullptr, n, nsets, s, &d, luts, lut_len);
  hipError_t e = launch_xdiag(precision, 1, 0, phi, nullptr, 1ull << n, d, luts, lut_len, nullptr, 0.0, nullptr,
                              nsets, s);
  if (e != hipSuccess) return e;
  return launch_xwht(precision, 1, phi, nullptr, n, nsets, s);
}

int xwht_passes(int n, int precision) {
  if (n >= wht_min_bits(precision)) return wht_tile_passes(n, precision);
  int b = 0, k = 0;
  while (b < n) {
    const int c = b == 0 ? 0 : (b < 5 ? b : 5);
    b += b == 0 ? (n < 12 ? n : 12) : ((n - b) < 12 - c ? (n - b) : 12 - c);
    k++;
  }
  return k;
}

}  // namespace qaoa
