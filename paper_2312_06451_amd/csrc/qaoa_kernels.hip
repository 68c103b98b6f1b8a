// HIP kernels for gfx950 (MI355X): QAOA statevector evolution with the transverse-field
// mixer (Golden et al., JuliQAOA, SC-W 2023).
//
//  (a) cost table C(x) over the feasible set (Sec. 2.1, pre-computation);
//  (b) phase separator e^{-i gamma C(x)} as a lookup-table multiply (Eq. (1));
//  (c) mixer e^{-i beta sum_q X_q} as one 2x2 rotation per qubit (the factorisation of
//      Eq. (2));
//  (d) <C> = sum_x |psi(x)|^2 C(x) (Sec. 1) and the gradient in (beta, gamma) by a reverse
//      sweep that undoes each layer (Sec. 2.3 gets this gradient by reverse-mode AD).
//
// Rotation form. A qubit rotation e^{-i b X} = cos b I - i sin b X is applied unnormalised as
// G(tau) = I - i tau X (four FMAs per amplitude pair) with tau = tan b, or, when |tan b| > 1,
// as X G(tau) with tau = -cot b. The dropped scalar (cos b, or -i sin b) is tracked by the
// host and folded into the next phase lookup table, so every applied rotation is exactly
// unitary up to that scalar and norm drift does not accumulate. The X of the second form is
// not applied either: the stored vector is the state with a known set of bits flipped
// (after a full round: all bits or none, so at every phase point). Steps that read the cost
// then read C(~x): tables with C(~x) = C(x) (every MaxCut table) are read unchanged, other
// tables through their reversed copy, chosen per angle set; a state export un-flips.
//
// Cost tables hold, per state, the index of its value among at most 1024 distinct values;
// the phase lookup tables and a small value table (staged in LDS) map indices to
// e^{-i gamma c} and to c.
//
// Tile passes. A workgroup of 256 threads holds a tile of 2^T amplitudes in registers
// (2^(T-8) per thread and vector). Tile bits [0,c) are contiguous address bits; the other
// T-c tile bits sit on a contiguous range of higher address bits. Rotations on tile bits that
// live in a thread's registers need no communication; three register assignments (H, M, L)
// cover all tile bits and the tile moves between them through a padded, bank-conflict-free
// LDS buffer. The phase multiply, the <C> reduction, the adjoint initialisation and the
// gradient inner products are fused into the passes.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>
#include <vector>
#include <cstdint>
#include "qaoa_internal.h"
#include "qaoa_tile.h"

namespace qaoa {

// ============================================================== (a) cost table

// C(x) = sum_e w_e [bit u_e of x != bit v_e of x], one x per thread (grid-stride, 64-bit x).
template <typename TT>
__global__ void k_cost_table_full(int n, int m, const int32_t *__restrict__ u,
                                  const int32_t *__restrict__ v, const int32_t *__restrict__ w,
                                  TT *__restrict__ table) {
  __shared__ int32_t su[512], sv[512], sw[512];
  for (int e = threadIdx.x; e < m; e += blockDim.x) {
    su[e] = u[e];
    sv[e] = v[e];
    sw[e] = w ? w[e] : 1;
  }
  __syncthreads();
  const uint64_t N = 1ull << n;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) {
    uint32_t c = 0;
    for (int e = 0; e < m; e++) c += (uint32_t)sw[e] * (uint32_t)(((x >> su[e]) ^ (x >> sv[e])) & 1u);
    table[x] = (TT)c;
  }
}

// Weight-k feasible set: the r-th weight-k integer in increasing order, found by the
// combinatorial number system (largest a with C(a, i) <= r, for i = k..1).
template <typename TT>
__global__ void k_cost_table_hw(int n, int k, int m, const int32_t *__restrict__ u,
                                const int32_t *__restrict__ v, const int32_t *__restrict__ w,
                                const int64_t *__restrict__ binom, uint64_t N,
                                TT *__restrict__ table) {
  __shared__ int32_t su[512], sv[512], sw[512];
  for (int e = threadIdx.x; e < m; e += blockDim.x) {
    su[e] = u[e];
    sv[e] = v[e];
    sw[e] = w ? w[e] : 1;
  }
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += stride) {
    uint64_t rem = r, x = 0;
    int a = n - 1;
    for (int i = k; i >= 1; i--) {
      while (a >= i && (uint64_t)binom[a * 33 + i] > rem) a--;
      x |= 1ull << a;
      rem -= (uint64_t)binom[a * 33 + i];
      a--;
    }
    uint32_t c = 0;
    for (int e = 0; e < m; e++) c += (uint32_t)sw[e] * (uint32_t)(((x >> su[e]) ^ (x >> sv[e])) & 1u);
    table[r] = (TT)c;
  }
}

template <typename TT>
__global__ void k_table_max(const TT *__restrict__ t, uint64_t N, unsigned *__restrict__ out) {
  unsigned mx = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    mx = max(mx, (unsigned)t[i]);
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (unsigned)__shfl_xor((int)mx, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, mx);
}

// dst[r * 2^T + e] = src[address(r, e)] for the tile geometry (T, c, h0).
template <typename TT>
__global__ void k_table_relayout(const TT *__restrict__ src, TT *__restrict__ dst, int n, int T,
                                 int c, int h0) {
  const uint64_t N = 1ull << n;
  const int lo_w = h0 - c;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    uint64_t r = i >> T, e = i & ((1ull << T) - 1);
    uint64_t x = ((r & ((1ull << lo_w) - 1)) << c) | ((r >> lo_w) << (h0 + T - c)) |
                 (e & ((1ull << c) - 1)) | ((e >> c) << h0);
    dst[i] = src[x];
  }
}

template <typename TT>
__global__ void k_table_widen(const TT *__restrict__ src, int64_t *__restrict__ dst, uint64_t N) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    dst[i] = (int64_t)src[i];
}

// dst[i] = src[N - 1 - i]: the table of C(~x) over the full space, in any tile-major layout
// (complementing x complements both the tile index and the element index).
template <typename TT>
__global__ void k_table_reverse(const TT *__restrict__ src, TT *__restrict__ dst, uint64_t N) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    dst[i] = src[N - 1 - i];
}

template <typename TT>
__global__ void k_table_values(const TT *__restrict__ src, const double *__restrict__ vals,
                               double *__restrict__ dst, uint64_t N) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    dst[i] = vals[src[i]];
}

// ============================================================== phase lookup tables

// luts[j][c] = s_j * exp(sign_j * i * gamma_j * vals[c]): FP64 argument and sincos, one
// rounding.
template <typename R>
__global__ void k_luts(const LutJob *__restrict__ jobs, int lut_len, const double *__restrict__ vals,
                       typename Cplx<R>::T2 *__restrict__ luts) {
  const LutJob J = jobs[blockIdx.x];
  for (int c = threadIdx.x; c < lut_len; c += blockDim.x) {
    double s, co;
    sincos(J.sign * J.gamma * vals[c], &s, &co);
    typename Cplx<R>::T2 o;
    o.x = (R)(J.sre * co - J.sim * s);
    o.y = (R)(J.sre * s + J.sim * co);
    luts[(size_t)blockIdx.x * lut_len + c] = o;
  }
}

// ============================================================== reductions

// out[q][o] = sum over contributions c < cnt[o] and tiles b < nwg of
// partials[((o * maxc + c) * nsets + q) * nwg + b], in a fixed order (deterministic): 1024
// threads, each with four interleaved running sums (four loads in flight per thread), then a
// fixed tree over the threads.
constexpr int FIN_THREADS = 1024;
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const double *__restrict__ partials,
                                                          const int *__restrict__ cnt, int maxc,
                                                          int nsets, int64_t nwg, int nout,
                                                          double *__restrict__ out) {
  __shared__ double red[FIN_THREADS];
  const int o = blockIdx.x, q = blockIdx.y, t = threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int c = 0; c < cnt[o]; c++) {
    const double *src = partials + (((int64_t)o * maxc + c) * nsets + q) * nwg;
    int64_t k = t;
    for (; k + 3 * FIN_THREADS < nwg; k += 4 * FIN_THREADS) {
      s0 += src[k];
      s1 += src[k + FIN_THREADS];
      s2 += src[k + 2 * FIN_THREADS];
      s3 += src[k + 3 * FIN_THREADS];
    }
    for (; k < nwg; k += FIN_THREADS) s0 += src[k];
  }
  red[t] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int h = FIN_THREADS / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) out[(int64_t)q * nout + o] = red[0];
}

// dst[i] = (re + i im) * src[i ^ flip]
template <typename R>
__global__ void k_scale_copy(const typename Cplx<R>::T2 *__restrict__ src,
                             typename Cplx<R>::T2 *__restrict__ dst, uint64_t N, double re,
                             double im, uint64_t flip) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    typename Cplx<R>::T2 v = src[i ^ flip], o;
    o.x = (R)((double)v.x * re - (double)v.y * im);
    o.y = (R)((double)v.x * im + (double)v.y * re);
    dst[i] = o;
  }
}

// ============================================================== whole-state kernel

// Block-wide sum of one double per thread (256 threads, fixed order).
__device__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

struct DC {
  double re, im;
};
__device__ __forceinline__ DC dmul(DC a, DC b) { return DC{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Rotation parameters of e^{-i beta X} in the unnormalised form (see file header): tau and
// the dropped scalar f of the forward rotation; the inverse rotation uses -tau and finv.
template <typename R>
__device__ void rot_params(double beta, R &tau, DC &f, DC &finv, bool &flip) {
  double sb, cb;
  sincos(beta, &sb, &cb);
  flip = !(fabs(sb) <= fabs(cb));
  if (!flip) {
    tau = (R)(sb / cb);
    double t = (double)tau, nrm = 1.0 / sqrt(1.0 + t * t);
    f = DC{nrm * (cb < 0 ? -1.0 : 1.0), 0.0};
    finv = f;
  } else {
    tau = (R)(-cb / sb);
    double t = (double)tau, s = (sb < 0 ? -1.0 : 1.0) / sqrt(1.0 + t * t);
    f = DC{0.0, -s};
    finv = DC{0.0, s};
  }
}

// One workgroup per (problem, angle set): both vectors and the table in LDS. Forward
// rounds of Eq. (1), <C>, and (grad != 0) the reverse sweep for the gradient.
template <typename R>
__global__ __launch_bounds__(256) void k_small(const SmallItem *__restrict__ items,
                                               const double *__restrict__ angles, int p, int grad,
                                               int max_n, int max_tb, int max_lut,
                                               double *__restrict__ out, int stage) {
  using T2 = typename Cplx<R>::T2;
  extern __shared__ __align__(16) unsigned char smem[];
  const SmallItem it = items[blockIdx.x];
  const int n = it.n;
  const uint32_t N = 1u << n;
  T2 *phi = (T2 *)smem;
  T2 *lam = phi + (1u << max_n);
  T2 *lut = lam + (1u << max_n);
  unsigned char *tab = (unsigned char *)(lut + max_lut);
  double *red = (double *)(tab + ((((size_t)max_tb << max_n) + 15) & ~(size_t)15));
  const int tid = threadIdx.x;
  const double *ang = angles + (size_t)it.angle_set * 2 * p;
  if (stage) {
    // the angle set is read once into LDS (the caller may pass it in host memory)
    double *sang = red + 8;
    for (int i = tid; i < 2 * p; i += 256) sang[i] = ang[i];
    __syncthreads();
    ang = sang;
  }

  for (uint32_t x = tid; x < N; x += 256) {
    if (it.tbytes == 1) ((unsigned char *)tab)[x] = ((const unsigned char *)it.table)[x];
    else ((uint16_t *)tab)[x] = ((const uint16_t *)it.table)[x];
  }
  // the stored vector is the state with the bits of F flipped (tangent form, see the file
  // header): its amplitude at x belongs to basis state x ^ F. F is all bits or none at every
  // phase point; a table with C(~x) = C(x) may ignore it.
  uint32_t F = 0;
  const uint32_t FALL = it.sym ? 0u : N - 1;
  auto cval = [&](uint32_t x) -> uint32_t {
    x ^= F;
    return it.tbytes == 1 ? (uint32_t)tab[x] : (uint32_t)((const uint16_t *)tab)[x];
  };
  auto cost = [&](uint32_t x) -> double { return it.vals[cval(x)]; };
  const R u0 = (R)(1.0 / sqrt((double)N));
  for (uint32_t x = tid; x < N; x += 256) phi[x] = T2{u0, (R)0};
  DC sig{1.0, 0.0};
  auto build_lut = [&](double gamma, double sign) {
    __syncthreads();
    for (int c = tid; c < it.lut_len; c += 256) {
      double s, co;
      sincos(sign * gamma * it.vals[c], &s, &co);
      lut[c] = T2{(R)(sig.re * co - sig.im * s), (R)(sig.re * s + sig.im * co)};
    }
    __syncthreads();
  };
  auto rotate_all = [&](T2 *v, R tau) {
    for (int qb = 0; qb < n; qb++) {
      const uint32_t bit = 1u << qb;
      __syncthreads();
      for (uint32_t i = tid; i < N / 2; i += 256) {
        uint32_t x0 = ((i >> qb) << (qb + 1)) | (i & (bit - 1));
        T2 va = v[x0], vb = v[x0 | bit];
        bfly(va, vb, tau);
        v[x0] = va;
        v[x0 | bit] = vb;
      }
    }
    __syncthreads();
  };

  for (int k = 0; k < p; k++) {
    build_lut(ang[p + k], -1.0);
    for (uint32_t x = tid; x < N; x += 256) {
      T2 L = lut[cval(x)], v = phi[x];
      phi[x] = T2{fmaR(v.x, L.x, -v.y * L.y), fmaR(v.x, L.y, v.y * L.x)};
    }
    sig = DC{1.0, 0.0};
    R tau; DC f, finv;
    bool fl;
    rot_params<R>(ang[k], tau, f, finv, fl);
    rotate_all(phi, tau);
    if (fl) F ^= FALL;
    for (int qb = 0; qb < n; qb++) sig = dmul(sig, f);
  }
  double e = 0.0, nr = 0.0;
  for (uint32_t x = tid; x < N; x += 256) {
    double pr = (double)phi[x].x * phi[x].x + (double)phi[x].y * phi[x].y;
    e += pr * cost(x);
    nr += pr;
  }
  e = block_sum(e, red);
  nr = block_sum(nr, red);
  const double ntrue = (sig.re * sig.re + sig.im * sig.im) * nr;
  double *o = out + (size_t)it.out_index * (1 + 2 * p);
  if (tid == 0) o[0] = e / nr;
  if (!grad) return;

  for (uint32_t x = tid; x < N; x += 256) {
    R kf = (R)(cost(x) - it.c0);
    lam[x] = T2{kf * phi[x].x, kf * phi[x].y};
  }
  __syncthreads();
  for (int k = p - 1; k >= 0; k--) {
    // d/dbeta_k: 2 Im <lam| sum_q X_q |phi>, one term per amplitude pair and qubit
    double gb = 0.0;
    for (int qb = 0; qb < n; qb++) {
      const uint32_t bit = 1u << qb;
      R s = 0;
      for (uint32_t i = tid; i < N / 2; i += 256) {
        uint32_t x0 = ((i >> qb) << (qb + 1)) | (i & (bit - 1));
        s = xpair(phi[x0], phi[x0 | bit], lam[x0], lam[x0 | bit], s);
      }
      gb += (double)s;
    }
    gb = block_sum(gb, red);
    const double wgt = sig.re * sig.re + sig.im * sig.im;
    if (tid == 0) o[1 + k] = 2.0 * wgt * gb / ntrue;
    R tau; DC f, finv;
    bool fl;
    rot_params<R>(ang[k], tau, f, finv, fl);
    rotate_all(phi, -tau);
    rotate_all(lam, -tau);
    if (fl) F ^= FALL;
    for (int qb = 0; qb < n; qb++) sig = dmul(sig, finv);
    // d/dgamma_k: 2 Im <lam| C |phi> = 2 Im <lam| C - c0 |phi> (<lam|phi> is real)
    double gg = 0.0;
    for (uint32_t x = tid; x < N; x += 256) {
      T2 l = lam[x], v = phi[x];
      gg += (double)(fmaR(l.x, v.y, -l.y * v.x)) * (cost(x) - it.c0);
    }
    gg = block_sum(gg, red);
    const double wg2 = sig.re * sig.re + sig.im * sig.im;
    if (tid == 0) o[1 + p + k] = 2.0 * wg2 * gg / ntrue;
    if (k > 0) {
      build_lut(ang[p + k], 1.0);
      for (uint32_t x = tid; x < N; x += 256) {
        T2 L = lut[cval(x)], v = phi[x], l = lam[x];
        phi[x] = T2{fmaR(v.x, L.x, -v.y * L.y), fmaR(v.x, L.y, v.y * L.x)};
        lam[x] = T2{fmaR(l.x, L.x, -l.y * L.y), fmaR(l.x, L.y, l.y * L.x)};
      }
      sig = DC{1.0, 0.0};
      __syncthreads();
    }
  }
}

// ============================================================== whole state in registers

// The same evaluation as k_small for a state of exactly 2^T amplitudes (T = 12, 13), held in
// registers as one tile (TileCfg<T>: 256 threads, 2^(T-8) amplitudes each): a layer is the
// phase multiply in the current register assignment and three register stages joined by two
// LDS exchanges, instead of one LDS pass per qubit. Layers alternate the stage order (H, M, L
// then L, M, H) so the next layer starts in the assignment the last one ended in; the reverse
// sweep undoes each layer in the opposite order, taking the X-pair terms of each group of
// bits before rotating it (weighted by the rotations of the layer done so far, as in the tile
// passes). Scalars, flips and the FP64 sums as in k_small.

// cost-table index of tile element e (the stored vector is flipped by F)
template <typename TT>
__device__ __forceinline__ uint32_t widx(const unsigned char *tab, uint32_t e, uint32_t F) {
  return (uint32_t)((const TT *)tab)[e ^ F];
}

template <typename R, int T, typename TT, int A, int NV>
__device__ __forceinline__ void w_phase(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                        const unsigned char *tab, const typename Cplx<R>::T2 *lut,
                                        uint32_t F, uint32_t t) {
  using T2 = typename Cplx<R>::T2;
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) {
    const T2 L = lut[widx<TT>(tab, elem<A, T>(t, j), F)];
    phi[j] = cmul<T2, R>(phi[j], L);
    if constexpr (NV == 2) lam[j] = cmul<T2, R>(lam[j], L);
  }
}

// <C> and norm partial sums, then lam = (C - c0) phi
template <typename R, int T, typename TT, int A>
__device__ __forceinline__ void w_end(const typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                      const unsigned char *tab, const double *dval, double c0, uint32_t F,
                                      uint32_t t, double &e, double &nr) {
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) {
    const double c = dval[widx<TT>(tab, elem<A, T>(t, j), F)];
    const double pr = (double)phi[j].x * phi[j].x + (double)phi[j].y * phi[j].y;
    e += pr * c;
    nr += pr;
    const R kf = (R)(c - c0);
    lam[j].x = kf * phi[j].x;
    lam[j].y = kf * phi[j].y;
  }
}

// sum of Im(conj(lam) phi) (C - c0)
template <typename R, int T, typename TT, int A>
__device__ __forceinline__ double w_ggamma(const typename Cplx<R>::T2 *phi, const typename Cplx<R>::T2 *lam,
                                           const unsigned char *tab, const double *dval, double c0, uint32_t F,
                                           uint32_t t) {
  double g = 0.0;
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) {
    const double c = dval[widx<TT>(tab, elem<A, T>(t, j), F)] - c0;
    g += (double)fmaR(lam[j].x, phi[j].y, -lam[j].y * phi[j].x) * c;
  }
  return g;
}

// Forward mixer of one layer: stages A0, M, A2 (A0 = H, A2 = L when DOWN).
template <typename R, int T, bool DOWN>
__device__ __forceinline__ void w_fwd_mixer(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lds, uint32_t t,
                                            R tau) {
  constexpr int A0 = DOWN ? AH : AL, A2 = DOWN ? AL : AH;
  constexpr uint32_t all = (1u << T) - 1;
  double w = 1.0, acc = 0.0;
  stage<R, T, 1, A0, false, false>(phi, phi, all, tau, w, acc);
  xchg1<R, T, A0, AM>(lds, phi, t);
  stage<R, T, 1, AM, false, false>(phi, phi, all, tau, w, acc);
  xchg1<R, T, AM, A2>(lds, phi, t);
  stage<R, T, 1, A2, false, false>(phi, phi, all, tau, w, acc);
}

// Reverse of a layer whose forward order was DOWN: undo stages A2, M, A0 on both vectors,
// X-pair terms first in each; returns the thread's weighted X-pair sum.
template <typename R, int T, bool DOWN>
__device__ __forceinline__ double w_rev_mixer(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                              typename Cplx<R>::T2 *lds, uint32_t t, R tau) {
  constexpr int A0 = DOWN ? AH : AL, A2 = DOWN ? AL : AH;
  constexpr uint32_t all = (1u << T) - 1;
  double w = 1.0, acc = 0.0;
  stage<R, T, 2, A2, true, true>(phi, lam, all, -tau, w, acc);
  xchg<R, T, 2, A2, AM>(lds, phi, lam, t);
  stage<R, T, 2, AM, true, true>(phi, lam, all, -tau, w, acc);
  xchg<R, T, 2, AM, A0>(lds, phi, lam, t);
  stage<R, T, 2, A0, true, true>(phi, lam, all, -tau, w, acc);
  return acc;
}

template <typename R, int T, typename TT>
__global__ __launch_bounds__(256) void k_whole(const SmallItem *__restrict__ items, const double *__restrict__ angles,
                                               int p, int grad, int max_lut, int pre, double *__restrict__ out,
                                               int stage) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  constexpr int RN = G::RN;
  constexpr uint32_t N = 1u << T;
  constexpr uint32_t kSlots = N + (N >> Pad<R>::PS);
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *lds = (T2 *)smem;
  T2 *lut = lds + kSlots;
  double *dval = (double *)(lut + max_lut);
  unsigned char *tab = (unsigned char *)(dval + max_lut);
  double *red = (double *)(tab + ((N * sizeof(TT) + 15) & ~15u));
  // pre != 0: every layer's phase table computed once (forward tables, then reverse ones),
  // per-layer scalars, and the per-wave partial gradient sums, reduced after the sweep
  T2 *plut = (T2 *)(red + 4);
  double *scal = (double *)(plut + (size_t)(pre ? 2 * p * max_lut : 0));  // 6 per layer
  double *gsum = scal + (pre ? 6 * p : 0);                                // 8 per layer
  const SmallItem it = items[blockIdx.x];
  const uint32_t t = threadIdx.x;
  const double *ang = angles + (size_t)it.angle_set * 2 * p;
  if (stage) {
    // the angle set is read once into LDS (the caller may pass it in host memory)
    double *sang = gsum + (pre ? 8 * p : 0);
    for (int i = t; i < 2 * p; i += 256) sang[i] = ang[i];
    __syncthreads();
    ang = sang;
  }

  for (uint32_t i = t; i < N * sizeof(TT) / 4; i += 256) ((uint32_t *)tab)[i] = ((const uint32_t *)it.table)[i];
  for (int c = t; c < it.lut_len; c += 256) dval[c] = it.vals[c];
  uint32_t F = 0;
  const uint32_t FALL = it.sym ? 0u : N - 1;
  DC sig{1.0, 0.0};
  auto lut_entry = [&](const DC &sc, double gamma, double sign, int c) -> T2 {
    double sn, co;
    sincos(sign * gamma * dval[c], &sn, &co);
    return T2{(R)(sc.re * co - sc.im * sn), (R)(sc.re * sn + sc.im * co)};
  };
  auto build_lut = [&](double gamma, double sign) {
    __syncthreads();
    for (int c = t; c < it.lut_len; c += 256) lut[c] = lut_entry(sig, gamma, sign, c);
    __syncthreads();
  };
  if (pre) {
    __syncthreads();  // dval staged
    // scalars of layer k, in the order the sweeps accumulate them: forward table scale
    // (f_{k-1}^T, 1 for k = 0), reverse table scale and weights before and after undoing
    // layer k (the last layer starts from the forward's final scalar)
    for (int k = t; k < p; k += 256) {
      R tau;
      DC f, finv, sf{1.0, 0.0}, before{1.0, 0.0};
      bool fl;
      if (k > 0) {
        rot_params<R>(ang[k - 1], tau, f, finv, fl);
        for (int qb = 0; qb < T; qb++) sf = dmul(sf, f);
      }
      rot_params<R>(ang[k], tau, f, finv, fl);
      if (k == p - 1)
        for (int qb = 0; qb < T; qb++) before = dmul(before, f);
      DC after = before;
      for (int qb = 0; qb < T; qb++) after = dmul(after, finv);
      double *sk = scal + 6 * k;
      sk[0] = sf.re;
      sk[1] = sf.im;
      sk[2] = after.re;
      sk[3] = after.im;
      sk[4] = before.re * before.re + before.im * before.im;
      sk[5] = after.re * after.re + after.im * after.im;
    }
    __syncthreads();
    for (int i = t; i < 2 * p * it.lut_len; i += 256) {
      const int kk = i / it.lut_len, c = i - kk * it.lut_len;
      const bool rev = kk >= p;
      const int k = rev ? kk - p : kk;
      const double *sk = scal + 6 * k;
      const DC sc = rev ? DC{sk[2], sk[3]} : DC{sk[0], sk[1]};
      plut[(size_t)kk * max_lut + c] = lut_entry(sc, ang[p + k], rev ? 1.0 : -1.0, c);
    }
    __syncthreads();
  }

  T2 phi[RN], lam[RN];
  const R u0 = (R)(1.0 / sqrt((double)N));
#pragma unroll
  for (int j = 0; j < RN; j++) phi[j] = T2{u0, (R)0};

  // ---- forward: layer k starts in H when k is even (H, M, L) and in L when odd (L, M, H)
  auto fwd_layer = [&](int k, auto down) {
    constexpr bool D = decltype(down)::value;
    const T2 *lk = lut;
    if (pre) lk = plut + (size_t)k * max_lut;
    else build_lut(ang[p + k], -1.0);
    w_phase<R, T, TT, D ? AH : AL, 1>(phi, lam, tab, lk, F, t);
    sig = DC{1.0, 0.0};
    R tau;
    DC f, finv;
    bool fl;
    rot_params<R>(ang[k], tau, f, finv, fl);
    w_fwd_mixer<R, T, D>(phi, lds, t, tau);
    if (fl) F ^= FALL;
    for (int qb = 0; qb < T; qb++) sig = dmul(sig, f);
  };
  for (int k = 0; k < p; k += 2) {
    fwd_layer(k, std::true_type{});
    if (k + 1 < p) fwd_layer(k + 1, std::false_type{});
  }
  // ends in L after an odd number of layers, in H after an even number
  double e = 0.0, nr = 0.0;
  if (p & 1) w_end<R, T, TT, AL>(phi, lam, tab, dval, it.c0, F, t, e, nr);
  else w_end<R, T, TT, AH>(phi, lam, tab, dval, it.c0, F, t, e, nr);
  e = block_sum(e, red);
  nr = block_sum(nr, red);
  const double ntrue = (sig.re * sig.re + sig.im * sig.im) * nr;
  double *o = out + (size_t)it.out_index * (1 + 2 * p);
  if (t == 0) o[0] = e / nr;
  if (!grad) return;

  // wave sums (the first half of block_sum); with pre they are kept per layer and wave
  auto wave_sum = [&](double v) -> double {
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return v;
  };
  // ---- reverse: layer k was DOWN when k is even; undoing it ends in its first assignment
  auto rev_layer = [&](int k, auto down) {
    constexpr bool D = decltype(down)::value;
    constexpr int A0 = D ? AH : AL;
    const double wgt = sig.re * sig.re + sig.im * sig.im;
    R tau;
    DC f, finv;
    bool fl;
    rot_params<R>(ang[k], tau, f, finv, fl);
    const double xb = w_rev_mixer<R, T, D>(phi, lam, lds, t, tau);
    if (pre) {
      const double v = wave_sum(xb);
      if ((t & 63) == 0) gsum[8 * k + (t >> 6)] = v;
    } else {
      const double gb = block_sum(xb, red);
      if (t == 0) o[1 + k] = 2.0 * wgt * gb / ntrue;
    }
    if (fl) F ^= FALL;
    for (int qb = 0; qb < T; qb++) sig = dmul(sig, finv);
    const double xg = w_ggamma<R, T, TT, A0>(phi, lam, tab, dval, it.c0, F, t);
    if (pre) {
      const double v = wave_sum(xg);
      if ((t & 63) == 0) gsum[8 * k + 4 + (t >> 6)] = v;
    } else {
      const double gg = block_sum(xg, red);
      const double wg2 = sig.re * sig.re + sig.im * sig.im;
      if (t == 0) o[1 + p + k] = 2.0 * wg2 * gg / ntrue;
    }
    if (k > 0) {
      const T2 *lk = lut;
      if (pre) lk = plut + (size_t)(p + k) * max_lut;
      else build_lut(ang[p + k], 1.0);
      w_phase<R, T, TT, A0, 2>(phi, lam, tab, lk, F, t);
      sig = DC{1.0, 0.0};
    }
  };
  for (int k = p - 1; k >= 0; k--) {
    if (k & 1) rev_layer(k, std::false_type{});
    else rev_layer(k, std::true_type{});
  }
  if (pre) {  // the block sums, in block_sum's order, and the layer weights
    __syncthreads();
    for (int k = t; k < p; k += 256) {
      const double *gk = gsum + 8 * k, *sk = scal + 6 * k;
      o[1 + k] = 2.0 * sk[4] * ((gk[0] + gk[1]) + (gk[2] + gk[3])) / ntrue;
      o[1 + p + k] = 2.0 * sk[5] * ((gk[4] + gk[5]) + (gk[6] + gk[7])) / ntrue;
    }
  }
}

// ============================================================== Walsh-Hadamard tile pass

// Hadamards on the tile bits in `mask` held in the registers of assignment A.
template <typename R, int T, int A>
__device__ __forceinline__ void hstage(typename Cplx<R>::T2 *v, uint32_t mask) {
  using G = TileCfg<T>;
  const R h = (R)0.70710678118654752440;
#pragma unroll
  for (int b = 0; b < G::RB; b++) {
    constexpr uint32_t grp = group<A, T>();
    const int tb = regbit<A, T>(b);
    if (((grp & mask) >> tb) & 1u) {  // uniform
#pragma unroll
      for (int j = 0; j < G::RN; j++)
        if (!(j & (1 << b))) {
          const typename Cplx<R>::T2 a = v[j], c = v[j | (1 << b)];
          v[j] = typename Cplx<R>::T2{(a.x + c.x) * h, (a.y + c.y) * h};
          v[j | (1 << b)] = typename Cplx<R>::T2{(a.x - c.x) * h, (a.y - c.y) * h};
        }
    }
  }
}

// One pass of the Walsh-Hadamard transform over tiles of 2^T amplitudes held in registers
// (T = 13 for complex64, 12 for complex128): tile bits [0, c) are contiguous index bits (rows),
// tile bits [c, T) are the transformed index bits [b0, b0 + T - c) (c = 0 and b0 = 0 for the
// first pass). Stages H, then M and L as far as the transformed bits reach, with LDS
// exchanges between them; loads and stores in assignment H (lanes over the low tile bits).
template <typename R, int T, int NV, bool PRE>
__global__ __launch_bounds__(256) void k_wht(typename Cplx<R>::T2 *__restrict__ phi,
                                             typename Cplx<R>::T2 *__restrict__ lam, uint64_t N, int b0, int c,
                                             XDiag pre, const typename Cplx<R>::T2 *__restrict__ luts, int lut_len) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *lds = (T2 *)smem;
  const uint32_t t = threadIdx.x;
  const uint64_t r = blockIdx.x;
  const int B = T - c, lo_w = b0 - c;
  const uint64_t base = ((r & ((1ull << lo_w) - 1)) << c) | ((r >> lo_w) << (b0 + B));
  const uint32_t cmask = (1u << c) - 1;
  const uint32_t mask = ((1u << T) - 1) & ~cmask;
  auto addr = [&](uint32_t e) -> uint64_t { return base | (e & cmask) | ((uint64_t)(e >> c) << b0); };
  T2 v[G::RN];
  for (int k = 0; k < NV; k++) {
    T2 *vec = (k == 0 ? phi : lam) + (size_t)blockIdx.y * N;
#pragma unroll
    for (int j = 0; j < G::RN; j++) v[j] = vec[addr(elem<AH, T>(t, j))];
    if constexpr (PRE) {  // the diagonal that precedes this transform, applied on load
      const T2 *lut = luts + (size_t)blockIdx.y * (pre.mode == XD_QUBIT ? 1024 : lut_len);
#pragma unroll
      for (int j = 0; j < G::RN; j++) v[j] = cmul<T2, R>(v[j], xdiag_value(pre, lut, addr(elem<AH, T>(t, j)), N));
    }
    hstage<R, T, AH>(v, mask);
    if (mask & group<AM, T>()) {
      xchg1<R, T, AH, AM>(lds, v, t);
      hstage<R, T, AM>(v, mask);
      if (mask & group<AL, T>()) {
        xchg1<R, T, AM, AL>(lds, v, t);
        hstage<R, T, AL>(v, mask);
        xchg1<R, T, AL, AH>(lds, v, t);
      } else {
        xchg1<R, T, AM, AH>(lds, v, t);
      }
    }
#pragma unroll
    for (int j = 0; j < G::RN; j++) vec[addr(elem<AH, T>(t, j))] = v[j];
  }
}

static int wht_tile_bits(int precision) { return precision == 0 ? 13 : 12; }

// Transformed bits of pass k of an n-qubit transform: the first pass takes the low T bits, the
// others T - 5 bits at a time (rows of 2^5 amplitudes), the last one the remaining B bits with
// T - B contiguous row bits.
static void wht_schedule(int n, int T, std::vector<std::pair<int, int>> &out) {
  int b = 0;
  while (b < n) {
    const int B = b == 0 ? T : (n - b < T - 5 ? n - b : T - 5);
    out.emplace_back(b, b == 0 ? 0 : T - B);
    b += B;
  }
}

template <typename R, int T>
static hipError_t wht_t(int nv, void *phi, void *lam, int n, int nsets, hipStream_t s, const XDiag *pre,
                        const void *luts, int lut_len) {
  using T2 = typename Cplx<R>::T2;
  const uint64_t N = 1ull << n;
  const size_t lds = (size_t)((1u << T) + ((1u << T) >> Pad<R>::PS)) * sizeof(T2);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k_wht<R, T, 1, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       96 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)k_wht<R, T, 1, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              96 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  std::vector<std::pair<int, int>> sched;
  wht_schedule(n, T, sched);
  const dim3 g((unsigned)(1ull << (n - T)), nsets);
  const XDiag none{};
  // one vector per launch: the single-vector kernel keeps two waves per SIMD
  for (int k = 0; k < nv; k++)
    for (size_t i = 0; i < sched.size(); i++) {
      T2 *v = (T2 *)(k == 0 ? phi : lam);
      if (i == 0 && k == 0 && pre)
        k_wht<R, T, 1, true><<<g, 256, lds, s>>>(v, nullptr, N, sched[i].first, sched[i].second, *pre,
                                                 (const T2 *)luts, lut_len);
      else
        k_wht<R, T, 1, false><<<g, 256, lds, s>>>(v, nullptr, N, sched[i].first, sched[i].second, none, nullptr, 0);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t launch_wht_tiles(int precision, int nv, void *phi, void *lam, int n, int nsets, hipStream_t s,
                            const XDiag *pre, const void *luts, int lut_len) {
  if (n < wht_tile_bits(precision)) return hipErrorInvalidValue;
  return precision == 0 ? wht_t<float, 13>(nv, phi, lam, n, nsets, s, pre, luts, lut_len)
                        : wht_t<double, 12>(nv, phi, lam, n, nsets, s, pre, luts, lut_len);
}

int wht_tile_passes(int n, int precision) {
  std::vector<std::pair<int, int>> sched;
  wht_schedule(n, wht_tile_bits(precision), sched);
  return (int)sched.size();
}

int wht_min_bits(int precision) { return wht_tile_bits(precision); }

// ============================================================== launch wrappers

static unsigned grid_for(uint64_t N, unsigned threads) {
  uint64_t g = (N + threads - 1) / threads;
  if (g > 65536 * 4) g = 65536 * 4;
  if (g < 1) g = 1;
  return (unsigned)g;
}

hipError_t launch_cost_table_full(int n, int m, const int32_t *du, const int32_t *dv,
                                  const int32_t *dw, void *table, int tbytes, hipStream_t s) {
  unsigned g = grid_for(1ull << n, 256);
  if (tbytes == 1) k_cost_table_full<uint8_t><<<g, 256, 0, s>>>(n, m, du, dv, dw, (uint8_t *)table);
  else k_cost_table_full<uint16_t><<<g, 256, 0, s>>>(n, m, du, dv, dw, (uint16_t *)table);
  return hipGetLastError();
}

hipError_t launch_cost_table_hw(int n, int k, int m, const int32_t *du, const int32_t *dv,
                                const int32_t *dw, const int64_t *dbinom, uint64_t N,
                                void *table, int tbytes, hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (tbytes == 1)
    k_cost_table_hw<uint8_t><<<g, 256, 0, s>>>(n, k, m, du, dv, dw, dbinom, N, (uint8_t *)table);
  else
    k_cost_table_hw<uint16_t><<<g, 256, 0, s>>>(n, k, m, du, dv, dw, dbinom, N, (uint16_t *)table);
  return hipGetLastError();
}

hipError_t launch_table_max(const void *table, int tbytes, uint64_t N, unsigned *dmax,
                            hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (g > 4096) g = 4096;
  if (tbytes == 1) k_table_max<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)table, N, dmax);
  else k_table_max<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)table, N, dmax);
  return hipGetLastError();
}

hipError_t launch_table_relayout(const void *src, void *dst, int tbytes, int n, int T, int c,
                                 int h0, hipStream_t s) {
  unsigned g = grid_for(1ull << n, 256);
  if (tbytes == 1)
    k_table_relayout<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)src, (uint8_t *)dst, n, T, c, h0);
  else
    k_table_relayout<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)src, (uint16_t *)dst, n, T, c, h0);
  return hipGetLastError();
}

hipError_t launch_table_widen(const void *src, int tbytes, int64_t *dst, uint64_t N,
                              hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (tbytes == 1) k_table_widen<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)src, dst, N);
  else k_table_widen<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)src, dst, N);
  return hipGetLastError();
}

hipError_t launch_luts(int precision, const LutJob *jobs, int njobs, int lut_len, const double *vals,
                       void *luts, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (precision == 0) k_luts<float><<<njobs, 256, 0, s>>>(jobs, lut_len, vals, (float2 *)luts);
  else k_luts<double><<<njobs, 256, 0, s>>>(jobs, lut_len, vals, (double2 *)luts);
  return hipGetLastError();
}

hipError_t launch_table_reverse(const void *src, void *dst, int tbytes, uint64_t count, hipStream_t s) {
  unsigned g = grid_for(count, 256);
  if (tbytes == 1) k_table_reverse<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)src, (uint8_t *)dst, count);
  else k_table_reverse<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)src, (uint16_t *)dst, count);
  return hipGetLastError();
}

hipError_t launch_table_values(const void *table, int tbytes, const double *vals, double *dst, uint64_t N,
                               hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (tbytes == 1) k_table_values<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)table, vals, dst, N);
  else k_table_values<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)table, vals, dst, N);
  return hipGetLastError();
}

size_t pass_lds_bytes(int precision, int tbytes, int lut_len) {
  return precision == 0 ? lds_for<float, TILE_BITS_F32>(tbytes, lut_len)
                        : lds_for<double, TILE_BITS_F64>(tbytes, lut_len);
}

template <typename R, int T, int KIND, typename TT>
static hipError_t launch_sx(const PassArgs<R> &a, int sx, int shape, hipStream_t s) {
  if (sx == 7) return launch_shape<R, T, KIND, TT, 7, 0>(a, shape, s);
  if (sx == 5) return launch_shape<R, T, KIND, TT, 5, 0>(a, shape, s);
  if (sx == 3) return launch_shape<R, T, KIND, TT, 3, 0>(a, shape, s);
  return launch_shape<R, T, KIND, TT, 1, 0>(a, shape, s);
}

template <typename R, int T, typename TT>
static hipError_t launch_kind(const PassArgs<R> &a, int kind, int sx, int shape, hipStream_t s) {
  if (kind == 1) return launch_sx<R, T, 1, TT>(a, sx, shape, s);
  if (kind == 2) return launch_sx<R, T, 2, TT>(a, sx, shape, s);
  if (kind == 4) return launch_sx<R, T, 4, TT>(a, sx, shape, s);
  return launch_sx<R, T, 3, TT>(a, sx, shape, s);
}

// The swizzled layout's passes (a.swz > 0) live in their own translation units.
hipError_t launch_pass_f32(const PassArgs<float> &a, int kind, int sx, int shape, int tbytes,
                           hipStream_t s) {
  if (a.swz) return launch_pass_swz_f32(a, kind, sx, shape, tbytes, s);
  return tbytes == 1 ? launch_kind<float, TILE_BITS_F32, uint8_t>(a, kind, sx, shape, s)
                     : launch_kind<float, TILE_BITS_F32, uint16_t>(a, kind, sx, shape, s);
}

hipError_t launch_pass_f64(const PassArgs<double> &a, int kind, int sx, int shape, int tbytes,
                           hipStream_t s) {
  if (a.swz) return launch_pass_swz_f64(a, kind, sx, shape, tbytes, s);
  return tbytes == 1 ? launch_kind<double, TILE_BITS_F64, uint8_t>(a, kind, sx, shape, s)
                     : launch_kind<double, TILE_BITS_F64, uint16_t>(a, kind, sx, shape, s);
}

hipError_t launch_finalize(const double *partials, const int *cnt, int maxc, int nsets,
                           int64_t nwg, int nout, double *out, hipStream_t s) {
  if (nout <= 0 || nsets <= 0) return hipSuccess;
  k_finalize<<<dim3(nout, nsets), FIN_THREADS, 0, s>>>(partials, cnt, maxc, nsets, nwg, nout, out);
  return hipGetLastError();
}

hipError_t launch_small(int precision, const SmallItem *items, int n_items, int max_n,
                        int max_tbytes, int max_lut, const double *angles, int p, int grad,
                        double *out, hipStream_t s, int stage) {
  size_t esz = precision == 0 ? 8 : 16;
  size_t lds = (2ull << max_n) * esz + (size_t)max_lut * esz +
               ((((size_t)max_tbytes << max_n) + 15) & ~(size_t)15) + 64;
  // a staged angle set that does not fit is read in place instead
  const size_t angb = (size_t)2 * p * sizeof(double);
  if (stage && lds + angb > 160 * 1024) stage = 0;
  if (stage) lds += angb;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_small<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)k_small<double>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (precision == 0)
    hipLaunchKernelGGL((k_small<float>), dim3(n_items), dim3(256), lds, s, items, angles, p, grad,
                       max_n, max_tbytes, max_lut, out, stage);
  else
    hipLaunchKernelGGL((k_small<double>), dim3(n_items), dim3(256), lds, s, items, angles, p,
                       grad, max_n, max_tbytes, max_lut, out, stage);
  return hipGetLastError();
}

template <typename R, int T, typename TT>
static hipError_t launch_whole_t(const SmallItem *items, int n_items, int max_lut, const double *angles, int p,
                                 int grad, double *out, hipStream_t s, int stage) {
  using T2 = typename Cplx<R>::T2;
  constexpr size_t N = size_t(1) << T;
  const size_t base = (N + (N >> Pad<R>::PS)) * sizeof(T2) + (size_t)max_lut * (sizeof(T2) + sizeof(double)) +
                      ((N * sizeof(TT) + 15) & ~size_t(15)) + 4 * sizeof(double);
  // precomputed phase tables and deferred sums when they fit without lowering occupancy:
  // complex64 at n = 12 keeps two workgroups per CU below 80 KB
  const size_t with_pre = base + (size_t)2 * p * max_lut * sizeof(T2) + (size_t)14 * p * sizeof(double);
  const size_t cap = (sizeof(R) == 4 && T == 12) ? 80 * 1024 : 160 * 1024;
  // the staged angle set sits after everything else; one that does not fit is read in place
  if (stage && base + 64 + (size_t)2 * p * sizeof(double) > 160 * 1024) stage = 0;
  const size_t angb = stage ? (size_t)2 * p * sizeof(double) : 0;
  const int pre = grad && with_pre + angb <= cap ? 1 : 0;
  const size_t lds = (pre ? with_pre : base + 64) + angb;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_whole<R, T, TT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_whole<R, T, TT>), dim3(n_items), dim3(256), lds, s, items, angles, p, grad, max_lut, pre, out,
                     stage);
  return hipGetLastError();
}

bool whole_supported(int precision, int n) { return precision == 0 ? (n == 12 || n == 13) : n == 12; }

hipError_t launch_whole(int precision, int n, int tbytes, const SmallItem *items, int n_items, int max_lut,
                        const double *angles, int p, int grad, double *out, hipStream_t s, int stage) {
  if (precision == 0) {
    if (n == 12)
      return tbytes == 1 ? launch_whole_t<float, 12, uint8_t>(items, n_items, max_lut, angles, p, grad, out, s, stage)
                         : launch_whole_t<float, 12, uint16_t>(items, n_items, max_lut, angles, p, grad, out, s, stage);
    if (n == 13)
      return tbytes == 1 ? launch_whole_t<float, 13, uint8_t>(items, n_items, max_lut, angles, p, grad, out, s, stage)
                         : launch_whole_t<float, 13, uint16_t>(items, n_items, max_lut, angles, p, grad, out, s, stage);
  } else if (n == 12) {
    return tbytes == 1 ? launch_whole_t<double, 12, uint8_t>(items, n_items, max_lut, angles, p, grad, out, s, stage)
                       : launch_whole_t<double, 12, uint16_t>(items, n_items, max_lut, angles, p, grad, out, s, stage);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_scale_copy(int precision, const void *src, void *dst, uint64_t N, double re,
                             double im, uint64_t flip, hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (precision == 0)
    k_scale_copy<float><<<g, 256, 0, s>>>((const float2 *)src, (float2 *)dst, N, re, im, flip);
  else
    k_scale_copy<double><<<g, 256, 0, s>>>((const double2 *)src, (double2 *)dst, N, re, im, flip);
  return hipGetLastError();
}

// Streaming copy (the measured HBM roof of a kernel that reads and writes every byte once):
// one 16-byte word per thread, consecutive threads consecutive words, non-temporal loads and
// stores (the data is touched once, so it should not displace other lines from the caches).
typedef unsigned int copy_word __attribute__((ext_vector_type(4)));
__global__ void k_stream_copy(const copy_word *__restrict__ src, copy_word *__restrict__ dst, uint64_t nwords) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nwords) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

hipError_t launch_stream_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s) {
  const uint64_t nwords = bytes / 16;
  if (nwords == 0) return hipSuccess;
  const uint64_t blocks = (nwords + 255) / 256;
  if (blocks > 0xffffffffull) return hipErrorInvalidValue;
  k_stream_copy<<<(unsigned)blocks, 256, 0, s>>>((const copy_word *)src, (copy_word *)dst, nwords);
  return hipGetLastError();
}

}  // namespace qaoa
