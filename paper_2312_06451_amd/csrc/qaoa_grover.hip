// Grover mixer (Golden et al., JuliQAOA, SC-W 2023, Sec. 2.4): H_M = |psi0><psi0|, psi0 the
// equal superposition over the feasible states. Every state of equal cost keeps an equal
// amplitude under the rounds of Eq. (1), so a whole evaluation runs on the distinct cost
// values c weighted by their degeneracies m_c (how many feasible states have cost c):
//
//   a_c <- e^{-i gamma c} a_c;   s = sum_c m_c a_c / sqrt(M);   a_c <- a_c + (e^{-i beta} - 1) s / sqrt(M)
//
// (M = number of feasible states, psi(x) = a_{C(x)}). The degeneracies are the data-parallel
// part: a histogram of a stored table, or, for MaxCut, a table-free count over all states
// (Gray-code order: consecutive states differ in one qubit, so the cut changes by the weights
// of that qubit's edges) or over the weight-k states (Gosper's order, Sec. 2.4).
#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

#include "qaoa_internal.h"

namespace qaoa {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum over a 256-thread block (all threads get the result); red holds 8 doubles.
__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

struct Z {
  double re, im;
};
__device__ __forceinline__ Z zmul(Z a, Z b) { return Z{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

}  // namespace

// ---------------------------------------------------------------- degeneracies

// counts[t[x]] += 1 over a stored table (block histogram in LDS, then 64-bit global adds).
template <typename TT>
__global__ __launch_bounds__(256) void k_hist_table(const TT *__restrict__ t, uint64_t N, int nbins,
                                                    unsigned long long *__restrict__ counts) {
  extern __shared__ unsigned int hs[];
  for (int b = threadIdx.x; b < nbins; b += 256) hs[b] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) atomicAdd(&hs[t[x]], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += 256)
    if (hs[b]) atomicAdd(&counts[b], (unsigned long long)hs[b]);
}

// Full space, MaxCut: thread g walks the 2^lo states whose high bits are base + g, in Gray-code
// order. Step i flips qubit q = ctz(i), the same qubit in every lane, so q's edges are
// wave-uniform data. With NW > 0 they are neighbour bitmasks, one per distinct edge weight w_j
// (masks[q * NW + j], classes beyond the graph's padded with empty masks), and the cut changes
// by (x_q ? -1 : 1) sum_j w_j (deg_j(q) - 2 popcount(mask_j(q) & x)) (an edge of q is cut after
// the flip iff its endpoints agree before it). For 2^lo >= 64 the walk runs in blocks of 32
// or 64 steps (walk_blocks); shorter walks take the flips one by one. With NW == 0, q's adjacency list
// (neighbour << 16 | weight, CSR) is walked instead. The histogram lives in LDS; with PRIV each
// thread owns a column of it.
template <int NW>
struct QMasks {
  uint64_t mk[NW > 0 ? NW : 1];
  int dg[NW > 0 ? NW : 1];
};

// Walk of the 2^lo states from x (low bits zero, cut c) in blocks of 2^LB steps. Steps
// 2^LB b + 1 .. 2^LB b + 2^LB - 1 flip qubits 0..LB-1; before step 2^LB b + r the low LB bits of
// x are G(r - 1) ^ 2^(LB-1) beta (G(r) = r ^ (r >> 1), beta = b & 1) and the bits above, H, stay
// fixed. With popcount(mask & x) = popcount(mask & H) + popcount(mask & low bits), step r
// changes the cut by s A_q + u_r, where
//   A_q = sum_j w_j (deg_j(q) - 2 popcount(mask_j(q) & H))        (per lane),
//   u_r = -2 s sum_j w_j popcount(mask_j(q) & low bits)            (wave-uniform),
// s = +1 when bit q is 0 before the step. Blocks run in pairs (beta = 0, 1), so q, s and the
// low bits are compile-time and one step is one add of three terms plus one LDS atomic. The
// cut is carried as its LDS byte address, cut * SC + the thread's column. Step 2^LB (b + 1)
// flips a qubit Q >= LB of H: its own cut change takes full popcounts, and A_q moves by
// -/+ 2 sum_j w_j [Q in mask_j(q)] as H gains or loses bit Q. Lane i of the wave holds qubit
// i's masks, read by Q with readlane (every lane is active: the launch has a multiple of 64
// threads). The u_r live in scalar registers for LB = 5 and in vector registers for LB = 6.
template <int LB, bool PRIV, int NW>
__device__ __forceinline__ void walk_blocks(uint64_t x, int c, uint64_t steps, int n, const uint64_t *__restrict__ masks,
                                            const int32_t *__restrict__ mdeg, const int *w, unsigned int *hist) {
  constexpr int BS = 1 << LB;
  constexpr uint32_t SC = PRIV ? 1024u : 4u;
  const uint32_t col = PRIV ? threadIdx.x * 4u : 0u;
  const int lane = threadIdx.x & 63;
  uint32_t lmlo[NW], lmhi[NW];
  int ldg[NW];
#pragma unroll
  for (int j = 0; j < NW; j++) {
    const uint64_t mk = lane < n ? masks[lane * NW + j] : 0ull;
    lmlo[j] = (uint32_t)mk;
    lmhi[j] = (uint32_t)(mk >> 32);
    ldg[j] = lane < n ? mdeg[lane * NW + j] : 0;
  }
  QMasks<NW> Qs[LB];
#pragma unroll
  for (int q = 0; q < LB; q++)
#pragma unroll
    for (int j = 0; j < NW; j++) {
      Qs[q].mk[j] = masks[q * NW + j];
      Qs[q].dg[j] = mdeg[q * NW + j];
    }
  uint32_t U[2][BS];
#pragma unroll
  for (int bt = 0; bt < 2; bt++)
#pragma unroll
    for (int r = 1; r < BS; r++) {
      const int q = __builtin_ctz(r);
      const uint32_t low = (uint32_t)((r - 1) ^ ((r - 1) >> 1)) ^ (uint32_t)(bt << (LB - 1));
      int K = 0;
#pragma unroll
      for (int j = 0; j < NW; j++) K += w[j] * __builtin_popcount((uint32_t)Qs[q].mk[j] & low);
      U[bt][r] = ((low >> q) & 1u) ? (uint32_t)(2 * K) * SC : (uint32_t)(-2 * K) * SC;
      // opaque: keeps u_r an added operand, not a subtraction, in the register file chosen
      if constexpr (LB <= 5) asm volatile("" : "+s"(U[bt][r]));
      else asm volatile("" : "+v"(U[bt][r]));
    }
  uint64_t H = x;  // low LB bits are 0 at the start
  uint32_t A[LB], nA[LB];
#pragma unroll
  for (int q = 0; q < LB; q++) {
    int a = 0;
#pragma unroll
    for (int j = 0; j < NW; j++) a += w[j] * (Qs[q].dg[j] - 2 * (int)__builtin_popcountll(Qs[q].mk[j] & H));
    A[q] = (uint32_t)a * SC;
    nA[q] = 0u - A[q];
  }
  // cs is the LDS address itself (the histogram's base included), so a step's atomic takes it
  // as is
  typedef __attribute__((address_space(3))) unsigned int lds_u32;
  uint32_t cs = (uint32_t)(size_t)(lds_u32 *)hist + (uint32_t)c * SC + col;
  auto at = [&](uint32_t a) { __atomic_fetch_add((lds_u32 *)(size_t)a, 1u, __ATOMIC_RELAXED); };
  auto block = [&](auto beta_c) {
    constexpr uint32_t bt = decltype(beta_c)::value;
#pragma unroll
    for (int r = 1; r < BS; r++) {
      const int q = __builtin_ctz(r);
      const uint32_t low = (uint32_t)((r - 1) ^ ((r - 1) >> 1)) ^ (bt << (LB - 1));
      cs = (cs + (((low >> q) & 1u) ? nA[q] : A[q])) + U[bt][r];
      at(cs);
    }
  };
  // flip of qubit Q >= LB with the low bits equal to lowx (wave-uniform)
  auto flip_high = [&](int Q, uint32_t lowx) {
    const uint32_t bit = (uint32_t)(H >> Q) & 1u;
    int t = 0;
#pragma unroll
    for (int j = 0; j < NW; j++) {
      const uint32_t mlo = (uint32_t)__builtin_amdgcn_readlane((int)lmlo[j], Q);
      const uint32_t mhi = (uint32_t)__builtin_amdgcn_readlane((int)lmhi[j], Q);
      const int dq = __builtin_amdgcn_readlane(ldg[j], Q);
      const int pc = (int)(__builtin_popcount(mlo & (uint32_t)H) + __builtin_popcount(mhi & (uint32_t)(H >> 32)) +
                           __builtin_popcount(mlo & lowx));
      t += __mul24(w[j], __mul24(-2, pc) + dq);
    }
    const int sgn = bit ? -(int)SC : (int)SC;  // s * SC
    cs += (uint32_t)__mul24(sgn, t);
#pragma unroll
    for (int q = 0; q < LB; q++) {
      int d = 0;
#pragma unroll
      for (int j = 0; j < NW; j++) d += w[j] * (int)((Qs[q].mk[j] >> Q) & 1ull);
      A[q] += (uint32_t)__mul24(sgn, -2 * d);
      nA[q] += (uint32_t)__mul24(sgn, 2 * d);
    }
    H ^= 1ull << Q;
    at(cs);
  };
  const uint64_t pairs = steps >> (LB + 1);
  for (uint64_t pr = 0; pr < pairs; pr++) {
    block(std::integral_constant<uint32_t, 0>{});
    flip_high(LB, 1u << (LB - 1));  // low bits after a beta = 0 block: G(2^LB - 1) = 2^(LB-1)
    block(std::integral_constant<uint32_t, 1>{});
    if (pr + 1 < pairs) flip_high(__builtin_ctzll(pr + 1) + LB + 1, 0u);
  }
}

template <bool PRIV, int NW>
__global__ __launch_bounds__(256) void k_enum_full(int n, int m, const int32_t *__restrict__ eu,
                                                   const int32_t *__restrict__ ev, const int32_t *__restrict__ ew,
                                                   const int32_t *__restrict__ adj_off, const int32_t *__restrict__ adj,
                                                   const uint64_t *__restrict__ masks, const int32_t *__restrict__ mdeg,
                                                   const int32_t *__restrict__ wvals, int lo, uint64_t base,
                                                   uint64_t nthreads, int nbins, unsigned long long *__restrict__ counts) {
  extern __shared__ unsigned int smem_u[];
  unsigned int *hist = smem_u;  // PRIV: [nbins][256], else [nbins]
  const int hsz = PRIV ? nbins * 256 : nbins;
  for (int i = threadIdx.x; i < hsz; i += 256) hist[i] = 0;
  __syncthreads();
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (g < nthreads) {
    uint64_t x = (base + g) << lo;
    int c = 0;
    for (int e = 0; e < m; e++) c += ew[e] * (int)(((x >> eu[e]) ^ (x >> ev[e])) & 1ull);
    auto bump = [&](int v) {
      if (PRIV) atomicAdd(&hist[v * 256 + threadIdx.x], 1u);  // private slot: no contention
      else atomicAdd(&hist[v], 1u);
    };
    bump(c);
    const uint64_t steps = 1ull << lo;
    if constexpr (NW > 0) {
      int w[NW];
#pragma unroll
      for (int j = 0; j < NW; j++) w[j] = wvals[j];
      auto load = [&](int q) {
        QMasks<NW> r;
#pragma unroll
        for (int j = 0; j < NW; j++) {
          r.mk[j] = masks[q * NW + j];
          r.dg[j] = mdeg[q * NW + j];
        }
        return r;
      };
      auto flip = [&](int q, const QMasks<NW> &Q) {
        int t = 0;
#pragma unroll
        for (int j = 0; j < NW; j++)  // 24-bit products: weights <= 16383, |deg - 2 popcount| <= 64
          t += __mul24(w[j], __mul24(-2, (int)__builtin_popcountll(Q.mk[j] & x)) + Q.dg[j]);
        c += ((x >> q) & 1ull) ? -t : t;
        x ^= 1ull << q;
        bump(c);
      };
      if (lo >= 7) {
        walk_blocks<6, PRIV, NW>(x, c, steps, n, masks, mdeg, w, hist);
      } else if (lo >= 6) {
        walk_blocks<5, PRIV, NW>(x, c, steps, n, masks, mdeg, w, hist);
      } else {
        for (uint64_t i = 1; i < steps; i++) {
          const int q = __builtin_ctzll(i);
          flip(q, load(q));
        }
      }
    } else {
      for (uint64_t i = 1; i < steps; i++) {
        const int q = __builtin_ctzll(i);
        const uint64_t d = ((x >> q) & 1ull) ? ~x : x;
        for (int j = adj_off[q]; j < adj_off[q + 1]; j++) {
          const int a = adj[j];
          const int vtx = a >> 16, wt = a & 0xffff;
          c += ((d >> vtx) & 1ull) ? -wt : wt;
        }
        x ^= 1ull << q;
        bump(c);
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += 256) {
    unsigned long long s = 0;
    if (PRIV)
      for (int t = 0; t < 256; t++) s += hist[b * 256 + ((t + b) & 255)];
    else
      s = hist[b];
    if (s) atomicAdd(&counts[b], s);
  }
}

// Weight-k states, MaxCut (n <= 32: binomials C(a, i) at binom[a * 33 + i]): thread g < nthreads
// takes ranks [r0 + g * per, ...) of the weight-k integers in increasing order, unranks the
// first one and steps with Gosper's hack.
__global__ __launch_bounds__(256) void k_enum_hw(int n, int k, int m, const int32_t *__restrict__ eu,
                                                 const int32_t *__restrict__ ev, const int32_t *__restrict__ ew,
                                                 const int64_t *__restrict__ binom, uint64_t r0, uint64_t per,
                                                 uint64_t total, uint64_t nthreads, int nbins,
                                                 unsigned long long *__restrict__ counts) {
  extern __shared__ unsigned int hist[];
  for (int i = threadIdx.x; i < nbins; i += 256) hist[i] = 0;
  __syncthreads();
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t first = r0 + g * per;
  if (g < nthreads && first < total) {
    const uint64_t cnt = (total - first < per) ? total - first : per;
    uint64_t rem = first, x = 0;
    int a = n - 1;
    for (int i = k; i >= 1; i--) {
      while (a >= i && (uint64_t)binom[a * 33 + i] > rem) a--;
      x |= 1ull << a;
      rem -= (uint64_t)binom[a * 33 + i];
      a--;
    }
    for (uint64_t s = 0; s < cnt; s++) {
      int c = 0;
      for (int e = 0; e < m; e++) c += ew[e] * (int)(((x >> eu[e]) ^ (x >> ev[e])) & 1ull);
      atomicAdd(&hist[c], 1u);
      if (k > 0) {  // next larger integer with the same number of ones
        const uint64_t lowbit = x & (~x + 1ull);
        const uint64_t r = x + lowbit;
        x = (((r ^ x) >> 2) >> __builtin_ctzll(lowbit)) | r;
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += 256)
    if (hist[b]) atomicAdd(&counts[b], (unsigned long long)hist[b]);
}

// ---------------------------------------------------------------- evaluation on the classes

// One workgroup per item: FP64 rounds on the classes, <C> and (grad) the adjoint sweep.
// Classes c = tid + 256 j, j < GROVER_CPT, held in registers.
__global__ __launch_bounds__(256) void k_grover(const GroverItem *__restrict__ items, const double *__restrict__ angles,
                                                int p, int grad, double *__restrict__ out) {
  __shared__ double red[8];
  const GroverItem it = items[blockIdx.x];
  const int tid = threadIdx.x, D = it.nclass;
  const double *ang = angles + (size_t)it.angle_set * 2 * p;
  const double rM = 1.0 / sqrt(it.total);
  double v[GROVER_CPT], mc[GROVER_CPT];
  Z phi[GROVER_CPT], lam[GROVER_CPT];
#pragma unroll
  for (int j = 0; j < GROVER_CPT; j++) {
    const int c = tid + 256 * j;
    v[j] = c < D ? it.vals[c] : 0.0;
    mc[j] = c < D ? it.counts[c] : 0.0;
    phi[j] = Z{rM, 0.0};
  }
  // <psi0|u> = sum_c m_c u_c / sqrt(M)
  auto overlap = [&](const Z *u) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int j = 0; j < GROVER_CPT; j++) {
      sr += mc[j] * u[j].re;
      si += mc[j] * u[j].im;
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red + 4);
    return Z{sr * rM, si * rM};
  };
  auto phase = [&](Z *u, double gamma) {
#pragma unroll
    for (int j = 0; j < GROVER_CPT; j++) {
      double s, c;
      sincos(-gamma * v[j], &s, &c);
      u[j] = zmul(u[j], Z{c, s});
    }
  };
  auto mix = [&](Z *u, double beta, Z ov) {  // u += (e^{-i beta} - 1) <psi0|u> psi0
    double s, c;
    sincos(-beta, &s, &c);
    const Z d = zmul(Z{c - 1.0, s}, ov);
#pragma unroll
    for (int j = 0; j < GROVER_CPT; j++) u[j] = Z{u[j].re + d.re * rM, u[j].im + d.im * rM};
  };
  for (int k = 0; k < p; k++) {
    phase(phi, ang[p + k]);
    mix(phi, ang[k], overlap(phi));
  }
  double e = 0.0, nr = 0.0;
#pragma unroll
  for (int j = 0; j < GROVER_CPT; j++) {
    const double pr = mc[j] * (phi[j].re * phi[j].re + phi[j].im * phi[j].im);
    e += pr * v[j];
    nr += pr;
  }
  e = block_sum(e, red);
  nr = block_sum(nr, red + 4);
  double *o = out + (size_t)it.out_index * (1 + 2 * p);
  if (tid == 0) o[0] = e / nr;
  if (it.amp_out) {
#pragma unroll
    for (int j = 0; j < GROVER_CPT; j++) {
      const int c = tid + 256 * j;
      if (c < D) it.amp_out[c] = double2{phi[j].re, phi[j].im};
    }
  }
  if (!grad) return;
  // lambda = (C - c0) psi_p; then for k = p..1: g_beta = 2 Im <lam|H_G|phi>
  // = 2 Im(conj(<psi0|lam>) <psi0|phi>), undo the mixer, g_gamma = 2 Im <lam|(C - c0)|phi>,
  // undo the phase
#pragma unroll
  for (int j = 0; j < GROVER_CPT; j++) lam[j] = Z{(v[j] - it.c0) * phi[j].re, (v[j] - it.c0) * phi[j].im};
  for (int k = p - 1; k >= 0; k--) {
    const Z ol = overlap(lam), op = overlap(phi);
    if (tid == 0) o[1 + k] = 2.0 * (ol.re * op.im - ol.im * op.re) / nr;
    mix(phi, -ang[k], op);
    mix(lam, -ang[k], ol);
    double gg = 0.0;
#pragma unroll
    for (int j = 0; j < GROVER_CPT; j++) gg += mc[j] * (v[j] - it.c0) * (lam[j].re * phi[j].im - lam[j].im * phi[j].re);
    gg = block_sum(gg, red);
    if (tid == 0) o[1 + p + k] = 2.0 * gg / nr;
    phase(phi, -ang[p + k]);
    phase(lam, -ang[p + k]);
  }
}

// psi(x) = amp[t[x]] for the state output (complex64 or complex128).
template <typename TT, typename T2>
__global__ void k_grover_expand(const TT *__restrict__ t, uint64_t N, const double2 *__restrict__ amp, T2 *out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) {
    const double2 a = amp[t[x]];
    out[x] = T2{(decltype(T2::x))a.x, (decltype(T2::x))a.y};
  }
}

// ---------------------------------------------------------------- launch wrappers

static unsigned grid_of(uint64_t N) {
  uint64_t g = (N + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_hist_table(const void *table, int tbytes, uint64_t N, int nbins, unsigned long long *counts,
                             hipStream_t s) {
  const size_t lds = (size_t)nbins * sizeof(unsigned int);
  if (tbytes == 1)
    k_hist_table<uint8_t><<<grid_of(N), 256, lds, s>>>((const uint8_t *)table, N, nbins, counts);
  else
    k_hist_table<uint16_t><<<grid_of(N), 256, lds, s>>>((const uint16_t *)table, N, nbins, counts);
  return hipGetLastError();
}

size_t enum_full_lds(int nbins, bool priv) { return (size_t)(priv ? nbins * 256 : nbins) * 4; }

template <bool P, int NW>
static hipError_t enum_full_t(dim3 blocks, size_t lds, hipStream_t s, int n, int m, const int32_t *eu,
                              const int32_t *ev, const int32_t *ew, const int32_t *adj_off, const int32_t *adj,
                              const uint64_t *masks, const int32_t *mdeg, const int32_t *wvals, int lo, uint64_t base,
                              uint64_t nthreads, int nbins, unsigned long long *counts) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k_enum_full<P, NW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  k_enum_full<P, NW><<<blocks, 256, lds, s>>>(n, m, eu, ev, ew, adj_off, adj, masks, mdeg, wvals, lo, base, nthreads,
                                              nbins, counts);
  return hipGetLastError();
}

hipError_t launch_enum_full(int n, int m, const int32_t *eu, const int32_t *ev, const int32_t *ew,
                            const int32_t *adj_off, const int32_t *adj, const uint64_t *masks, const int32_t *mdeg,
                            const int32_t *wvals, int nw, int lo, uint64_t base, uint64_t nthreads, int nbins,
                            bool priv, unsigned long long *counts, hipStream_t s) {
  const size_t lds = enum_full_lds(nbins, priv);
  const dim3 blocks((unsigned)((nthreads + 255) / 256));
  if (masks && nw != 1 && nw != 2 && nw != 4 && nw != 8) return hipErrorInvalidValue;
  if (masks && lo >= 6 && (nthreads & 63)) return hipErrorInvalidValue;  // the block walk reads every lane
  const int k = masks ? nw : 0;
#define QAOA_ENUM_CASE(P, NW)                                                                                 \
  if (priv == P && k == NW)                                                                                    \
    return enum_full_t<P, NW>(blocks, lds, s, n, m, eu, ev, ew, adj_off, adj, masks, mdeg, wvals, lo, base, nthreads, \
                              nbins, counts);
  QAOA_ENUM_CASE(true, 0) QAOA_ENUM_CASE(true, 1) QAOA_ENUM_CASE(true, 2) QAOA_ENUM_CASE(true, 4)
  QAOA_ENUM_CASE(true, 8) QAOA_ENUM_CASE(false, 0) QAOA_ENUM_CASE(false, 1) QAOA_ENUM_CASE(false, 2)
  QAOA_ENUM_CASE(false, 4) QAOA_ENUM_CASE(false, 8)
#undef QAOA_ENUM_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_enum_hw(int n, int k, int m, const int32_t *eu, const int32_t *ev, const int32_t *ew,
                          const int64_t *binom, uint64_t r0, uint64_t per, uint64_t total, uint64_t nthreads,
                          int nbins, unsigned long long *counts, hipStream_t s) {
  const unsigned blocks = (unsigned)((nthreads + 255) / 256);
  k_enum_hw<<<blocks, 256, (size_t)nbins * 4, s>>>(n, k, m, eu, ev, ew, binom, r0, per, total, nthreads, nbins,
                                                   counts);
  return hipGetLastError();
}

hipError_t launch_grover(const GroverItem *items, int n_items, const double *angles, int p, int grad, double *out,
                         hipStream_t s) {
  k_grover<<<n_items, 256, 0, s>>>(items, angles, p, grad, out);
  return hipGetLastError();
}

hipError_t launch_grover_expand(const void *table, int tbytes, uint64_t N, const double2 *amp, void *out,
                                int precision, hipStream_t s) {
  if (precision == 0) {
    if (tbytes == 1) k_grover_expand<uint8_t, float2><<<grid_of(N), 256, 0, s>>>((const uint8_t *)table, N, amp, (float2 *)out);
    else k_grover_expand<uint16_t, float2><<<grid_of(N), 256, 0, s>>>((const uint16_t *)table, N, amp, (float2 *)out);
  } else {
    if (tbytes == 1) k_grover_expand<uint8_t, double2><<<grid_of(N), 256, 0, s>>>((const uint8_t *)table, N, amp, (double2 *)out);
    else k_grover_expand<uint16_t, double2><<<grid_of(N), 256, 0, s>>>((const uint16_t *)table, N, amp, (double2 *)out);
  }
  return hipGetLastError();
}

}  // namespace qaoa
