// Mixers applied through their eigendecomposition (Golden et al., JuliQAOA, SC-W 2023,
// Sec. 2.1-2.2): the clique mixer sum_{i<j} X_iX_j + Y_iY_j, the ring mixer
// sum_i X_iX_{i+1} + Y_iY_{i+1} (i + 1 mod n), or any real symmetric matrix handed over by the
// caller. On the weight-k states (increasing integer order) the clique and ring mixers are
// real symmetric matrices H with entry 2 between states that differ by one allowed swap.
// H is diagonalised once in FP64 (H = V D V^T, rocSOLVER), and every round applies
//     psi <- exp(-i gamma C) psi,   psi <- V exp(-i beta D) V^T psi,
// i.e. two dense products per round, for all angle sets at once: the state of S angle sets is
// an N x 2S real matrix (real and imaginary parts as separate columns).
//
// FP32 form: each product is formed from FP16 halves with FP32 accumulation (MFMA GEMMs of
// hipBLASLt; for each product shape the fastest of the library's candidate algorithms is
// timed and kept on first use, rocBLAS when none runs): with x = x_hi + 2^-11 x_lo
// (x_hi = fp16(x), x_lo = fp16(2^11 (x - x_hi))),
//     V B ~ V_hi B_hi + 2^-11 (V_hi B_lo + V_lo B_hi),
// two GEMM calls (K = N, then K = 2N on the stacked halves); the dropped V_lo B_lo term is
// 2^-22 relative. FP64 form: DGEMM on the FP64 eigenbasis.
//
// Gradient: the reverse sweep of the X path with H_M = V D V^T. The forward sweep keeps, per
// round, the phased state (before V^T) and its eigen-coefficients after exp(-i beta D); then
// only the adjoint vector needs products:
//   lam~ = V^T lam;  g_beta = 2 sum_r D_r Im(conj(lam~_r) phi~_r);  lam~ *= exp(+i beta D);
//   lam = V lam~;    g_gamma = 2 sum_x (C - c0) Im(conj(lam) phi);  lam *= exp(+i gamma C).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <hipblaslt/hipblaslt.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/qaoa.h"
#include "qaoa_clique.h"
#include "qaoa_internal.h"

namespace qaoa {

namespace {

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
  void *get(size_t bytes) {
    if (bytes <= cap && p) return p;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (bytes == 0) return nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw CliqueError{QAOA_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    cap = bytes;
    return p;
  }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

void hipchk(hipError_t e, const char *what) {
  if (e != hipSuccess) throw CliqueError{QAOA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}
void ltchk(hipblasStatus_t s, const char *what) {
  if (s != HIPBLAS_STATUS_SUCCESS)
    throw CliqueError{QAOA_ERR_HIP, std::string(what) + ": hipBLASLt status " + std::to_string((int)s)};
}
void blaschk(rocblas_status s, const char *what) {
  if (s != rocblas_status_success)
    throw CliqueError{QAOA_ERR_HIP, std::string(what) + ": " + rocblas_status_to_string(s)};
}

int64_t binom64(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return r;
}

constexpr int RB_ROWS = 1024;  // rows per block in the elementwise kernels (4 per thread)

}  // namespace

// One FP16 x FP16 -> FP32 GEMM shape of the split products with its selected algorithm.
struct LtGemm {
  hipblasLtMatmulDesc_t desc = nullptr;
  hipblasLtMatrixLayout_t a = nullptr, b = nullptr, c = nullptr;
  hipblasLtMatmulAlgo_t algo{};
  size_t ws = 0;
  bool ok = false;  // false: no hipBLASLt algorithm ran, use rocBLAS
  ~LtGemm() {
    if (a) (void)hipblasLtMatrixLayoutDestroy(a);
    if (b) (void)hipblasLtMatrixLayoutDestroy(b);
    if (c) (void)hipblasLtMatrixLayoutDestroy(c);
    if (desc) (void)hipblasLtMatmulDescDestroy(desc);
  }
};

struct CliqueMixer {
  int n = 0, k = 0;
  int64_t N = 0;
  rocblas_handle blas = nullptr;
  hipblasLtHandle_t lt = nullptr;
  std::map<std::tuple<int, int, int>, std::unique_ptr<LtGemm>> gemms;  // (transpose, K/N, cols)
  Buf ltws;                                                               // hipBLASLt workspace
  Buf V, D, Vcols, Vrows;  // FP64 eigenbasis (N x N col-major, column j = eigenvector j),
                           // eigenvalues, FP16 halves [V_hi | V_lo] (N x 2N) and [V_hi; V_lo] (2N x N)
  Buf X, Y, B, ckP, ckT, partials, params, luts, results, hres_dev;
  std::vector<double> hres;
  CliqueTimer timer;
  ~CliqueMixer() {
    gemms.clear();
    if (lt) (void)hipblasLtDestroy(lt);
    if (blas) (void)rocblas_destroy_handle(blas);
  }
};

void CliqueMixerDeleter::operator()(CliqueMixer *m) const { delete m; }

void clique_set_timer(CliqueMixer &m, const CliqueTimer &t) { m.timer = t; }

// ---------------------------------------------------------------- kernels

// Rank of a weight-k integer y among the weight-k integers in increasing order
// (combinatorial number system: sum over its set bits b_1 < ... < b_k of C(b_i, i)).
__device__ int64_t rank_hw(uint64_t y, const int64_t *binom) {
  int64_t r = 0;
  int i = 1;
  for (int b = 0; b < 64 && y; b++) {
    if ((y >> b) & 1u) {
      r += binom[b * 33 + i];
      i++;
      y &= ~(1ull << b);
    }
  }
  return r;
}

// The r-th weight-k integer in increasing order.
__device__ uint64_t unrank_hw(int64_t r, int n, int k, const int64_t *binom) {
  uint64_t rem = (uint64_t)r, x = 0;
  int a = n - 1;
  for (int i = k; i >= 1; i--) {
    while (a >= i && (uint64_t)binom[a * 33 + i] > rem) a--;
    x |= 1ull << a;
    rem -= (uint64_t)binom[a * 33 + i];
    a--;
  }
  return x;
}

// H[c, r] = 2 for every swap neighbour c of state r (H zeroed beforehand): any 1-bit moved to
// any 0-bit (clique), or only across the ring edges (i, i + 1 mod n) (ring).
__global__ void k_clique_matrix(int n, int k, int ring, int64_t N, const int64_t *__restrict__ binom,
                                double *__restrict__ H) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const uint64_t x = unrank_hw(r, n, k, binom);
  for (int a = 0; a < n; a++) {
    if (!((x >> a) & 1u)) continue;
    for (int b = 0; b < n; b++) {
      if ((x >> b) & 1u) continue;
      if (ring && b != (a + 1) % n && a != (b + 1) % n) continue;
      const uint64_t y = x ^ (1ull << a) ^ (1ull << b);
      H[rank_hw(y, binom) + r * N] = 2.0;
    }
  }
}

// FP16 halves of V: hi = fp16(v), lo = fp16(2^11 (v - hi)).
__global__ void k_split_v(const double *__restrict__ V, int64_t N, __half *__restrict__ Vcols,
                          __half *__restrict__ Vrows) {
  const int64_t total = N * N, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t row = i % N, col = i / N;
    const double v = V[i];
    const __half hi = __float2half((float)v);
    const __half lo = __float2half((float)((v - (double)__half2float(hi)) * 2048.0));
    Vcols[row + col * N] = hi;
    Vcols[row + (col + N) * N] = lo;
    Vrows[row + col * 2 * N] = hi;
    Vrows[row + N + col * 2 * N] = lo;
  }
}

template <typename R> struct CT;
template <> struct CT<float> { using T2 = float2; };
template <> struct CT<double> { using T2 = double2; };

// Write the complex value v of row x, set s as the next product's input: FP16 halves in the
// stacked layout [lo; hi] (2N rows) for the FP32 form, the value itself for the FP64 form.
template <typename R>
__device__ __forceinline__ void emit(void *B, int64_t N, int64_t x, int s, R re, R im) {
  if constexpr (sizeof(R) == 4) {
    __half *b = (__half *)B;
    const __half hr = __float2half(re), hi = __float2half(im);
    const int64_t c0 = (int64_t)(2 * s) * 2 * N, c1 = (int64_t)(2 * s + 1) * 2 * N;
    b[c0 + N + x] = hr;
    b[c0 + x] = __float2half((re - __half2float(hr)) * 2048.0f);
    b[c1 + N + x] = hi;
    b[c1 + x] = __float2half((im - __half2float(hi)) * 2048.0f);
  } else {
    R *b = (R *)B;
    b[(int64_t)(2 * s) * N + x] = re;
    b[(int64_t)(2 * s + 1) * N + x] = im;
  }
}

template <typename TT>
__device__ __forceinline__ uint32_t cval(const void *t, int64_t x) {
  return (uint32_t)((const TT *)t)[x];
}

// Block sum of two doubles per thread (256 threads), written as partials.
__device__ void block_sum2(double a, double b, double *pa, double *pb) {
  __shared__ double ra[4], rb[4];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = a;
    rb[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (pa) *pa = (ra[0] + ra[1]) + (ra[2] + ra[3]);
    if (pb) *pb = (rb[0] + rb[1]) + (rb[2] + rb[3]);
  }
}

// Initial state (uniform over the weight-k states, or the caller's) -> phase of round 1 ->
// next product's input (and the phased state kept for the gradient).
template <typename R>
__global__ void k_init(R *__restrict__ X, int64_t N, const void *psi0) {
  const int s = blockIdx.y;
  const R u = (R)(1.0 / sqrt((double)N));
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    R re = u, im = 0;
    if (psi0) {
      const typename CT<R>::T2 v = ((const typename CT<R>::T2 *)psi0)[x];
      re = v.x;
      im = v.y;
    }
    X[(int64_t)(2 * s) * N + x] = re;
    X[(int64_t)(2 * s + 1) * N + x] = im;
  }
}

// psi(x, s) *= LUT_s[C(x)]; keep the result (ck) and emit it for V^T.
template <typename R, typename TT>
__global__ void k_phase(const R *__restrict__ X, int64_t N, const void *table,
                        const typename CT<R>::T2 *__restrict__ luts, int lut_len, R *ck, void *B) {
  const int s = blockIdx.y;
  const typename CT<R>::T2 *L = luts + (int64_t)s * lut_len;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    const R a = X[(int64_t)(2 * s) * N + x], b = X[(int64_t)(2 * s + 1) * N + x];
    const typename CT<R>::T2 l = L[cval<TT>(table, x)];
    const R re = a * l.x - b * l.y, im = a * l.y + b * l.x;
    if (ck) {
      ck[(int64_t)(2 * s) * N + x] = re;
      ck[(int64_t)(2 * s + 1) * N + x] = im;
    }
    emit<R>(B, N, x, s, re, im);
  }
}

// Eigen-coefficients t(r, s) (product output Y) times exp(sign i beta_s D_r), phase in FP64.
// With tref: g_beta partial sum_r D_r Im(conj(t) tref) before the phase (one per block).
template <typename R>
__global__ __launch_bounds__(256) void k_eig(const R *__restrict__ Y, int64_t N, const double *__restrict__ D,
                                             const double *__restrict__ betas, double sign,
                                             const R *tref, R *ck, void *B, double *gpart, int nblk) {
  const int s = blockIdx.y;
  const double beta = betas[s];
  double acc = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * RB_ROWS;
  for (int64_t r = r0 + threadIdx.x; r < N && r < r0 + RB_ROWS; r += 256) {
    const R a = Y[(int64_t)(2 * s) * N + r], b = Y[(int64_t)(2 * s + 1) * N + r];
    const double d = D[r];
    if (tref) {
      const R ta = tref[(int64_t)(2 * s) * N + r], tb = tref[(int64_t)(2 * s + 1) * N + r];
      acc += d * ((double)a * tb - (double)b * ta);
    }
    double sn, cs;
    sincos(sign * beta * d, &sn, &cs);
    const R re = (R)((double)a * cs - (double)b * sn), im = (R)((double)a * sn + (double)b * cs);
    if (ck) {
      ck[(int64_t)(2 * s) * N + r] = re;
      ck[(int64_t)(2 * s + 1) * N + r] = im;
    }
    emit<R>(B, N, r, s, re, im);
  }
  if (gpart) block_sum2(acc, 0.0, gpart + (int64_t)s * nblk + blockIdx.x, nullptr);
}

// E and Nrm partials of the final state.
template <typename R, typename TT>
__global__ __launch_bounds__(256) void k_expect(const R *__restrict__ X, int64_t N, const void *table,
                                                const double *__restrict__ vals, double *epart, double *npart,
                                                int nblk) {
  const int s = blockIdx.y;
  double e = 0.0, nr = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * RB_ROWS;
  for (int64_t x = r0 + threadIdx.x; x < N && x < r0 + RB_ROWS; x += 256) {
    const double a = X[(int64_t)(2 * s) * N + x], b = X[(int64_t)(2 * s + 1) * N + x];
    const double pr = a * a + b * b;
    e += pr * vals[cval<TT>(table, x)];
    nr += pr;
  }
  block_sum2(e, nr, epart + (int64_t)s * nblk + blockIdx.x, npart + (int64_t)s * nblk + blockIdx.x);
}

// lam = (C - c0) psi_p, emitted for V^T.
template <typename R, typename TT>
__global__ void k_lambda(const R *__restrict__ X, int64_t N, const void *table, const double *__restrict__ vals,
                         double c0, void *B) {
  const int s = blockIdx.y;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    const R k = (R)(vals[cval<TT>(table, x)] - c0);
    emit<R>(B, N, x, s, k * X[(int64_t)(2 * s) * N + x], k * X[(int64_t)(2 * s + 1) * N + x]);
  }
}

// g_gamma partial sum_x (C - c0) Im(conj(lam) phi) with phi the kept phased state; then
// lam *= LUT_s[C] (inverse phase) and emit it for the next V^T (if B).
template <typename R, typename TT>
__global__ __launch_bounds__(256) void k_gamma(const R *__restrict__ L, int64_t N, const void *table,
                                               const double *__restrict__ vals, double c0, const R *__restrict__ phi,
                                               const typename CT<R>::T2 *luts, int lut_len, void *B,
                                               double *gpart, int nblk) {
  const int s = blockIdx.y;
  double acc = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * RB_ROWS;
  for (int64_t x = r0 + threadIdx.x; x < N && x < r0 + RB_ROWS; x += 256) {
    const R a = L[(int64_t)(2 * s) * N + x], b = L[(int64_t)(2 * s + 1) * N + x];
    const R pa = phi[(int64_t)(2 * s) * N + x], pb = phi[(int64_t)(2 * s + 1) * N + x];
    const uint32_t c = cval<TT>(table, x);
    acc += (vals[c] - c0) * ((double)a * pb - (double)b * pa);
    if (B) {
      const typename CT<R>::T2 l = luts[(int64_t)s * lut_len + c];
      emit<R>(B, N, x, s, a * l.x - b * l.y, a * l.y + b * l.x);
    }
  }
  block_sum2(acc, 0.0, gpart + (int64_t)s * nblk + blockIdx.x, nullptr);
}

template <typename R>
__global__ void k_export(const R *__restrict__ X, int64_t N, typename CT<R>::T2 *out) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x)
    out[x] = typename CT<R>::T2{X[x], X[N + x]};
}

// ---------------------------------------------------------------- setup

std::unique_ptr<CliqueMixer, CliqueMixerDeleter> clique_create(int kind, int n, int k, const double *host_matrix,
                                                                 const double *host_eigenvalues, hipStream_t st) {
  std::unique_ptr<CliqueMixer, CliqueMixerDeleter> m(new CliqueMixer());
  m->n = n;
  m->k = k;
  const int64_t N = k < 0 ? (int64_t(1) << n) : binom64(n, k);
  m->N = N;
  blaschk(rocblas_create_handle(&m->blas), "rocblas_create_handle");
  blaschk(rocblas_set_stream(m->blas, st), "rocblas_set_stream");
  // clique matrix (FP64, dense) -> eigendecomposition in place
  double *H = (double *)m->V.get((size_t)N * N * sizeof(double));
  double *Dv = (double *)m->D.get((size_t)N * sizeof(double));
  std::vector<int64_t> hb(33 * 33);
  for (int a = 0; a <= 32; a++)
    for (int b = 0; b <= 32; b++) hb[a * 33 + b] = binom64(a, b);
  Buf dbin, E, info;
  int64_t *db = (int64_t *)dbin.get(hb.size() * sizeof(int64_t));
  hipchk(hipMemcpyAsync(db, hb.data(), hb.size() * sizeof(int64_t), hipMemcpyHostToDevice, st), "binom upload");
  if (kind == MIX_EIGEN) {
    // a stored eigendecomposition: V (column j = eigenvector j) and D, no eigensolver
    hipchk(hipMemcpyAsync(H, host_matrix, (size_t)N * N * sizeof(double), hipMemcpyHostToDevice, st), "V upload");
    hipchk(hipMemcpyAsync(Dv, host_eigenvalues, (size_t)N * sizeof(double), hipMemcpyHostToDevice, st), "D upload");
  } else if (kind == MIX_MATRIX) {
    hipchk(hipMemcpyAsync(H, host_matrix, (size_t)N * N * sizeof(double), hipMemcpyHostToDevice, st), "matrix upload");
  } else {
    hipchk(hipMemsetAsync(H, 0, (size_t)N * N * sizeof(double), st), "clear H");
    k_clique_matrix<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(n, k, kind == MIX_RING ? 1 : 0, N, db, H);
    hipchk(hipGetLastError(), "k_clique_matrix");
  }
  if (kind != MIX_EIGEN) {
    double *dE = (double *)E.get((size_t)N * sizeof(double));
    rocblas_int *dinfo = (rocblas_int *)info.get(sizeof(rocblas_int));
    blaschk(rocsolver_dsyevd(m->blas, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)N, H,
                             (rocblas_int)N, Dv, dE, dinfo),
            "rocsolver_dsyevd");
    rocblas_int hinfo = 0;
    hipchk(hipMemcpyAsync(&hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, st), "info download");
    hipchk(hipStreamSynchronize(st), "eigendecomposition");
    if (hinfo != 0) throw CliqueError{QAOA_ERR_HIP, "eigendecomposition did not converge"};
  }
  // FP16 halves for the FP32 form
  __half *Vc = (__half *)m->Vcols.get((size_t)2 * N * N * sizeof(__half));
  __half *Vr = (__half *)m->Vrows.get((size_t)2 * N * N * sizeof(__half));
  k_split_v<<<4096, 256, 0, st>>>(H, N, Vc, Vr);
  hipchk(hipGetLastError(), "k_split_v");
  hipchk(hipStreamSynchronize(st), "split V");
  return m;
}

void clique_export(const CliqueMixer &m, double *host_V, double *host_D, hipStream_t st) {
  const size_t N = (size_t)m.N;
  hipchk(hipMemcpyAsync(host_V, m.V.p, N * N * sizeof(double), hipMemcpyDeviceToHost, st), "V download");
  hipchk(hipMemcpyAsync(host_D, m.D.p, N * sizeof(double), hipMemcpyDeviceToHost, st), "D download");
  hipchk(hipStreamSynchronize(st), "eigenbasis download");
}

int64_t clique_size(const CliqueMixer &m) { return m.N; }

// ---------------------------------------------------------------- evaluation

namespace {

constexpr size_t LT_WORKSPACE = 64ull << 20;

// Creates the descriptors of one split-product GEMM (D = alpha op(A) B + beta D, A the FP16
// eigenbasis halves, B the FP16 state halves with leading dimension 2N, D FP32 N x cols) and
// times the library's candidate algorithms on the given operands; keeps the fastest.
// Overwrites out (the caller recomputes it afterwards).
void lt_select(CliqueMixer &m, LtGemm &g, bool transpose, int kmul, int cols, const void *A, const void *B,
               float *out, hipStream_t st) {
  const int64_t N = m.N, K = kmul * N;
  ltchk(hipblasLtMatmulDescCreate(&g.desc, HIPBLAS_COMPUTE_32F, HIP_R_32F), "matmul desc");
  const int32_t opA = transpose ? HIPBLAS_OP_T : HIPBLAS_OP_N, opB = HIPBLAS_OP_N;
  ltchk(hipblasLtMatmulDescSetAttribute(g.desc, HIPBLASLT_MATMUL_DESC_TRANSA, &opA, sizeof(opA)), "transA");
  ltchk(hipblasLtMatmulDescSetAttribute(g.desc, HIPBLASLT_MATMUL_DESC_TRANSB, &opB, sizeof(opB)), "transB");
  if (transpose) ltchk(hipblasLtMatrixLayoutCreate(&g.a, HIP_R_16F, K, N, 2 * N), "layout A");
  else ltchk(hipblasLtMatrixLayoutCreate(&g.a, HIP_R_16F, N, K, N), "layout A");
  ltchk(hipblasLtMatrixLayoutCreate(&g.b, HIP_R_16F, K, cols, 2 * N), "layout B");
  ltchk(hipblasLtMatrixLayoutCreate(&g.c, HIP_R_32F, N, cols, N), "layout C");
  hipblasLtMatmulPreference_t pref = nullptr;
  ltchk(hipblasLtMatmulPreferenceCreate(&pref), "preference");
  const uint64_t wmax = LT_WORKSPACE;
  (void)hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wmax, sizeof(wmax));
  hipblasLtMatmulHeuristicResult_t res[16];
  int found = 0;
  hipblasStatus_t hs = hipblasLtMatmulAlgoGetHeuristic(m.lt, g.desc, g.a, g.b, g.c, g.c, pref, 16, res, &found);
  (void)hipblasLtMatmulPreferenceDestroy(pref);
  if (hs != HIPBLAS_STATUS_SUCCESS || found <= 0) return;
  void *ws = m.ltws.get(LT_WORKSPACE);
  hipEvent_t e0, e1;
  hipchk(hipEventCreate(&e0), "event");
  hipchk(hipEventCreate(&e1), "event");
  const float one = 1.0f;
  float best = 1e30f;
  for (int i = 0; i < found; i++) {
    if (res[i].state != HIPBLAS_STATUS_SUCCESS || res[i].workspaceSize > LT_WORKSPACE) continue;
    bool good = true;
    for (int r = 0; r < 4 && good; r++) {
      if (r == 1) (void)hipEventRecord(e0, st);
      good = hipblasLtMatmul(m.lt, g.desc, &one, A, g.a, B, g.b, &one, out, g.c, out, g.c, &res[i].algo, ws,
                             res[i].workspaceSize, st) == HIPBLAS_STATUS_SUCCESS;
    }
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) good = false;
    float ms = 0.f;
    if (good && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best) {
      best = ms;
      g.algo = res[i].algo;
      g.ws = res[i].workspaceSize;
      g.ok = true;
    }
  }
  (void)hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <typename R>
struct Dense {
  CliqueMixer &m;
  hipStream_t st;
  int64_t N;
  int cols;  // 2S

  LtGemm *gemm(bool transpose, int kmul, const void *A, const void *B, float *out) {
    auto key = std::make_tuple(transpose ? 1 : 0, kmul, cols);
    auto it = m.gemms.find(key);
    if (it != m.gemms.end()) return it->second.get();
    auto g = std::make_unique<LtGemm>();
    lt_select(m, *g, transpose, kmul, cols, A, B, out, st);
    LtGemm *p = g.get();
    m.gemms[key] = std::move(g);
    return p;
  }

  // out (N x cols) = op(V) in (next-product input B), op = V^T (transpose) or V
  void product(bool transpose, const void *B, R *out) {
    const rocblas_int n = (rocblas_int)N, c = cols;
    blaschk(rocblas_set_stream(m.blas, st), "rocblas_set_stream");
    LtGemm *l1 = nullptr, *l2 = nullptr;
    if constexpr (sizeof(R) == 4) {
      // algorithm selection runs before the timed product (it overwrites out)
      const __half *A = transpose ? (const __half *)m.Vrows.p : (const __half *)m.Vcols.p;
      if (!m.lt) ltchk(hipblasLtCreate(&m.lt), "hipblasLtCreate");
      l1 = gemm(transpose, 1, A, (const __half *)B + N, (float *)out);
      l2 = gemm(transpose, 2, A, B, (float *)out);
    }
    if (m.timer.begin) m.timer.begin(m.timer.ctx, st);
    double flops;
    if constexpr (sizeof(R) == 4) {
      const float one = 1.0f, zero = 0.0f, s11 = 1.0f / 2048.0f;
      const __half *b = (const __half *)B;
      const rocblas_operation op = transpose ? rocblas_operation_transpose : rocblas_operation_none;
      const __half *A = transpose ? (const __half *)m.Vrows.p : (const __half *)m.Vcols.p;
      const rocblas_int lda = transpose ? 2 * n : n;
      void *ws = m.ltws.p;
      if (l1->ok)
        ltchk(hipblasLtMatmul(m.lt, l1->desc, &one, A, l1->a, b + N, l1->b, &zero, out, l1->c, out, l1->c,
                              &l1->algo, ws, l1->ws, st),
              "hipblasLtMatmul (hi x hi)");
      else
        blaschk(rocblas_gemm_ex(m.blas, op, rocblas_operation_none, n, c, n, &one, A, rocblas_datatype_f16_r, lda,
                                b + N, rocblas_datatype_f16_r, 2 * n, &zero, out, rocblas_datatype_f32_r, n, out,
                                rocblas_datatype_f32_r, n, rocblas_datatype_f32_r, rocblas_gemm_algo_standard, 0, 0),
                "rocblas_gemm_ex (hi x hi)");
      if (l2->ok)
        ltchk(hipblasLtMatmul(m.lt, l2->desc, &s11, A, l2->a, b, l2->b, &one, out, l2->c, out, l2->c, &l2->algo,
                              ws, l2->ws, st),
              "hipblasLtMatmul (hi x lo + lo x hi)");
      else
        blaschk(rocblas_gemm_ex(m.blas, op, rocblas_operation_none, n, c, 2 * n, &s11, A, rocblas_datatype_f16_r,
                                lda, b, rocblas_datatype_f16_r, 2 * n, &one, out, rocblas_datatype_f32_r, n, out,
                                rocblas_datatype_f32_r, n, rocblas_datatype_f32_r, rocblas_gemm_algo_standard, 0, 0),
                "rocblas_gemm_ex (hi x lo + lo x hi)");
      flops = 3.0 * 2.0 * (double)N * N * cols;
    } else {
      const double one = 1.0, zero = 0.0;
      blaschk(rocblas_dgemm(m.blas, transpose ? rocblas_operation_transpose : rocblas_operation_none,
                            rocblas_operation_none, n, c, n, &one, (const double *)m.V.p, n, (const double *)B, n,
                            &zero, out, n),
              "rocblas_dgemm");
      flops = 2.0 * (double)N * N * cols;
    }
    // algorithmic work of one real N x N x cols product (the three half products are the
    // cost of the FP32 form, not the algorithm)
    if (m.timer.end) m.timer.end(m.timer.ctx, st, QAOA_KC_DENSE, 0.0, 2.0 * (double)N * N * cols);
    (void)flops;
  }
};

template <typename R, typename TT>
void run_clique(CliqueMixer &m, const CliqueEval &ev, int p, const double *angles, int S, const void *d_psi0,
                int grad, double *out_expect, double *out_grad, void *d_state, hipStream_t st) {
  using T2 = typename CT<R>::T2;
  const int64_t N = m.N;
  const int cols = 2 * S;
  const size_t mat = (size_t)N * cols * sizeof(R);
  R *X = (R *)m.X.get(mat);
  R *Y = (R *)m.Y.get(mat);
  void *B = m.B.get(sizeof(R) == 4 ? (size_t)2 * N * cols * sizeof(__half) : mat);
  R *ckP = grad ? (R *)m.ckP.get(mat * p) : nullptr;
  R *ckT = grad ? (R *)m.ckT.get(mat * p) : nullptr;
  const int nblk = (int)((N + RB_ROWS - 1) / RB_ROWS);
  const int nout = 2 + 2 * p;
  double *part = (double *)m.partials.get((size_t)nout * S * nblk * sizeof(double));
  auto pslot = [&](int o) { return part + (size_t)o * S * nblk; };
  // parameters: betas [p][S], LUT jobs (forward, inverse) [2p][S], contribution counts
  std::vector<double> betas((size_t)p * S);
  std::vector<LutJob> jobs((size_t)2 * p * S);
  for (int s = 0; s < S; s++)
    for (int k = 0; k < p; k++) {
      betas[(size_t)k * S + s] = angles[(size_t)s * 2 * p + k];
      const double g = angles[(size_t)s * 2 * p + p + k];
      jobs[(size_t)k * S + s] = LutJob{g, 1.0, 0.0, -1.0};
      jobs[(size_t)(p + k) * S + s] = LutJob{g, 1.0, 0.0, 1.0};
    }
  std::vector<int> cnt(nout, 1);
  const size_t b_bytes = betas.size() * sizeof(double), j_bytes = jobs.size() * sizeof(LutJob);
  const size_t off_j = (b_bytes + 255) & ~size_t(255), off_c = (off_j + j_bytes + 255) & ~size_t(255);
  const size_t total = off_c + nout * sizeof(int);
  std::vector<unsigned char> h(total);
  std::memcpy(h.data(), betas.data(), b_bytes);
  std::memcpy(h.data() + off_j, jobs.data(), j_bytes);
  std::memcpy(h.data() + off_c, cnt.data(), nout * sizeof(int));
  unsigned char *d = (unsigned char *)m.params.get(total);
  hipchk(hipMemcpyAsync(d, h.data(), total, hipMemcpyHostToDevice, st), "parameter upload");
  const double *dbeta = (const double *)d;
  T2 *dluts = (T2 *)m.luts.get(jobs.size() * (size_t)ev.lut_len * sizeof(T2));
  hipchk(launch_luts(sizeof(R) == 4 ? 0 : 1, (const LutJob *)(d + off_j), (int)jobs.size(), ev.lut_len, ev.vals,
                     dluts, st),
         "LUTs");
  auto lut_f = [&](int k) { return dluts + (size_t)k * S * ev.lut_len; };
  auto lut_b = [&](int k) { return dluts + (size_t)(p + k) * S * ev.lut_len; };

  Dense<R> dense{m, st, N, cols};
  const dim3 eg((unsigned)((N + 255) / 256 < 1024 ? (N + 255) / 256 : 1024), (unsigned)S);
  const dim3 rg((unsigned)nblk, (unsigned)S);
  auto launched = [&](const char *w) { hipchk(hipGetLastError(), w); };
  auto tbegin = [&]() {
    if (m.timer.begin) m.timer.begin(m.timer.ctx, st);
  };
  auto tend = [&](double bytes) {
    if (m.timer.end) m.timer.end(m.timer.ctx, st, QAOA_KC_OTHER, bytes, 0.0);
  };

  // forward sweep
  tbegin();
  k_init<R><<<eg, 256, 0, st>>>(X, N, d_psi0);
  launched("k_init");
  tend((double)mat);
  for (int k = 0; k < p; k++) {
    tbegin();
    k_phase<R, TT><<<eg, 256, 0, st>>>(X, N, ev.table, lut_f(k), ev.lut_len, grad ? ckP + (size_t)k * N * cols : nullptr, B);
    launched("k_phase");
    tend((double)mat * (grad ? 3 : 2));
    dense.product(true, B, Y);
    tbegin();
    k_eig<R><<<rg, 256, 0, st>>>(Y, N, m.D.p ? (const double *)m.D.p : nullptr, dbeta + (size_t)k * S, -1.0, nullptr,
                                 grad ? ckT + (size_t)k * N * cols : nullptr, B, nullptr, nblk);
    launched("k_eig");
    tend((double)mat * (grad ? 3 : 2));
    dense.product(false, B, X);
  }
  tbegin();
  k_expect<R, TT><<<rg, 256, 0, st>>>(X, N, ev.table, ev.vals, pslot(0), pslot(1), nblk);
  launched("k_expect");
  tend((double)mat);
  if (d_state) {
    k_export<R><<<eg.x, 256, 0, st>>>(X, N, (T2 *)d_state);
    launched("k_export");
  }
  // reverse sweep (only the adjoint vector is multiplied; phi comes from the forward keeps)
  if (grad) {
    k_lambda<R, TT><<<eg, 256, 0, st>>>(X, N, ev.table, ev.vals, ev.c0, B);
    launched("k_lambda");
    for (int k = p - 1; k >= 0; k--) {
      dense.product(true, B, Y);
      tbegin();
      k_eig<R><<<rg, 256, 0, st>>>(Y, N, (const double *)m.D.p, dbeta + (size_t)k * S, 1.0,
                                   ckT + (size_t)k * N * cols, nullptr, B, pslot(2 + k), nblk);
      launched("k_eig");
      tend((double)mat * 3);
      dense.product(false, B, X);
      tbegin();
      k_gamma<R, TT><<<rg, 256, 0, st>>>(X, N, ev.table, ev.vals, ev.c0, ckP + (size_t)k * N * cols, lut_b(k), ev.lut_len,
                                         k > 0 ? B : nullptr, pslot(2 + p + k), nblk);
      launched("k_gamma");
      tend((double)mat * 3);
    }
  }
  // fixed-order reduction of the partials: out[s][o]
  double *dres = (double *)m.results.get((size_t)S * nout * sizeof(double));
  hipchk(launch_finalize(part, (const int *)(d + off_c), 1, S, nblk, nout, dres, st), "finalize");
  m.hres.resize((size_t)S * nout);
  hipchk(hipMemcpyAsync(m.hres.data(), dres, (size_t)S * nout * sizeof(double), hipMemcpyDeviceToHost, st),
         "result download");
  hipchk(hipStreamSynchronize(st), "constrained evaluation");
  for (int s = 0; s < S; s++) {
    const double *r = m.hres.data() + (size_t)s * nout;
    const double E = r[0], Nr = r[1];
    if (out_expect) out_expect[s] = E / Nr;
    if (grad && out_grad)
      for (int k = 0; k < 2 * p; k++) out_grad[(size_t)s * 2 * p + k] = 2.0 * r[2 + k] / Nr;
  }
}

}  // namespace

void clique_evaluate(CliqueMixer &m, const CliqueEval &ev, int p, const double *angles, int nsets,
                     const void *d_psi0, int precision, int grad, double *out_expect, double *out_grad,
                     void *d_state, hipStream_t st) {
  if (ev.N != m.N) throw CliqueError{QAOA_ERR_INVALID_ARG, "problem size differs from the mixer's subspace"};
  if (d_state && nsets != 1) throw CliqueError{QAOA_ERR_INVALID_ARG, "state output needs one angle set"};
  if (precision == QAOA_FP32) {
    if (ev.tbytes == 1) run_clique<float, uint8_t>(m, ev, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
    else run_clique<float, uint16_t>(m, ev, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
  } else {
    if (ev.tbytes == 1) run_clique<double, uint8_t>(m, ev, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
    else run_clique<double, uint16_t>(m, ev, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
  }
}

}  // namespace qaoa
