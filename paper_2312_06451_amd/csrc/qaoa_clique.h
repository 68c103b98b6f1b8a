// Constrained (clique-mixer) path: H_M = V D V^T on the Hamming-weight-k subspace, applied as
// two dense products per round (Sec. 2.1 and Sec. 2.2 of the paper).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <memory>
#include <string>

namespace qaoa {

struct CliqueMixer;  // eigenbasis and workspaces (qaoa_clique.hip)
struct CliqueMixerDeleter {
  void operator()(CliqueMixer *m) const;
};

// Error raised by the constrained path (status code of include/qaoa.h and a message).
struct CliqueError {
  int code;
  std::string msg;
};

struct CliqueEval {
  const void *table;   // device table over the weight-k states (increasing order): value index
  const double *vals;  // device: cost value of each index (lut_len entries)
  int tbytes;
  int64_t N;
  int lut_len;         // number of indices
  double c0;           // mean of C over the states
};

// kind: MIX_CLIQUE, MIX_RING (matrices built on the device over the weight-k states),
// MIX_MATRIX (host_matrix: N x N real symmetric, N = 2^n for k < 0 else C(n, k)) or MIX_EIGEN
// (host_matrix: eigenvectors, column j at host_matrix[j * N ..], host_eigenvalues: N values).
enum { MIX_CLIQUE = 0, MIX_RING = 1, MIX_MATRIX = 2, MIX_EIGEN = 3 };
std::unique_ptr<CliqueMixer, CliqueMixerDeleter> clique_create(int kind, int n, int k, const double *host_matrix,
                                                                 const double *host_eigenvalues, hipStream_t st);
// Copy the FP64 eigenbasis (column j = eigenvector j) and eigenvalues to the host.
void clique_export(const CliqueMixer &m, double *host_V, double *host_D, hipStream_t st);
int64_t clique_size(const CliqueMixer &m);
void clique_evaluate(CliqueMixer &m, const CliqueEval &ev, int p, const double *angles, int nsets,
                     const void *d_psi0, int precision, int grad, double *out_expect,
                     double *out_grad, void *d_state, hipStream_t st);
// Kernel timing hook: (class, ms-start event, bytes, flops) recorder supplied by the caller.
struct CliqueTimer {
  void *ctx = nullptr;
  void (*begin)(void *ctx, hipStream_t st) = nullptr;
  void (*end)(void *ctx, hipStream_t st, int cls, double bytes, double flops) = nullptr;
};
void clique_set_timer(CliqueMixer &m, const CliqueTimer &t);

}  // namespace qaoa
