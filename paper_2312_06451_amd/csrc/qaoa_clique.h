// Constrained (clique-mixer) path: H_M = V D V^T on the Hamming-weight-k subspace, applied as
// two dense products per round (Sec. 2.1 and Sec. 2.2 of the paper).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <memory>

namespace qaoa {

struct CliqueMixer;  // eigenbasis and workspaces (qaoa_clique.hip)
struct CliqueMixerDeleter {
  void operator()(CliqueMixer *m) const;
};

struct CliqueUnsupported {};

struct CliqueEval {
  const void *table;
  int tbytes;
  int64_t N;
  int lut_len;
  double c0;
};

std::unique_ptr<CliqueMixer, CliqueMixerDeleter> clique_create(int n, int k, hipStream_t st);
void clique_evaluate(CliqueMixer &m, const CliqueEval &ev, int p, const double *angles, int nsets,
                     const void *d_psi0, int precision, int grad, double *out_expect,
                     double *out_grad, void *d_state, hipStream_t st);

}  // namespace qaoa
