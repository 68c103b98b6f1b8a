// Constrained (clique-mixer) path. Not yet built: every entry reports UNSUPPORTED.
#include "qaoa_clique.h"
#include <stdexcept>
#include <string>

namespace qaoa {

struct CliqueMixer {
  int n = 0, k = 0;
};

void CliqueMixerDeleter::operator()(CliqueMixer *m) const { delete m; }

std::unique_ptr<CliqueMixer, CliqueMixerDeleter> clique_create(int, int, hipStream_t) {
  throw CliqueUnsupported{};
}

void clique_evaluate(CliqueMixer &, const CliqueEval &, int, const double *, int, const void *,
                     int, int, double *, double *, void *, hipStream_t) {
  throw CliqueUnsupported{};
}

}  // namespace qaoa
