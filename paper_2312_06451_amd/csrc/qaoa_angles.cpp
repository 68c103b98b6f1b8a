// Angle-finding outer loop (Sec. 2.3; the find_angles calls of Sec. 3): BFGS local
// minimisation, basinhopping, iterative p-1 -> p seeding with a per-round checkpoint file, and
// the random local-minima search. Host code above the evaluation entry points: every
// objective value and gradient comes from one qaoa_expect_grad_pairs call per step, with all
// restarts or chains of that step, of every instance being solved, as its pairs, so the device
// sees one large launch per optimiser step instead of one small evaluation per start.
//
// Algorithms (the paper names them and leaves their details open):
//  * BFGS in inverse-Hessian form (Nocedal and Wright, Numerical Optimization, Alg. 6.1 and
//    Eq. 6.17), H_0 = I rescaled to (s.y / y.y) I before the first update (their Eq. 6.20),
//    updates skipped when s.y <= 1e-10 |s| |y|; backtracking line search by halving (their
//    Alg. 3.1) that accepts on sufficient decrease (c1 = 1e-4) or on the approximate Wolfe
//    conditions (sigma = 0.9, delta = 0.1, eps = 1e-6); first trial step min(1, 1 / max|d|)
//    along the direction d, so no angle moves more than one radian in a trial (the landscape
//    repeats, and an uncapped quasi-Newton step can jump by thousands of radians); 20
//    halvings without acceptance end the minimisation; converged when
//    max|g| <= gtol max(1, |f|).
//  * Basinhopping (Wales and Doye, J. Phys. Chem. A 101, 5111 (1997)): minimise, perturb every
//    angle by a uniform draw in [-step, step], minimise, accept by the Metropolis rule
//    exp(-(f_new - f_cur) / T).
//  * Round seeding: the round r-1 optimum padded with a zero layer (the identity, so the same
//    <C>) and its linear interpolation to r layers (the INTERP rule of Zhou, Wang, Choi,
//    Pichler and Lukin, Phys. Rev. X 10, 021067 (2020)).
//  * Random draws: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a counter-based
//    generator: the j-th draw of key (round, chain, hop) is the j-th output of the SplitMix64
//    sequence whose state starts at seed XOR mix(round << 48 | chain << 32 | (hop + 1) << 16).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include "../../include/qaoa.h"

namespace qaoa {
void set_last_error(const char *msg);
}

namespace {

struct Fail {
  int code;
  std::string msg;
};

#define NEED(cond, msg)                                                                       \
  do {                                                                                        \
    if (!(cond)) throw Fail{QAOA_ERR_INVALID_ARG, msg};                                       \
  } while (0)

// A failed evaluation call: its status and message are already in place.
struct Passed {
  int code;
};

template <typename F>
int guarded(F &&f) {
  try {
    f();
    qaoa::set_last_error("");
    return QAOA_OK;
  } catch (const Fail &e) {
    qaoa::set_last_error(e.msg.c_str());
    return e.code;
  } catch (const Passed &e) {
    return e.code;
  } catch (const std::bad_alloc &) {
    qaoa::set_last_error("host allocation failed");
    return QAOA_ERR_OUT_OF_MEMORY;
  } catch (...) {
    qaoa::set_last_error("unexpected exception");
    return QAOA_ERR_HIP;
  }
}

// ---------------------------------------------------------------- random draws

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Uniform in [0, 1): draw j of key (round, chain, hop), hop >= -1.
double uniform(uint64_t seed, int round, int chain, int hop, int j) {
  const uint64_t key = ((uint64_t)round << 48) | ((uint64_t)chain << 32) | ((uint64_t)(hop + 1) << 16);
  const uint64_t state = seed ^ mix64(key);
  return (double)(mix64(state + (uint64_t)(j + 1) * kGolden) >> 11) * 0x1.0p-53;
}

constexpr double kTwoPi = 6.283185307179586476925286766559;

// ---------------------------------------------------------------- objective

struct Objective {
  std::vector<const qaoa_problem *> probs;  // one per instance
  std::vector<const qaoa_mixer *> mixes;
  int p;
  int precision;
  double sign;  // f = sign * <C> is minimised
  void *stream;
  int chunk;
  std::vector<const qaoa_problem *> pp;
  std::vector<const qaoa_mixer *> pm;
  std::vector<double> ebuf, gbuf;

  Objective(const qaoa_problem *const *pr, const qaoa_mixer *const *mx, int n_inst, int p_, const qaoa_angle_opts &o,
            void *st)
      : probs(pr, pr + n_inst), mixes(mx, mx + n_inst), p(p_), precision(o.precision),
        sign(o.maximize ? -1.0 : 1.0), stream(st) {
    int64_t big = 1;
    for (int i = 0; i < n_inst; i++) {
      int64_t size = 0;
      int rc = qaoa_problem_info(probs[i], nullptr, nullptr, &size, nullptr);
      if (rc != QAOA_OK) throw Passed{rc};
      big = std::max(big, size);
      int apl = 0;
      rc = qaoa_mixer_info(mixes[i], nullptr, nullptr, &apl);
      if (rc != QAOA_OK) throw Passed{rc};
      if (apl != 2) throw Fail{QAOA_ERR_UNSUPPORTED, "angle finding takes mixers with one angle per layer"};
    }
    if (o.max_sets_per_call > 0) {
      chunk = o.max_sets_per_call;
    } else {
      const double per_set = 2.0 * (double)big * 16.0;
      chunk = (int)std::max(1.0, std::min(65536.0, std::floor(4294967296.0 / per_set)));
    }
  }

  // points xs[m][2p], point i of instance owner[i] -> f[m], g[m][2p] (derivatives of f)
  void eval(int m, const int *owner, const double *xs, double *f, double *g) {
    const int D = 2 * p;
    for (int i0 = 0; i0 < m; i0 += chunk) {
      const int c = std::min(chunk, m - i0);
      ebuf.resize(c);
      gbuf.resize((size_t)c * D);
      pp.resize(c);
      pm.resize(c);
      for (int i = 0; i < c; i++) {
        pp[i] = probs[owner[i0 + i]];
        pm[i] = mixes[owner[i0 + i]];
      }
      const int rc = qaoa_expect_grad_pairs(pp.data(), pm.data(), c, p, xs + (size_t)i0 * D, precision, ebuf.data(),
                                            gbuf.data(), stream);
      if (rc != QAOA_OK) throw Passed{rc};
      for (int i = 0; i < c; i++) {
        f[i0 + i] = sign * ebuf[i];
        for (int j = 0; j < D; j++) g[(size_t)(i0 + i) * D + j] = sign * gbuf[(size_t)i * D + j];
      }
    }
  }
};

// ---------------------------------------------------------------- BFGS, many starts at once

double maxabs(const double *v, int D) {
  double m = 0.0;
  for (int i = 0; i < D; i++) m = std::max(m, std::fabs(v[i]));
  return m;
}

double dot(const double *a, const double *b, int D) {
  double s = 0.0;
  for (int i = 0; i < D; i++) s += a[i] * b[i];
  return s;
}

struct Run {
  std::vector<double> x, g, H, d, xt;
  std::vector<double> s, y, Hy;  // scratch of the update, allocated once per run
  double f = 0.0, gd = 0.0, alpha = 1.0;
  int iters = 0, halvings = 0, owner = 0;
  bool unscaled = true;  // H = I, not yet rescaled by a first update
  bool init = true;      // xt is the starting point, not yet evaluated
  bool done = false;
};

constexpr double kArmijo = 1e-4;  // sufficient decrease
constexpr double kSigma = 0.9;    // approximate Wolfe: slope no steeper than sigma times the first
constexpr double kDelta = 0.1;    // approximate Wolfe: slope no larger than (1 - 2 delta) |first|
constexpr double kEps = 1e-6;     // approximate Wolfe: f may rise by eps |f|
constexpr int kMaxHalvings = 20;

void set_identity(Run &r, int D) {
  std::fill(r.H.begin(), r.H.end(), 0.0);
  for (int i = 0; i < D; i++) r.H[(size_t)i * D + i] = 1.0;
  r.unscaled = true;
}

void start_run(Run &r, int owner, const double *x0, int D) {
  r.x.assign(D, 0.0);
  r.g.assign(D, 0.0);
  r.d.assign(D, 0.0);
  r.H.assign((size_t)D * D, 0.0);
  r.xt.assign(x0, x0 + D);
  r.s.assign(D, 0.0);
  r.y.assign(D, 0.0);
  r.Hy.assign(D, 0.0);
  r.f = r.gd = 0.0;
  r.alpha = 1.0;
  r.iters = r.halvings = 0;
  r.owner = owner;
  r.init = true;
  r.done = false;
  set_identity(r, D);
}

bool converged(const Run &r, const qaoa_angle_opts &o, int D) {
  return maxabs(r.g.data(), D) <= o.gtol * std::max(1.0, std::fabs(r.f));
}

// Search direction from the current (x, g, H); ends the run when g vanishes.
void new_direction(Run &r, int D) {
  for (int i = 0; i < D; i++) {
    double s = 0.0;
    for (int j = 0; j < D; j++) s -= r.H[(size_t)i * D + j] * r.g[j];
    r.d[i] = s;
  }
  r.gd = dot(r.g.data(), r.d.data(), D);
  if (!(r.gd < 0.0)) {  // not a descent direction: restart from steepest descent
    set_identity(r, D);
    for (int i = 0; i < D; i++) r.d[i] = -r.g[i];
    r.gd = dot(r.g.data(), r.d.data(), D);
    if (!(r.gd < 0.0)) {
      r.done = true;
      return;
    }
  }
  r.alpha = std::min(1.0, 1.0 / maxabs(r.d.data(), D));  // no angle moves more than one radian
  r.halvings = 0;
  for (int i = 0; i < D; i++) r.xt[i] = r.x[i] + r.alpha * r.d[i];
}

// Inverse-Hessian update with s = x_new - x, y = g_new - g (both already formed).
void bfgs_update(Run &r, const double *s, const double *y, int D) {
  const double sy = dot(s, y, D);
  const double ns = std::sqrt(dot(s, s, D)), ny = std::sqrt(dot(y, y, D));
  if (!(sy > 1e-10 * ns * ny)) return;
  if (r.unscaled) {
    const double scale = sy / dot(y, y, D);
    std::fill(r.H.begin(), r.H.end(), 0.0);
    for (int i = 0; i < D; i++) r.H[(size_t)i * D + i] = scale;
    r.unscaled = false;
  }
  // H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, expanded with Hy = H y (H symmetric)
  const double rho = 1.0 / sy;
  double *Hy = r.Hy.data();
  for (int i = 0; i < D; i++) Hy[i] = dot(&r.H[(size_t)i * D], y, D);
  const double yHy = dot(y, Hy, D);
  const double c = rho * rho * yHy + rho;
  for (int i = 0; i < D; i++)
    for (int j = 0; j < D; j++)
      r.H[(size_t)i * D + j] += -rho * (s[i] * Hy[j] + Hy[i] * s[j]) + c * s[i] * s[j];
}

// Consume the evaluation (ft, gt) of r.xt: the start point, or a line-search trial. A trial
// is accepted on sufficient decrease (Armijo) or on the approximate Wolfe conditions of Hager
// and Zhang (SIAM J. Optim. 16, 170 (2005)), which judge the step by the slope at the trial
// point: with single-precision evaluations the change of f near an optimum drops below the
// rounding of f while the gradient is still accurate.
void advance(Run &r, double ft, const double *gt, int D, const qaoa_angle_opts &o) {
  if (r.init) {
    r.init = false;
    std::copy(r.xt.begin(), r.xt.end(), r.x.begin());
    r.f = ft;
    std::copy(gt, gt + D, r.g.begin());
    if (!std::isfinite(r.f) || converged(r, o, D) || o.max_iter <= 0) r.done = true;
    else new_direction(r, D);
    return;
  }
  bool accept = false;
  if (std::isfinite(ft)) {
    const double slope = dot(gt, r.d.data(), D);
    accept = ft <= r.f + kArmijo * r.alpha * r.gd ||
             (ft <= r.f + kEps * std::fabs(r.f) && slope >= kSigma * r.gd && slope <= (2.0 * kDelta - 1.0) * r.gd);
  }
  if (accept) {
    double *s = r.s.data(), *y = r.y.data();
    for (int j = 0; j < D; j++) {
      s[j] = r.xt[j] - r.x[j];
      y[j] = gt[j] - r.g[j];
    }
    bfgs_update(r, s, y, D);
    std::copy(r.xt.begin(), r.xt.end(), r.x.begin());
    r.f = ft;
    std::copy(gt, gt + D, r.g.begin());
    r.iters++;
    if (converged(r, o, D) || r.iters >= o.max_iter) r.done = true;
    else new_direction(r, D);
  } else {
    r.alpha *= 0.5;
    if (++r.halvings > kMaxHalvings) r.done = true;
    else
      for (int j = 0; j < D; j++) r.xt[j] = r.x[j] + r.alpha * r.d[j];
  }
}

// Evaluate every live run's pending point in one paired call and advance each run.
struct Stepper {
  std::vector<double> pts, fv, gv;
  std::vector<int> own;
  void operator()(Objective &obj, const std::vector<Run *> &live, const qaoa_angle_opts &o) {
    const int D = 2 * obj.p, L = (int)live.size();
    pts.resize((size_t)L * D);
    gv.resize((size_t)L * D);
    fv.resize(L);
    own.resize(L);
    for (int a = 0; a < L; a++) {
      std::memcpy(&pts[(size_t)a * D], live[a]->xt.data(), D * sizeof(double));
      own[a] = live[a]->owner;
    }
    obj.eval(L, own.data(), pts.data(), fv.data(), gv.data());
    // the runs are independent: their O(D^2) updates on the host cores
#pragma omp parallel for schedule(static) if (L >= 32)
    for (int a = 0; a < L; a++) advance(*live[a], fv[a], &gv[(size_t)a * D], D, o);
  }
};

// Minimise from m starts (xs, in place; start i belongs to instance owner[i]) -> f[m]
// (objective f), iters[m]. Every step evaluates all unfinished runs together.
void minimize_many(Objective &obj, int m, const int *owner, double *xs, double *fout, int *iters,
                   const qaoa_angle_opts &o) {
  const int D = 2 * obj.p;
  std::vector<Run> runs(m);
  for (int i = 0; i < m; i++) start_run(runs[i], owner[i], xs + (size_t)i * D, D);
  std::vector<Run *> live;
  Stepper step;
  for (;;) {
    live.clear();
    for (auto &r : runs)
      if (!r.done) live.push_back(&r);
    if (live.empty()) break;
    step(obj, live, o);
  }
  for (int i = 0; i < m; i++) {
    std::memcpy(xs + (size_t)i * D, runs[i].x.data(), D * sizeof(double));
    fout[i] = runs[i].f;
    if (iters) iters[i] = runs[i].iters;
  }
}

// ---------------------------------------------------------------- basinhopping

// Basinhopping for n_inst instances at once: chain c of instance i starts at
// seeds[(i * C + c) * 2p ..]; instance i's best optimum -> best_x[i * 2p ..], best_f[i]
// (objective f), ties to the earliest hop, then the lowest chain. Chains run independently:
// a chain starts its next hop as soon as its minimisation ends, and every step evaluates the
// pending points of all chains together. Draws depend on (round, c, hop) only, so a chain's
// path, and an instance's result, do not depend on the other chains or instances.
void basinhop(Objective &obj, int round, int n_inst, const double *seeds, const qaoa_angle_opts &o, double *best_x,
              double *best_f) {
  const int D = 2 * obj.p, C = o.n_chains, m = n_inst * C;
  struct Chain {
    Run run;
    std::vector<double> cur, bx;
    double fcur = 0.0, bf = 0.0;
    int hop = -1, bh = -1;
    bool finished = false;
  };
  std::vector<Chain> ch(m);
  for (int i = 0; i < m; i++) start_run(ch[i].run, i / C, seeds + (size_t)i * D, D);
  std::vector<Run *> live;
  std::vector<double> xt(D);
  Stepper step;
  for (;;) {
    live.clear();
    for (auto &c : ch)
      if (!c.finished) live.push_back(&c.run);
    if (live.empty()) break;
    step(obj, live, o);
    for (int i = 0; i < m; i++) {
      Chain &c = ch[i];
      if (c.finished || !c.run.done) continue;
      const int cc = i % C;
      if (c.hop < 0) {
        c.cur = c.run.x;
        c.fcur = c.run.f;
        c.bx = c.cur;
        c.bf = c.fcur;
      } else {
        const double ft = c.run.f, df = ft - c.fcur;
        bool accept = ft < c.fcur;
        if (!accept && o.temperature > 0.0 && std::isfinite(df))
          accept = uniform(o.seed, round, cc, c.hop, D) < std::exp(-df / o.temperature);
        if (ft < c.bf) {
          c.bf = ft;
          c.bh = c.hop;
          c.bx = c.run.x;
        }
        if (accept) {
          c.cur = c.run.x;
          c.fcur = ft;
        }
      }
      if (++c.hop < o.n_hops) {
        for (int j = 0; j < D; j++) xt[j] = c.cur[j] + o.step * (2.0 * uniform(o.seed, round, cc, c.hop, j) - 1.0);
        start_run(c.run, i / C, xt.data(), D);
      } else {
        c.finished = true;
      }
    }
  }
  for (int i = 0; i < n_inst; i++) {
    int b = i * C;
    for (int c = i * C + 1; c < (i + 1) * C; c++)
      if (ch[c].bf < ch[b].bf || (ch[c].bf == ch[b].bf && ch[c].bh < ch[b].bh)) b = c;
    std::memcpy(best_x + (size_t)i * D, ch[b].bx.data(), D * sizeof(double));
    best_f[i] = ch[b].bf;
  }
}

// ---------------------------------------------------------------- checks

void check_opts(const qaoa_angle_opts &o) {
  NEED(o.precision == QAOA_FP32 || o.precision == QAOA_FP64, "precision must be QAOA_FP32 or QAOA_FP64");
  NEED(o.max_iter >= 0, "max_iter must be >= 0");
  NEED(std::isfinite(o.gtol) && o.gtol >= 0.0, "gtol must be finite and >= 0");
  NEED(o.n_chains >= 1 && o.n_chains <= 65535, "n_chains must be in [1, 65535]");
  NEED(o.n_hops >= 0 && o.n_hops <= 65534, "n_hops must be in [0, 65534]");
  NEED(std::isfinite(o.step) && o.step >= 0.0, "step must be finite and >= 0");
  NEED(std::isfinite(o.temperature) && o.temperature >= 0.0, "temperature must be finite and >= 0");
  NEED(o.max_sets_per_call >= 0, "max_sets_per_call must be >= 0");
}

qaoa_angle_opts opts_or_default(const qaoa_angle_opts *o) {
  qaoa_angle_opts d;
  qaoa_angle_opts_default(&d);
  return o ? *o : d;
}

void check_points(const double *x, size_t count) {
  NEED(x != nullptr, "angles are NULL");
  for (size_t i = 0; i < count; i++) NEED(std::isfinite(x[i]), "angles must be finite");
}

// ---------------------------------------------------------------- round seeding

// INTERP: a_1..a_q -> b_1..b_{q+1}, b_i = ((i-1)/q) a_{i-1} + ((q-i+1)/q) a_i, a_0 = a_{q+1} = 0
void interp(const double *a, int q, double *b) {
  for (int i = 1; i <= q + 1; i++) {
    const double lo = i >= 2 ? a[i - 2] : 0.0;
    const double hi = i <= q ? a[i - 1] : 0.0;
    b[i - 1] = ((double)(i - 1) / q) * lo + ((double)(q - i + 1) / q) * hi;
  }
}

// ---------------------------------------------------------------- checkpoint file

struct Header {
  int n = 0, k = 0, maximize = 0;
  int64_t size = 0;
  uint64_t hash = 0;
};

Header header_of(const qaoa_problem *prob, int maximize, void *stream) {
  Header h;
  int rc = qaoa_problem_info(prob, &h.n, &h.k, &h.size, nullptr);
  if (rc != QAOA_OK) throw Passed{rc};
  h.maximize = maximize ? 1 : 0;
  if (h.size <= (int64_t(1) << 24)) {  // FNV-1a over the value table's bytes
    std::vector<double> v((size_t)h.size);
    rc = qaoa_problem_copy_values(prob, v.data(), v.size(), stream);
    if (rc != QAOA_OK) throw Passed{rc};
    uint64_t x = 0xcbf29ce484222325ull;
    const unsigned char *b = (const unsigned char *)v.data();
    for (size_t i = 0; i < v.size() * sizeof(double); i++) x = (x ^ b[i]) * 0x100000001b3ull;
    h.hash = x;
  }
  return h;
}

std::string header_line(const Header &h) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "qaoa-angles 1 n %d hamming_k %d size %lld maximize %d values %016llx", h.n, h.k,
                (long long)h.size, h.maximize, (unsigned long long)h.hash);
  return buf;
}

// Rounds stored in `path` (empty if the file does not exist): angles[r-1] has 2r entries.
void load_checkpoint(const char *path, const Header &h, std::vector<std::vector<double>> &angles,
                     std::vector<double> &values) {
  std::ifstream in(path);
  if (!in.is_open()) {
    if (access(path, F_OK) == 0) throw Fail{QAOA_ERR_INVALID_ARG, "checkpoint file exists but cannot be read"};
    return;
  }
  std::string line;
  NEED(std::getline(in, line), "checkpoint file is empty");
  NEED(line == header_line(h), "checkpoint file belongs to another problem or objective sense");
  while (std::getline(in, line)) {
    if (line.empty()) continue;
    std::istringstream ss(line);
    std::string w1, w2, w3;
    int r = 0;
    std::string vtok;
    ss >> w1 >> r >> w2 >> vtok >> w3;
    NEED(w1 == "round" && w2 == "value" && w3 == "angles", "checkpoint file is malformed");
    NEED(r == (int)angles.size() + 1, "checkpoint rounds are not consecutive from 1");
    char *end = nullptr;
    const double v = std::strtod(vtok.c_str(), &end);
    NEED(end && *end == 0 && std::isfinite(v), "checkpoint value is malformed");
    std::vector<double> a;
    std::string tok;
    while (ss >> tok) {
      const double x = std::strtod(tok.c_str(), &end);
      NEED(end && *end == 0 && std::isfinite(x), "checkpoint angle is malformed");
      a.push_back(x);
    }
    NEED((int)a.size() == 2 * r, "checkpoint round has the wrong number of angles");
    angles.push_back(a);
    values.push_back(v);
  }
}

void save_checkpoint(const char *path, const Header &h, const std::vector<std::vector<double>> &angles,
                     const std::vector<double> &values) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) throw Fail{QAOA_ERR_INVALID_ARG, "cannot write the checkpoint file " + tmp};
  bool ok = std::fprintf(f, "%s\n", header_line(h).c_str()) > 0;
  for (size_t r = 0; r < angles.size() && ok; r++) {
    ok = std::fprintf(f, "round %zu value %.17g angles", r + 1, values[r]) > 0;
    for (double a : angles[r]) ok = ok && std::fprintf(f, " %.17g", a) > 0;
    ok = ok && std::fprintf(f, "\n") > 0;
  }
  ok = ok && std::fflush(f) == 0 && fsync(fileno(f)) == 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0)
    throw Fail{QAOA_ERR_INVALID_ARG, std::string("cannot write the checkpoint file ") + path};
}

}  // namespace

extern "C" {

void qaoa_angle_opts_default(qaoa_angle_opts *o) {
  if (!o) return;
  o->maximize = 1;
  o->precision = QAOA_FP32;
  o->max_iter = 100;
  o->gtol = 1e-5;
  o->n_chains = 8;
  o->n_hops = 10;
  o->step = 0.5;
  o->temperature = 1.0;
  o->seed = 0;
  o->max_sets_per_call = 0;
}

int qaoa_minimize(const qaoa_problem *prob, const qaoa_mixer *mix, int p, int n_starts, double *angles,
                  double *out_values, int *out_iters, const qaoa_angle_opts *opts, void *stream) {
  return guarded([&] {
    const qaoa_angle_opts o = opts_or_default(opts);
    check_opts(o);
    NEED(p >= 1 && p <= 4096, "p must be in [1, 4096]");
    NEED(n_starts >= 1, "n_starts must be >= 1");
    NEED(out_values != nullptr, "out_values is NULL");
    check_points(angles, (size_t)n_starts * 2 * p);
    Objective obj(&prob, &mix, 1, p, o, stream);
    std::vector<int> owner(n_starts, 0);
    minimize_many(obj, n_starts, owner.data(), angles, out_values, out_iters, o);
    for (int i = 0; i < n_starts; i++) out_values[i] *= obj.sign;
  });
}

int qaoa_basinhopping(const qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *x0,
                      const qaoa_angle_opts *opts, double *out_angles, double *out_value, void *stream) {
  return guarded([&] {
    const qaoa_angle_opts o = opts_or_default(opts);
    check_opts(o);
    NEED(p >= 1 && p <= 4096, "p must be in [1, 4096]");
    NEED(out_angles && out_value, "out_angles or out_value is NULL");
    check_points(x0, 2 * (size_t)p);
    const int D = 2 * p;
    std::vector<double> seeds((size_t)o.n_chains * D);
    for (int c = 0; c < o.n_chains; c++) std::memcpy(&seeds[(size_t)c * D], x0, D * sizeof(double));
    Objective obj(&prob, &mix, 1, p, o, stream);
    double bf = 0.0;
    basinhop(obj, p, 1, seeds.data(), o, out_angles, &bf);
    *out_value = obj.sign * bf;
  });
}

int qaoa_find_angles_multi(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_inst,
                           int p_max, const qaoa_angle_opts *opts, const char *const *checkpoint_paths,
                           double *out_angles, double *out_values, void *stream) {
  return guarded([&] {
    const qaoa_angle_opts o = opts_or_default(opts);
    check_opts(o);
    NEED(probs && mixers, "probs or mixers is NULL");
    NEED(n_inst >= 1, "n_inst must be >= 1");
    NEED(p_max >= 1 && p_max <= 4096, "p_max must be in [1, 4096]");
    NEED(out_angles && out_values, "out_angles or out_values is NULL");
    std::vector<std::vector<std::vector<double>>> rounds(n_inst);
    std::vector<std::vector<double>> values(n_inst);
    std::vector<Header> hdr(n_inst);
    auto path = [&](int i) -> const char * { return checkpoint_paths ? checkpoint_paths[i] : nullptr; };
    for (int i = 0; i < n_inst; i++) {
      NEED(probs[i] && mixers[i], "a problem or mixer handle is NULL");
      if (path(i)) {
        hdr[i] = header_of(probs[i], o.maximize, stream);
        load_checkpoint(path(i), hdr[i], rounds[i], values[i]);
      }
    }
    int first = p_max + 1;
    for (int i = 0; i < n_inst; i++) first = std::min(first, (int)rounds[i].size() + 1);
    for (int r = first; r <= p_max; r++) {
      const int D = 2 * r, C = o.n_chains;
      std::vector<int> act;  // instances with exactly r - 1 rounds done
      for (int i = 0; i < n_inst; i++)
        if ((int)rounds[i].size() == r - 1) act.push_back(i);
      if (act.empty()) continue;
      const int A = (int)act.size();
      std::vector<double> seeds((size_t)A * C * D);
      for (int a = 0; a < A; a++) {
        double *sd = &seeds[(size_t)a * C * D];
        if (r == 1) {
          for (int c = 0; c < C; c++)
            for (int j = 0; j < D; j++) sd[(size_t)c * D + j] = kTwoPi * uniform(o.seed, 1, c, -1, j);
        } else {
          const std::vector<double> &prev = rounds[act[a]][r - 2];  // beta_1..beta_{r-1}, gamma_1..gamma_{r-1}
          const int q = r - 1;
          std::vector<double> pad(D, 0.0), itp(D);
          for (int t = 0; t < q; t++) {
            pad[t] = prev[t];
            pad[r + t] = prev[q + t];
          }
          interp(prev.data(), q, itp.data());
          interp(prev.data() + q, q, itp.data() + r);
          for (int c = 0; c < C; c++)
            std::memcpy(sd + (size_t)c * D, c == 0 ? pad.data() : itp.data(), D * sizeof(double));
        }
      }
      std::vector<const qaoa_problem *> ap(A);
      std::vector<const qaoa_mixer *> am(A);
      for (int a = 0; a < A; a++) {
        ap[a] = probs[act[a]];
        am[a] = mixers[act[a]];
      }
      Objective obj(ap.data(), am.data(), A, r, o, stream);
      std::vector<double> bx((size_t)A * D), bf(A);
      basinhop(obj, r, A, seeds.data(), o, bx.data(), bf.data());
      for (int a = 0; a < A; a++) {
        const int i = act[a];
        rounds[i].emplace_back(bx.begin() + (size_t)a * D, bx.begin() + (size_t)(a + 1) * D);
        values[i].push_back(obj.sign * bf[a]);
        if (path(i)) save_checkpoint(path(i), hdr[i], rounds[i], values[i]);
      }
    }
    const size_t row = (size_t)2 * p_max;
    std::fill(out_angles, out_angles + (size_t)n_inst * p_max * row, 0.0);
    for (int i = 0; i < n_inst; i++)
      for (int r = 1; r <= p_max; r++) {
        std::memcpy(out_angles + ((size_t)i * p_max + (r - 1)) * row, rounds[i][r - 1].data(), 2 * r * sizeof(double));
        out_values[(size_t)i * p_max + (r - 1)] = values[i][r - 1];
      }
  });
}

int qaoa_find_angles(const qaoa_problem *prob, const qaoa_mixer *mix, int p_max, const qaoa_angle_opts *opts,
                     const char *checkpoint_path, double *out_angles, double *out_values, void *stream) {
  return qaoa_find_angles_multi(&prob, &mix, 1, p_max, opts, &checkpoint_path, out_angles, out_values, stream);
}

int qaoa_find_angles_random(const qaoa_problem *prob, const qaoa_mixer *mix, int p, int n_restarts,
                            const qaoa_angle_opts *opts, double *out_angles, double *out_value,
                            double *out_all_values, void *stream) {
  return guarded([&] {
    const qaoa_angle_opts o = opts_or_default(opts);
    check_opts(o);
    NEED(p >= 1 && p <= 4096, "p must be in [1, 4096]");
    NEED(n_restarts >= 1 && n_restarts <= 65535, "n_restarts must be in [1, 65535]");
    NEED(out_angles && out_value, "out_angles or out_value is NULL");
    const int D = 2 * p;
    std::vector<double> xs((size_t)n_restarts * D), f(n_restarts);
    for (int i = 0; i < n_restarts; i++)
      for (int j = 0; j < D; j++) xs[(size_t)i * D + j] = kTwoPi * uniform(o.seed, p, i, -1, j);
    Objective obj(&prob, &mix, 1, p, o, stream);
    std::vector<int> owner(n_restarts, 0);
    minimize_many(obj, n_restarts, owner.data(), xs.data(), f.data(), nullptr, o);
    int bi = 0;
    for (int i = 1; i < n_restarts; i++)
      if (f[i] < f[bi]) bi = i;
    std::memcpy(out_angles, &xs[(size_t)bi * D], D * sizeof(double));
    *out_value = obj.sign * f[bi];
    if (out_all_values)
      for (int i = 0; i < n_restarts; i++) out_all_values[i] = obj.sign * f[i];
  });
}

}  // extern "C"
