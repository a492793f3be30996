// Fitting loops on the batched chi^2 and its adjoint: a particle swarm whose
// particles are one batched likelihood launch per step, and L-BFGS chains
// from several starts whose trial points are one batched gradient launch
// per round.  Host double precision for the optimiser state.
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "jt_host.hpp"

using namespace jt;

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * kGamma;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform_at(uint64_t seed, uint64_t i) { return (double)(splitmix64_at(seed, i) >> 11) * 0x1p-53; }

int fit_params(const jt_fit_problem* p) { return 7 + 7 * (p->n_src + p->n_ll); }

// The box must lie inside the domain every parameter accepts.
jt_status check_problem(const jt_grid* grid, const jt_fit_problem* p, bool grad) {
  if (!grid || !p) return fail(JT_EINVAL, "fit: null argument");
  if (p->n_src < 0 || p->n_ll < 0 || p->n_src + p->n_ll < 1) return fail(JT_EINVAL, "fit: no light component");
  if (p->n_src > JT_MAX_SERSIC || p->n_ll > JT_MAX_SERSIC) return fail(JT_EUNSUPPORTED, "fit: too many components");
  if (grad && p->n_src + p->n_ll > 3) return fail(JT_EUNSUPPORTED, "fit: gradient takes at most 3 components");
  if (!p->lower || !p->upper || !p->data || !p->inv_var) return fail(JT_EINVAL, "fit: null bounds, data or weights");
  if (p->n_sub < 0 || (p->n_sub > 0 && (!p->sub_x || !p->sub_y || !p->sub_Rs || !p->sub_alpha_Rs)))
    return fail(JT_EINVAL, "fit: bad subhalo arrays");
  if ((p->psf == nullptr) != (p->k == 0)) return fail(JT_EINVAL, "fit: psf and k must be given together");
  const int P = fit_params(p);
  for (int i = 0; i < P; ++i) {
    const double lo = p->lower[i], hi = p->upper[i];
    if (!std::isfinite(lo) || !std::isfinite(hi) || lo > hi) return fail(JT_EINVAL, "fit: bad box in parameter %d", i);
    bool ok = true;
    if (i == 0) ok = lo >= 0.0;                                  // theta_E
    else if (i == 1) ok = lo > 0.0 && hi <= 1.0;                 // SIE q
    else if (i >= 7) {
      const int f = (i - 7) % 7;
      if (f == 1) ok = lo > 0.0;                                 // R_sersic
      else if (f == 2) ok = lo >= 0.2 && hi <= 10.0;             // n_sersic
      else if (f == 3) ok = lo > 0.0 && hi <= 1.0;               // q
    }
    if (!ok) return fail(JT_EINVAL, "fit: box of parameter %d outside its domain", i);
  }
  return JT_OK;
}

// Device buffers of one fitting run (allocated per call, freed on return).
struct FitBuffers {
  float *sx = nullptr, *sy = nullptr, *srs = nullptr, *sars = nullptr, *gm = nullptr, *gs = nullptr;
  double* logL = nullptr;
  ~FitBuffers() {
    for (void* q : {(void*)sx, (void*)sy, (void*)srs, (void*)sars, (void*)gm, (void*)gs, (void*)logL})
      if (q) (void)hipFree(q);
  }
};

// Batched evaluation of B parameter vectors (rows of X): log L, and with
// grad the gradient of log L [B][P].
struct Evaluator {
  jt_ctx* ctx;
  const jt_grid* grid;
  const jt_fit_problem* p;
  hipStream_t st;
  int Bmax, P;
  FitBuffers buf;
  std::vector<jt_sie> sie;
  std::vector<jt_shear> shear;
  std::vector<jt_sersic> src, ll;
  std::vector<float> gm_host;

  jt_status init(bool grad) {
    const size_t n = (size_t)p->n_sub;
    if (n > 0) {
      const size_t bytes = sizeof(float) * Bmax * n;
      float** dst[4] = {&buf.sx, &buf.sy, &buf.srs, &buf.sars};
      const float* srcp[4] = {p->sub_x, p->sub_y, p->sub_Rs, p->sub_alpha_Rs};
      for (int a = 0; a < 4; ++a) {
        JT_TRY(check_hip(hipMalloc((void**)dst[a], bytes), "hipMalloc(fit subhalos)"));
        for (int b = 0; b < Bmax; ++b)
          JT_TRY(check_hip(hipMemcpyAsync(*dst[a] + b * n, srcp[a], sizeof(float) * n, hipMemcpyDeviceToDevice, st),
                           "hipMemcpyAsync(fit subhalos)"));
      }
      if (grad) JT_TRY(check_hip(hipMalloc((void**)&buf.gs, sizeof(float) * Bmax * n * 3), "hipMalloc(fit g_sub)"));
    }
    JT_TRY(check_hip(hipMalloc((void**)&buf.logL, sizeof(double) * Bmax), "hipMalloc(fit logL)"));
    if (grad) JT_TRY(check_hip(hipMalloc((void**)&buf.gm, sizeof(float) * Bmax * P), "hipMalloc(fit g_macro)"));
    sie.resize(Bmax);
    shear.resize(Bmax);
    src.resize((size_t)Bmax * std::max(p->n_src, 1));
    ll.resize((size_t)Bmax * std::max(p->n_ll, 1));
    gm_host.resize((size_t)Bmax * P);
    return JT_OK;
  }

  jt_status run(int B, const double* X, double* logL, double* G) {
    for (int b = 0; b < B; ++b) {
      const double* x = X + (size_t)b * P;
      sie[b] = jt_sie{x[0], x[1], x[2], x[3], x[4]};
      shear[b] = jt_shear{x[5], x[6]};
      for (int c = 0; c < p->n_src + p->n_ll; ++c) {
        const double* q = x + 7 + 7 * c;
        const jt_sersic s{q[0], q[1], q[2], q[3], q[4], q[5], q[6]};
        if (c < p->n_src) src[(size_t)b * p->n_src + c] = s;
        else ll[(size_t)b * p->n_ll + (c - p->n_src)] = s;
      }
    }
    jt_draws d;
    std::memset(&d, 0, sizeof(d));
    d.B = B;
    d.sie = sie.data();
    d.shear = shear.data();
    d.n_sub = p->n_sub;
    d.sub_x = buf.sx;
    d.sub_y = buf.sy;
    d.sub_Rs = buf.srs;
    d.sub_alpha_Rs = buf.sars;
    d.n_src = p->n_src;
    d.n_ll = p->n_ll;
    d.src = p->n_src ? src.data() : nullptr;
    d.ll = p->n_ll ? ll.data() : nullptr;
    if (G) {
      JT_TRY(jt_chi2_grad(ctx, grid, &d, p->psf, p->k, p->data, p->inv_var, buf.logL, buf.gm, buf.gs, st));
      JT_TRY(check_hip(hipMemcpyAsync(gm_host.data(), buf.gm, sizeof(float) * B * P, hipMemcpyDeviceToHost, st),
                       "hipMemcpyAsync(fit gradient)"));
    } else {
      JT_TRY(jt_chi2(ctx, grid, &d, p->psf, p->k, p->data, p->inv_var, buf.logL, st));
    }
    JT_TRY(check_hip(hipMemcpyAsync(logL, buf.logL, sizeof(double) * B, hipMemcpyDeviceToHost, st),
                     "hipMemcpyAsync(fit logL)"));
    JT_TRY(check_hip(hipStreamSynchronize(st), "fit sync"));
    if (G)
      for (size_t i = 0; i < (size_t)B * P; ++i) G[i] = gm_host[i];
    return JT_OK;
  }
};

double dot(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

double norm2(const double* a, int n) { return std::sqrt(dot(a, a, n)); }

}  // namespace

extern "C" double jt_uniform(uint64_t seed, uint64_t i) { return uniform_at(seed, i); }

extern "C" jt_status jt_pso_move(int N, int P, int t, uint64_t seed, double w, double c1, double c2,
                                 const double* lower, const double* upper, double* x, double* v,
                                 const double* pbest, const double* gbest) {
  if (N < 1 || P < 1 || t < 1) return fail(JT_EINVAL, "pso move: N = %d, P = %d, t = %d", N, P, t);
  if (!lower || !upper || !x || !v || !pbest || !gbest) return fail(JT_EINVAL, "pso move: null array");
  for (int p = 0; p < N; ++p)
    for (int d = 0; d < P; ++d) {
      const uint64_t base = (((uint64_t)t * N + p) * P + d) * 2;
      const double r0 = uniform_at(seed, base), r1 = uniform_at(seed, base + 1);
      const size_t i = (size_t)p * P + d;
      double vv = w * v[i] + c1 * r0 * (pbest[i] - x[i]) + c2 * r1 * (gbest[d] - x[i]);
      double xx = x[i] + vv;
      if (xx < lower[d]) {
        xx = lower[d];
        vv = 0.0;
      } else if (xx > upper[d]) {
        xx = upper[d];
        vv = 0.0;
      }
      x[i] = xx;
      v[i] = vv;
    }
  return JT_OK;
}

extern "C" jt_status jt_pso(jt_ctx* ctx, const jt_grid* grid, const jt_fit_problem* prob, const jt_pso_cfg* cfg,
                            double* best, double* best_logL, double* history, hipStream_t stream) {
  JT_TRY(ctx_enter(ctx));
  JT_TRY(check_problem(grid, prob, false));
  if (!cfg || !best || !best_logL) return fail(JT_EINVAL, "pso: null argument");
  if (cfg->n_particles < 1 || cfg->n_iterations < 0)
    return fail(JT_EINVAL, "pso: %d particles, %d steps", cfg->n_particles, cfg->n_iterations);
  const int N = cfg->n_particles, P = fit_params(prob);
  Evaluator ev{ctx, grid, prob, stream, N, P};
  JT_TRY(ev.init(false));
  std::vector<double> x((size_t)N * P), v((size_t)N * P, 0.0), pb, pbf(N), f(N), gb(P);
  for (int p = 0; p < N; ++p)
    for (int d = 0; d < P; ++d)
      x[(size_t)p * P + d] = prob->lower[d] + uniform_at(cfg->seed, (uint64_t)p * P + d) * (prob->upper[d] - prob->lower[d]);
  const double ninf = -std::numeric_limits<double>::infinity();
  auto update = [&](bool first) {
    for (int p = 0; p < N; ++p) {
      const double fp = std::isnan(f[p]) ? ninf : f[p];
      if (first || fp > pbf[p]) {
        pbf[p] = fp;
        std::memcpy(&pb[(size_t)p * P], &x[(size_t)p * P], sizeof(double) * P);
      }
    }
    int g = 0;
    for (int p = 1; p < N; ++p)
      if (pbf[p] > pbf[g]) g = p;
    std::memcpy(gb.data(), &pb[(size_t)g * P], sizeof(double) * P);
    return pbf[g];
  };
  pb = x;
  JT_TRY(ev.run(N, x.data(), f.data(), nullptr));
  double gbf = update(true);
  for (int t = 1; t <= cfg->n_iterations; ++t) {
    JT_TRY(jt_pso_move(N, P, t, cfg->seed, cfg->inertia, cfg->c_cognitive, cfg->c_social, prob->lower, prob->upper,
                       x.data(), v.data(), pb.data(), gb.data()));
    JT_TRY(ev.run(N, x.data(), f.data(), nullptr));
    gbf = update(false);
    if (history) history[t - 1] = gbf;
  }
  std::memcpy(best, gb.data(), sizeof(double) * P);
  *best_logL = gbf;
  return JT_OK;
}

namespace {
// One L-BFGS chain; the rounds of jt_lbfgs advance every chain by one
// evaluation, which keeps each chain's sequence that of a single run.
struct Chain {
  std::vector<double> x, g, d, xt, gt;
  std::vector<std::vector<double>> S, Y;
  double f = 0.0, ft = 0.0, step = 1.0;
  int it = 0, halvings = 0;
  bool done = false, in_search = false;
};
}  // namespace

extern "C" jt_status jt_lbfgs(jt_ctx* ctx, const jt_grid* grid, const jt_fit_problem* prob, const jt_lbfgs_cfg* cfg,
                              const double* x0, double* x_out, double* logL_out, int* iterations, hipStream_t stream) {
  JT_TRY(ctx_enter(ctx));
  JT_TRY(check_problem(grid, prob, true));
  if (!cfg || !x0 || !x_out || !logL_out) return fail(JT_EINVAL, "lbfgs: null argument");
  if (cfg->starts < 1 || cfg->memory < 1 || cfg->max_iter < 0)
    return fail(JT_EINVAL, "lbfgs: %d starts, memory %d, %d steps", cfg->starts, cfg->memory, cfg->max_iter);
  const int C = cfg->starts, P = fit_params(prob);
  const double* lo = prob->lower;
  const double* hi = prob->upper;
  Evaluator ev{ctx, grid, prob, stream, C, P};
  JT_TRY(ev.init(true));
  auto clampv = [&](std::vector<double>& v) {
    for (int i = 0; i < P; ++i) v[i] = std::min(std::max(v[i], lo[i]), hi[i]);
  };
  std::vector<Chain> ch(C);
  std::vector<double> X((size_t)C * P), L(C), G((size_t)C * P);
  for (int c = 0; c < C; ++c) {
    ch[c].x.assign(x0 + (size_t)c * P, x0 + (size_t)(c + 1) * P);
    clampv(ch[c].x);
    std::memcpy(&X[(size_t)c * P], ch[c].x.data(), sizeof(double) * P);
  }
  JT_TRY(ev.run(C, X.data(), L.data(), G.data()));
  for (int c = 0; c < C; ++c) {
    ch[c].f = -L[c];
    ch[c].g.resize(P);
    for (int i = 0; i < P; ++i) ch[c].g[i] = -G[(size_t)c * P + i];
  }
  std::vector<int> act;
  for (;;) {
    act.clear();
    for (int c = 0; c < C; ++c) {
      Chain& h = ch[c];
      if (h.done) continue;
      if (h.in_search) {                    // the last trial was rejected: halve
        if (++h.halvings > 40) {
          h.done = true;
          continue;
        }
        h.step *= 0.5;
      } else {                              // a new direction from the accepted point
        if (h.it >= cfg->max_iter) {
          h.done = true;
          continue;
        }
        // coordinates on a bound whose gradient points out of the box are
        // held; the recursion runs on the free ones
        std::vector<double> m(P);
        double pgmax = 0.0;
        for (int i = 0; i < P; ++i) {
          const bool pinned = (h.x[i] <= lo[i] && h.g[i] > 0.0) || (h.x[i] >= hi[i] && h.g[i] < 0.0);
          m[i] = pinned ? 0.0 : 1.0;
          if (!pinned) pgmax = std::max(pgmax, std::fabs(h.g[i]));
        }
        if (pgmax <= cfg->gtol) {
          h.done = true;
          continue;
        }
        const size_t np_ = h.S.size();
        std::vector<std::vector<double>> Sf(np_, std::vector<double>(P)), Yf(np_, std::vector<double>(P));
        for (size_t k = 0; k < np_; ++k)
          for (int i = 0; i < P; ++i) {
            Sf[k][i] = m[i] * h.S[k][i];
            Yf[k][i] = m[i] * h.Y[k][i];
          }
        std::vector<double> gf(P);
        for (int i = 0; i < P; ++i) gf[i] = m[i] * h.g[i];
        std::vector<double> q = gf;
        std::vector<double> alphas;
        for (int k = (int)np_ - 1; k >= 0; --k) {
          const double a = dot(Sf[k].data(), q.data(), P) / dot(Yf[k].data(), Sf[k].data(), P);
          for (int i = 0; i < P; ++i) q[i] -= a * Yf[k][i];
          alphas.push_back(a);
        }
        const double gnorm = norm2(gf.data(), P);
        if (np_ > 0) {
          const double sc = dot(Sf.back().data(), Yf.back().data(), P) / dot(Yf.back().data(), Yf.back().data(), P);
          for (double& e : q) e *= sc;
        } else {
          for (double& e : q) e /= gnorm;
        }
        for (size_t k = 0; k < np_; ++k) {
          const double a = alphas[np_ - 1 - k];
          const double b = dot(Yf[k].data(), q.data(), P) / dot(Yf[k].data(), Sf[k].data(), P);
          for (int i = 0; i < P; ++i) q[i] += Sf[k][i] * (a - b);
        }
        h.d.resize(P);
        for (int i = 0; i < P; ++i) h.d[i] = -q[i];
        if (!(dot(h.g.data(), h.d.data(), P) < 0.0)) {
          h.S.clear();
          h.Y.clear();
          for (int i = 0; i < P; ++i) h.d[i] = -gf[i] / gnorm;
        }
        h.step = 1.0;
        h.halvings = 0;
        h.in_search = true;
      }
      h.xt.resize(P);
      for (int i = 0; i < P; ++i) h.xt[i] = h.x[i] + h.step * h.d[i];
      clampv(h.xt);
      std::memcpy(&X[act.size() * P], h.xt.data(), sizeof(double) * P);
      act.push_back(c);
    }
    if (act.empty()) break;
    JT_TRY(ev.run((int)act.size(), X.data(), L.data(), G.data()));
    for (size_t a = 0; a < act.size(); ++a) {
      Chain& h = ch[act[a]];
      const double ft = -L[a];
      double slope = 0.0;
      for (int i = 0; i < P; ++i) slope += h.g[i] * (h.xt[i] - h.x[i]);
      if (!(ft <= h.f + 1e-4 * slope)) continue;          // rejected (NaN included): halve next round
      h.gt.resize(P);
      for (int i = 0; i < P; ++i) h.gt[i] = -G[a * P + i];
      std::vector<double> s(P), y(P);
      for (int i = 0; i < P; ++i) {
        s[i] = h.xt[i] - h.x[i];
        y[i] = h.gt[i] - h.g[i];
      }
      if (dot(s.data(), y.data(), P) > 1e-12 * norm2(s.data(), P) * norm2(y.data(), P)) {
        h.S.push_back(s);
        h.Y.push_back(y);
        if ((int)h.S.size() > cfg->memory) {
          h.S.erase(h.S.begin());
          h.Y.erase(h.Y.begin());
        }
      }
      ++h.it;
      const bool flat = std::fabs(h.f - ft) <= cfg->ftol * std::max(1.0, std::fabs(h.f));
      h.x = h.xt;
      h.f = ft;
      h.g = h.gt;
      h.in_search = false;
      if (flat) h.done = true;
    }
  }
  for (int c = 0; c < C; ++c) {
    std::memcpy(x_out + (size_t)c * P, ch[c].x.data(), sizeof(double) * P);
    logL_out[c] = -ch[c].f;
    if (iterations) iterations[c] = ch[c].it;
  }
  return JT_OK;
}
