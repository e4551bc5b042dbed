// Host runtime of the C ABI (include/fa.h, include/fa_inspect.h): the pair
// object, its device buffers, the pyramid, the level/iteration driver of
// Algorithm 1 and the error reporting.  All device work is enqueued on the
// pair's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "fa.h"
#include "fa_batch.h"
#include "fa_host.h"
#include "fa_inspect.h"
#include "fa_inverse.h"
#include "fa_symmetric.h"
#include "fa_internal.h"

using fa::check_shape;
using fa::choose_tiling;
using fa::Ctl;
using fa::fail;
using fa::Tiling;
using fa::Tuning;
using fa::voxels;

namespace fa {

// Sampled Gaussian taps exp(-k^2 / 2 sigma^2), |k| <= ceil(3 sigma),
// normalised to sum 1 (computed in double).  sigma <= 0 gives the single tap 1.
std::vector<float> gaussian_taps(float sigma_f) {
  const double s = (double)sigma_f;
  if (!(s > 0.0)) return {1.0f};
  const int R = (int)std::ceil(3.0 * s);
  std::vector<double> w(2 * R + 1);
  double tot = 0.0;
  for (int k = -R; k <= R; ++k) {
    w[k + R] = std::exp(-(double)k * k / (2.0 * s * s));
    tot += w[k + R];
  }
  std::vector<float> out(w.size());
  for (size_t i = 0; i < w.size(); ++i) out[i] = (float)(w[i] / tot);
  return out;
}

int tap_radius(float sigma) { return (int)(gaussian_taps(sigma).size() / 2); }

fa_status check_params(const fa_params* p) {
  if (!p) return fail(FA_EINVAL, "params is NULL");
  if (!(p->eta > 0.0f) || !std::isfinite(p->eta)) return fail(FA_EINVAL, "eta must be a finite value > 0");
  if (p->cc_window < 1 || p->cc_window > fa::kMaxWindow || (p->cc_window % 2) == 0)
    return fail(FA_EINVAL, "cc_window must be odd and in [1, 9]");
  if (!(p->cc_eps >= 0.0f) || !std::isfinite(p->cc_eps)) return fail(FA_EINVAL, "cc_eps must be finite and >= 0");
  if (!(p->adam_beta1 >= 0.0f && p->adam_beta1 < 1.0f)) return fail(FA_EINVAL, "adam_beta1 must be in [0, 1)");
  if (!(p->adam_beta2 >= 0.0f && p->adam_beta2 < 1.0f)) return fail(FA_EINVAL, "adam_beta2 must be in [0, 1)");
  if (!(p->adam_eps >= 0.0f) || !std::isfinite(p->adam_eps)) return fail(FA_EINVAL, "adam_eps must be finite and >= 0");
  if (!std::isfinite(p->sigma_grad) || !std::isfinite(p->sigma_warp))
    return fail(FA_EINVAL, "sigma_grad and sigma_warp must be finite");
  if (tap_radius(p->sigma_grad) > fa::kMaxWideRadius || tap_radius(p->sigma_warp) > fa::kMaxWideRadius)
    return fail(FA_EINVAL, "Gaussian radius ceil(3 sigma) must be <= 24 (sigma <= 8 voxels)");
  if (p->use_jac != 0 && p->use_jac != 1) return fail(FA_EINVAL, "use_jac must be 0 or 1");
  return FA_OK;
}

fa_shape level_shape(const fa_shape& s, float scale) {
  const double sc = (double)scale;
  auto one = [&](int n) { return std::max(1, (int)std::floor((double)n / sc + 0.5)); };
  return fa_shape{one(s.n0), one(s.n1), one(s.n2)};
}

}  // namespace fa

using fa::check_params;
using fa::gaussian_taps;
using fa::level_shape;
using fa::tap_radius;

namespace {

thread_local std::string g_err;

struct Level {
  fa_shape shape{};
  int64_t n = 0;
  float scale = 1.0f;
  int iters = 0;
  float* fixed = nullptr;   // owned unless it aliases the input copy
  float* moving = nullptr;
  float* moving_pad = nullptr;  // moving with a zero border (owned), sampled by the gradient kernel
  float* moving_quad = nullptr; // the same as corner quads (owned; NULL where it would reach 4 GiB)
  bool owns = false;
  Tiling tg{}, tsg{}, tsc{}, tsw{};  // gradient, sigma_grad, composition and sigma_warp launches
  bool tuned[4] = {false, false, false, false};  // set by fa_pair_autotune (by KernelKind)
};

// Launch shapes chosen by fa_pair_autotune, per device, kernel kind, level
// grid and the parameter that selects the kernel's form (window, Gaussian
// radius, or whether the composition stages d in LDS).  Later schedules reuse
// them.
using TuneKey = std::tuple<int, int, int, int, int, int>;   // device, kind, n0, n1, n2, form
std::map<TuneKey, Tiling>& tune_cache() {
  static std::map<TuneKey, Tiling> m;
  return m;
}
std::mutex& tune_mutex() {
  static std::mutex mu;
  return mu;
}

}  // namespace

struct fa_pair_s {
  hipStream_t stream = nullptr;
  int device = 0;
  fa_shape shape{};
  int64_t n = 0;
  fa_params p{};
  float* in_fixed = nullptr;
  float* in_moving = nullptr;
  std::vector<Level> levels;
  int64_t cap = 0;            // voxels each state buffer can hold
  float* d = nullptr;         // state at the current level, SoA [3][n]
  float* m = nullptr;
  float* v = nullptr;
  float* a = nullptr;         // Adam direction
  float* tmp = nullptr;       // smoothed direction s, then the composed d'
  float* wide = nullptr;      // [3][cap] scratch of the smoothing passes with a radius above 6
  float* blur0 = nullptr;     // pyramid scratch (input size)
  float* blur1 = nullptr;
  Ctl* ctl = nullptr;
  float* loss_hist = nullptr;
  int loss_cap = 0;
  double* partials = nullptr;
  int partials_cap = 0;
  double* scratch = nullptr;  // kMeanBlocks + 1 doubles
  float* wts = nullptr;       // device tap tables
  std::vector<float> wts_host;
  std::vector<float> wts_dev;  // the table last copied to wts (empty: none)
  int rg = 0, rw = 0;         // Gaussian radii (sigma_grad, sigma_warp)
  int off_g = 0, off_w = 0;   // offsets of their taps in wts
  int off_one = 0;            // the single tap 1 (pointwise launches)
  std::vector<int> off_blur;  // per level, pyramid blur taps
  // kernel timing (fa_pair_profile)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  struct Pending { hipEvent_t e[5]; int level; };
  std::vector<Pending> pending;
  std::vector<double> prof_ms;   // [level][kind]
  std::vector<int> prof_n;
  Tuning tune[4];   // gradient, sigma_grad, sigma_warp and composition launches
  int cur_level = 0, cur_iter = 0;
  int t_done = 0;      // Adam steps taken (set_state may change it)
  int iters_done = 0;  // schedule iterations run = losses recorded
  bool scheduled = false;
  // the fixed image of every iteration instead of the level's own (a half of
  // the symmetric registration: the other half's warped image)
  const float* fixed_override = nullptr;
};

namespace {

// The parameter that selects kernel `kind`'s form (key of the tuned-shape cache).
int tune_form(const fa_pair P, int kind) {
  switch (kind) {
    case fa::KIND_GRAD: return P->p.cc_window;
    case fa::KIND_SMOOTH_MAX: return tap_radius(P->p.sigma_grad);
    case fa::KIND_WARP_SMOOTH: return tap_radius(P->p.sigma_warp);
    default: return P->p.eta <= 2.0f ? 1 : 0;
  }
}

void free_levels(fa_pair P) {
  for (auto& L : P->levels) {
    if (L.owns) {
      (void)hipFree(L.fixed);
      (void)hipFree(L.moving);
    }
    if (L.moving_pad) (void)hipFree(L.moving_pad);
    if (L.moving_quad) (void)hipFree(L.moving_quad);
  }
  P->levels.clear();
}

void free_all(fa_pair P) {
  free_levels(P);
  float* fbufs[] = {P->in_fixed, P->in_moving, P->d, P->m, P->v, P->a, P->tmp, P->wide, P->blur0,
                    P->blur1, P->loss_hist, P->wts};
  for (float* b : fbufs)
    if (b) (void)hipFree(b);
  if (P->ctl) (void)hipFree(P->ctl);
  if (P->partials) (void)hipFree(P->partials);
  if (P->scratch) (void)hipFree(P->scratch);
}

template <typename T>
fa_status dalloc(T** out, size_t count, const char* what) {
  *out = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)out, count * sizeof(T));
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(FA_ENOMEM, std::string("hipMalloc failed for ") + what + " (" +
                               std::to_string(count * sizeof(T)) + " bytes): " + hipGetErrorString(e));
  }
  return FA_OK;
}




// Blur (sigma = scale/2, replicate) then resample at corner-aligned positions.
fa_status build_level_image(fa_pair P, const float* src, float* dst, const Level& L, int off) {
  const fa_shape& s = P->shape;
  const int rad = tap_radius(L.scale / 2.0f);
  const float* w = P->wts + off;
  FA_HIP(fa::launch_blur_axis(src, P->blur0, s.n0, s.n1, s.n2, 0, w, rad, P->stream));
  FA_HIP(fa::launch_blur_axis(P->blur0, P->blur1, s.n0, s.n1, s.n2, 1, w, rad, P->stream));
  FA_HIP(fa::launch_blur_axis(P->blur1, P->blur0, s.n0, s.n1, s.n2, 2, w, rad, P->stream));
  FA_HIP(fa::launch_resample(P->blur0, dst, s.n0, s.n1, s.n2, L.shape.n0, L.shape.n1, L.shape.n2, 1,
                             1.0f, 1.0f, 1.0f, P->stream));
  return FA_OK;
}

fa_status get_event(fa_pair P, hipEvent_t* e) {
  if (!P->ev_pool.empty()) {
    *e = P->ev_pool.back();
    P->ev_pool.pop_back();
    return FA_OK;
  }
  FA_HIP(hipEventCreate(e));
  return FA_OK;
}

// Fold recorded event pairs into the per-level totals (synchronises).
fa_status drain_profile(fa_pair P) {
  if (P->pending.empty()) return FA_OK;
  FA_HIP(hipStreamSynchronize(P->stream));
  // launch order of an iteration, as kernel kinds (fa_pair_set_tuning's numbering)
  static const int kind_of_launch[4] = {fa::KIND_GRAD, fa::KIND_SMOOTH_MAX, fa::KIND_COMPOSE, fa::KIND_WARP_SMOOTH};
  for (auto& pe : P->pending) {
    for (int k = 0; k < 4; ++k) {
      float ms = 0.0f;
      FA_HIP(hipEventElapsedTime(&ms, pe.e[k], pe.e[k + 1]));
      const size_t slot = (size_t)pe.level * 4 + kind_of_launch[k];
      if (slot < P->prof_ms.size()) {
        P->prof_ms[slot] += ms;
        P->prof_n[slot] += 1;
      }
    }
    for (int k = 0; k < 5; ++k) P->ev_pool.push_back(pe.e[k]);
  }
  P->pending.clear();
  return FA_OK;
}

// The launches of one iteration of Algorithm 1 at level L: the fused
// gradient (+ Adam), s = G_sigma_grad * a with M = max |s|, the composition
// d' = u + d(x + u), and d = G_sigma_warp * d'.  One launch also records the
// loss from the gradient kernel's partials and advances t: the warp smoothing
// when it is a brick launch, else the composition.
struct IterPlan {
  fa::GradArgs ga;
  Tiling tg;
  int window;
  fa::GaussArgs g[3];
  Tiling tgs[3];
  int radius[3];
  int epi[3];
};

// fixed: the image the pair is registered to this iteration (NULL: the
// level's own fixed image; the symmetric registration passes the other
// half's warped image).
void plan_iteration(fa_pair P, const Level& L, IterPlan& it, const float* fixed = nullptr) {
  fa::GradArgs& ga = it.ga;
  ga = fa::GradArgs{};
  ga.fixed = fixed ? fixed : (P->fixed_override ? P->fixed_override : L.fixed);
  ga.moving_pad = L.moving_pad;
  ga.moving_quad = L.moving_quad;
  ga.d = P->d;
  ga.m = P->m;
  ga.v = P->v;
  ga.out = P->a;
  ga.partials = P->partials;
  ga.ctl = P->ctl;
  ga.n0 = L.shape.n0;
  ga.n1 = L.shape.n1;
  ga.n2 = L.shape.n2;
  ga.zc = L.tg.zc;
  ga.tiles_y = L.tg.tiles_y;
  ga.tiles_x = L.tg.tiles_x;
  ga.eps_cc = P->p.cc_eps;
  ga.beta1 = P->p.adam_beta1;
  ga.beta2 = P->p.adam_beta2;
  ga.adam_eps = P->p.adam_eps;
  ga.inv_n = (float)(1.0 / (double)L.n);
  // use_jac: the kernel writes the Gateaux gradient, and a second launch turns
  // it into the Eulerian direction and applies Adam
  ga.mode = P->p.use_jac ? 1 : 0;
  it.tg = L.tg;
  it.window = P->p.cc_window;

  fa::GaussArgs gs{};
  gs.ctl = P->ctl;
  gs.n0 = L.shape.n0;
  gs.n1 = L.shape.n1;
  gs.n2 = L.shape.n2;
  gs.eta = P->p.eta;
  gs.inv_n = (float)(1.0 / (double)L.n);

  fa::GaussArgs& g1 = it.g[0];  // s = G * a into tmp, M = max |s|
  g1 = gs;
  g1.in = P->a;
  g1.out = P->tmp;
  g1.wts = P->wts + P->off_g;
  g1.wide_tmp = P->wide;
  g1.zc = L.tsg.zc;
  g1.tiles_y = L.tsg.tiles_y;
  g1.tiles_x = L.tsg.tiles_x;
  it.tgs[0] = L.tsg;
  it.radius[0] = P->rg;
  it.epi[0] = fa::EPI_SMOOTH_MAX;

  // d' = u + d(x + u) with u = -eta s / (2M), in place over s: the single-tap
  // launch reads s only at the voxel it writes, one plane ahead
  fa::GaussArgs& g2 = it.g[1];
  g2 = gs;
  g2.in = P->tmp;
  g2.out = P->tmp;
  g2.d = P->d;
  g2.wts = P->wts + P->off_one;
  g2.zc = L.tsc.zc;
  g2.tiles_y = L.tsc.tiles_y;
  g2.tiles_x = L.tsc.tiles_x;
  it.tgs[1] = L.tsc;
  it.radius[1] = 0;
  // |u| <= eta / 2: with eta <= 2 the sample stays within one voxel, and d
  // is staged in LDS instead of gathered
  it.epi[1] = P->p.eta <= 2.0f ? fa::EPI_COMPOSE_LDS : fa::EPI_COMPOSE;

  fa::GaussArgs& g3 = it.g[2];  // d = G * d'
  g3 = gs;
  g3.in = P->tmp;
  g3.out = P->d;
  g3.wts = P->wts + P->off_w;
  g3.wide_tmp = P->wide;
  g3.zc = L.tsw.zc;
  g3.tiles_y = L.tsw.tiles_y;
  g3.tiles_x = L.tsw.tiles_x;
  it.tgs[2] = L.tsw;
  it.radius[2] = P->rw;
  it.epi[2] = fa::EPI_STORE;

  // the loss record and step count
  fa::GaussArgs& gr = it.g[record_launch(L.tsw)];
  gr.partials = P->partials;
  gr.n_partials = L.tg.blocks();
  gr.loss_hist = P->loss_hist;
  gr.loss_cap = P->loss_cap;
}

fa_status launch_eulerian(fa_pair P, const Level& L) {
  FA_HIP(fa::launch_eulerian_adam(P->a, P->d, P->m, P->v, P->ctl, L.shape.n0, L.shape.n1, L.shape.n2,
                                  P->p.adam_beta1, P->p.adam_beta2, P->p.adam_eps, P->stream));
  return FA_OK;
}

fa_status launch_iteration(fa_pair P, const Level& L, const float* fixed = nullptr) {
  fa_pair_s::Pending pe{};
  pe.level = P->cur_level;
  if (P->profiling) {
    for (int k = 0; k < 5; ++k) FA_TRY(get_event(P, &pe.e[k]));
    FA_HIP(hipEventRecord(pe.e[0], P->stream));
  }
  IterPlan it;
  plan_iteration(P, L, it, fixed);
  FA_HIP(fa::launch_grad(it.ga, it.window, it.tg, P->stream));
  if (P->p.use_jac) FA_TRY(launch_eulerian(P, L));
  if (P->profiling) FA_HIP(hipEventRecord(pe.e[1], P->stream));
  for (int k = 0; k < 3; ++k) {
    FA_HIP(fa::launch_gauss(it.g[k], it.radius[k], it.epi[k], it.tgs[k], P->stream));
    if (P->profiling) FA_HIP(hipEventRecord(pe.e[2 + k], P->stream));
  }
  if (P->profiling) {
    P->pending.push_back(pe);
    if (P->pending.size() >= 4096) FA_TRY(drain_profile(P));
  }
  return FA_OK;
}

// Carry d (rescaled to the new voxel units), m and v to the next level.
fa_status transition(fa_pair P) {
  const Level& C = P->levels[P->cur_level];
  const Level& F = P->levels[P->cur_level + 1];
  auto rho = [](int nf, int nc) { return nc > 1 ? (float)((double)(nf - 1) / (double)(nc - 1)) : 1.0f; };
  const float r0 = rho(F.shape.n0, C.shape.n0), r1 = rho(F.shape.n1, C.shape.n1), r2 = rho(F.shape.n2, C.shape.n2);
  const fa_shape& c = C.shape;
  const fa_shape& f = F.shape;
  FA_HIP(fa::launch_resample(P->d, P->tmp, c.n0, c.n1, c.n2, f.n0, f.n1, f.n2, 3, r0, r1, r2, P->stream));
  FA_HIP(fa::launch_resample(P->m, P->a, c.n0, c.n1, c.n2, f.n0, f.n1, f.n2, 3, 1.f, 1.f, 1.f, P->stream));
  // v's coarse data moves into the buffer that held m (already consumed).
  FA_HIP(fa::launch_resample(P->v, P->m, c.n0, c.n1, c.n2, f.n0, f.n1, f.n2, 3, 1.f, 1.f, 1.f, P->stream));
  float* old_d = P->d;
  float* old_m = P->m;
  float* old_v = P->v;
  float* old_a = P->a;
  float* old_t = P->tmp;
  P->d = old_t;
  P->m = old_a;
  P->v = old_m;
  P->a = old_d;
  P->tmp = old_v;
  return FA_OK;
}

// Advance past finished levels (upsampling at each boundary) while another
// level remains.
fa_status advance_levels(fa_pair P) {
  while (P->cur_level + 1 < (int)P->levels.size() && P->cur_iter >= P->levels[P->cur_level].iters) {
    FA_TRY(transition(P));
    P->cur_level += 1;
    P->cur_iter = 0;
  }
  return FA_OK;
}

bool schedule_done(const fa_pair P) {
  return P->cur_level == (int)P->levels.size() - 1 && P->cur_iter >= P->levels.back().iters;
}

// ---- batched launches -------------------------------------------------------
// One iteration of several pairs as one launch per kernel and launch form: the
// entries of a launch are the pairs whose kernel shares the template
// parameters (gradient: window and tiling form; smoothing and composition:
// radius, epilogue and tiling form).  The tables of all launches live in one
// device buffer, uploaded again only when the batch's composition changes (a
// level transition or a finished pair): every value that changes from one
// iteration to the next is in the pairs' control blocks on the device.
struct BatchLaunch {
  int stage;       // 0: gradient; 1, 2, 3: the three launches that follow it
  Tiling t;        // tile shape and form shared by the entries
  int param;       // window (stage 0) or Gaussian radius
  int epi;         // epilogue (stages 1 to 3)
  size_t ent_off;  // byte offsets of the entries and the owner array
  size_t own_off;
  int total;       // workgroups of the launch
  bool quad = false;   // gradient: the entries gather from corner quads
  bool adam = false;   // gradient: every entry runs mode 0 (gradient and Adam)
  // radius above 6: no batched form; each entry's launches run one after
  // another from these host-side arguments instead
  std::vector<fa::GaussArgs> singles;
  std::vector<Tiling> single_t;
};

struct BatchTables {
  std::vector<BatchLaunch> launches;
  std::vector<unsigned char> host;
  std::vector<int> jac;   // live pairs with use_jac (their Eulerian launch follows stage 0)
  void* dev = nullptr;
  size_t dev_cap = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <class Args>
void append_launch(BatchTables& bt, int stage, const Tiling& t, int param, int epi,
                   const std::vector<const Args*>& args, const std::vector<int>& nblocks) {
  using E = fa::BatchEntry<Args>;
  BatchLaunch bl{stage, t, param, epi, 0, 0, 0};
  for (int nb : nblocks) bl.total += nb;
  bl.ent_off = align256(bt.host.size());
  bl.own_off = align256(bl.ent_off + args.size() * sizeof(E));
  bt.host.resize(bl.own_off + (size_t)bl.total * sizeof(int));
  int first = 0;
  for (size_t e = 0; e < args.size(); ++e) {
    E en;
    en.a = *args[e];
    en.first = first;
    en.nblocks = nblocks[e];
    std::memcpy(bt.host.data() + bl.ent_off + e * sizeof(E), &en, sizeof(E));
    for (int k = 0; k < en.nblocks; ++k) {
      const int v = (int)e;
      std::memcpy(bt.host.data() + bl.own_off + (size_t)(first + k) * sizeof(int), &v, sizeof(int));
    }
    first += en.nblocks;
  }
  bt.launches.push_back(bl);
}

fa_status build_batch_tables(const std::vector<fa_pair>& live, BatchTables& bt) {
  bt.launches.clear();
  bt.host.clear();
  bt.jac.clear();
  const size_t n = live.size();
  std::vector<IterPlan> its(n);
  for (size_t i = 0; i < n; ++i) {
    plan_iteration(live[i], live[i]->levels[live[i]->cur_level], its[i]);
    if (live[i]->p.use_jac) bt.jac.push_back((int)i);
  }
  auto same_form = [](const Tiling& a, const Tiling& b) {
    return a.cube == b.cube && (a.cube || (a.ty == b.ty && a.tx == b.tx));
  };
  // stage 0: the gradient, grouped by window and tiling form
  std::vector<char> taken(n, 0);
  for (size_t i = 0; i < n; ++i) {
    if (taken[i]) continue;
    std::vector<size_t> mem;
    for (size_t j = i; j < n; ++j) {
      if (taken[j] || its[j].window != its[i].window || !same_form(its[j].tg, its[i].tg) ||
          (its[j].ga.moving_quad != nullptr) != (its[i].ga.moving_quad != nullptr) ||
          (its[j].ga.mode == 0) != (its[i].ga.mode == 0))
        continue;
      taken[j] = 1;
      mem.push_back(j);
    }
    if (!fa::grad_batch_supported(its[i].window, its[i].tg))
      return fail(FA_EINVAL, "no batched gradient launch for this window and tiling");
    std::vector<Tiling*> ts;
    std::vector<int> n0s;
    std::vector<char> pinned;
    for (size_t j : mem) {
      ts.push_back(&its[j].tg);
      n0s.push_back(its[j].ga.n0);
      // a chunk set by fa_pair_set_tuning is kept; an autotuned one is not:
      // it was timed with the GPU to one pair, and the entries of a batched
      // launch share the resident slots (the tuned tile shape and form stay)
      pinned.push_back(live[j]->tune[fa::KIND_GRAD].zc > 0);
    }
    std::vector<Tiling> orig;
    for (size_t j : mem) orig.push_back(its[j].tg);
    fa::batch_chunks(fa::KIND_GRAD, 4 * (its[i].window / 2), ts, n0s, pinned);
    std::vector<const fa::GradArgs*> args;
    std::vector<int> nb;
    for (size_t q = 0; q < mem.size(); ++q) {
      const size_t j = mem[q];
      // one loss partial per workgroup: stay within the pair's partials buffer
      if (its[j].tg.blocks() > live[j]->partials_cap) its[j].tg = orig[q];
      its[j].ga.zc = its[j].tg.zc;
      // the loss record sums every gradient workgroup
      its[j].g[record_launch(its[j].tgs[2])].n_partials = its[j].tg.blocks();
      args.push_back(&its[j].ga);
      nb.push_back(its[j].tg.blocks());
    }
    append_launch(bt, 0, its[i].tg, its[i].window, 0, args, nb);
    bt.launches.back().quad = its[i].ga.moving_quad != nullptr;
    bt.launches.back().adam = its[i].ga.mode == 0;
  }
  // stages 1 to 3, grouped by radius, epilogue and tiling form
  static const fa::KernelKind kinds[3] = {fa::KIND_SMOOTH_MAX, fa::KIND_COMPOSE, fa::KIND_WARP_SMOOTH};
  for (int k = 0; k < 3; ++k) {
    std::fill(taken.begin(), taken.end(), 0);
    for (size_t i = 0; i < n; ++i) {
      if (taken[i]) continue;
      std::vector<size_t> mem;
      for (size_t j = i; j < n; ++j) {
        if (taken[j] || its[j].radius[k] != its[i].radius[k] || its[j].epi[k] != its[i].epi[k] ||
            !same_form(its[j].tgs[k], its[i].tgs[k]))
          continue;
        taken[j] = 1;
        mem.push_back(j);
      }
      if (its[i].radius[k] > fa::kMaxRadius) {
        BatchLaunch bl{k + 1, its[i].tgs[k], its[i].radius[k], its[i].epi[k], 0, 0, 0};
        for (size_t j : mem) {
          bl.singles.push_back(its[j].g[k]);
          bl.single_t.push_back(its[j].tgs[k]);
        }
        bt.launches.push_back(std::move(bl));
        continue;
      }
      if (!fa::gauss_batch_supported(its[i].radius[k], its[i].epi[k], its[i].tgs[k]))
        return fail(FA_EINVAL, "no batched smoothing launch for this radius, epilogue and tiling");
      std::vector<Tiling*> ts;
      std::vector<int> n0s;
      std::vector<char> pinned;
      for (size_t j : mem) {
        ts.push_back(&its[j].tgs[k]);
        n0s.push_back(its[j].g[k].n0);
        pinned.push_back(live[j]->tune[kinds[k]].zc > 0);   // as for the gradient launch
      }
      // halo planes: 2R of the smoothing, one plane ahead for the composition
      fa::batch_chunks(kinds[k], k == 1 ? 2 : 2 * its[i].radius[k], ts, n0s, pinned);
      std::vector<const fa::GaussArgs*> args;
      std::vector<int> nb;
      for (size_t j : mem) {
        its[j].g[k].zc = its[j].tgs[k].zc;
        args.push_back(&its[j].g[k]);
        nb.push_back(its[j].tgs[k].blocks());
      }
      append_launch(bt, k + 1, its[i].tgs[k], its[i].radius[k], its[i].epi[k], args, nb);
    }
  }
  return FA_OK;
}

// Copies the host image to the device.  Synchronises: the launches already
// queued read the previous tables, and the host image may change after this.
fa_status upload_batch_tables(BatchTables& bt, hipStream_t s) {
  const size_t need = std::max<size_t>(bt.host.size(), 256);
  FA_HIP(hipStreamSynchronize(s));
  if (need > bt.dev_cap) {
    if (bt.dev) FA_HIP(hipFree(bt.dev));
    bt.dev = nullptr;
    bt.dev_cap = 0;
    FA_TRY(dalloc((unsigned char**)&bt.dev, need, "batch tables"));
    bt.dev_cap = need;
  }
  if (!bt.host.empty())
    FA_HIP(hipMemcpyAsync(bt.dev, bt.host.data(), bt.host.size(), hipMemcpyHostToDevice, s));
  FA_HIP(hipStreamSynchronize(s));
  return FA_OK;
}

fa_status launch_batch_iteration(const std::vector<fa_pair>& live, const BatchTables& bt, hipStream_t s) {
  const unsigned char* base = static_cast<const unsigned char*>(bt.dev);
  bool jac_done = false;
  for (const BatchLaunch& bl : bt.launches) {
    if (bl.stage >= 1 && !jac_done) {
      for (int j : bt.jac) FA_TRY(launch_eulerian(live[j], live[j]->levels[live[j]->cur_level]));
      jac_done = true;
    }
    if (!bl.singles.empty()) {
      for (size_t e = 0; e < bl.singles.size(); ++e)
        FA_HIP(fa::launch_gauss(bl.singles[e], bl.param, bl.epi, bl.single_t[e], s));
      continue;
    }
    const int* own = reinterpret_cast<const int*>(base + bl.own_off);
    if (bl.stage == 0) {
      const auto* E = reinterpret_cast<const fa::BatchEntry<fa::GradArgs>*>(base + bl.ent_off);
      FA_HIP(fa::launch_grad_batch(E, own, bl.total, bl.param, bl.t, bl.quad, bl.adam, s));
    } else {
      const auto* E = reinterpret_cast<const fa::BatchEntry<fa::GaussArgs>*>(base + bl.ent_off);
      FA_HIP(fa::launch_gauss_batch(E, own, bl.total, bl.param, bl.epi, bl.t, s));
    }
  }
  return FA_OK;
}

fa_status check_batch(fa_pair* pairs, int n, int max_iters) {
  if (n < 0 || (n > 0 && !pairs)) return fail(FA_EINVAL, "pairs is NULL or n < 0");
  if (max_iters < 0) return fail(FA_EINVAL, "max_iters must be >= 0");
  for (int i = 0; i < n; ++i) {
    if (!pairs[i]) return fail(FA_EINVAL, "pairs[" + std::to_string(i) + "] is NULL");
    if (!pairs[i]->scheduled) return fail(FA_ESTATE, "pairs[" + std::to_string(i) + "] has no schedule");
    for (int j = 0; j < i; ++j)
      if (pairs[j] == pairs[i]) return fail(FA_EINVAL, "a pair appears twice");
  }
  return FA_OK;
}

int count_finished(fa_pair* pairs, int n) {
  int f = 0;
  for (int i = 0; i < n; ++i) f += schedule_done(pairs[i]) ? 1 : 0;
  return f;
}

// Whether fa_batch_step_fused replays captured HIP graphs (fa_batch_use_graphs).
bool g_batch_graphs = false;

// The fused batch proper, with every pair's work on stream s.  With graphs:
// the first iteration of each batch composition runs eagerly, then its
// launches are captured once and the graph replays every later iteration
// until the composition changes (nothing in an iteration depends on host
// values that change between iterations).
fa_status run_batch_fused(fa_pair* pairs, int n, int max_iters, hipStream_t s) {
  BatchTables bt;
  hipGraphExec_t gexec = nullptr;
  bool capture_next = false;
  std::vector<char> alive(n, 1);
  std::vector<std::pair<int, int>> sig, last;
  std::vector<fa_pair> live;
  fa_status st = FA_OK;
  for (int k = 0; k < max_iters && st == FA_OK; ++k) {
    live.clear();
    sig.clear();
    for (int i = 0; i < n && st == FA_OK; ++i) {
      if (!alive[i]) continue;
      st = advance_levels(pairs[i]);
      if (st != FA_OK) break;
      if (schedule_done(pairs[i])) {
        alive[i] = 0;
        continue;
      }
      live.push_back(pairs[i]);
      sig.emplace_back(i, pairs[i]->cur_level);
    }
    if (st != FA_OK || live.empty()) break;
    if (sig != last) {
      if (gexec) {
        // the replays already queued use the old tables: upload_batch_tables synchronises first
        (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
      }
      if ((st = build_batch_tables(live, bt)) != FA_OK) break;
      if ((st = upload_batch_tables(bt, s)) != FA_OK) break;
      last = sig;
      capture_next = g_batch_graphs;
    }
    if (gexec) {
      const hipError_t he = hipGraphLaunch(gexec, s);
      if (he != hipSuccess) {
        st = fail(FA_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(he));
        break;
      }
    } else {
      if ((st = launch_batch_iteration(live, bt, s)) != FA_OK) break;
      if (capture_next) {
        capture_next = false;
        hipGraph_t graph = nullptr;
        hipError_t he = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (he == hipSuccess) {
          const fa_status cst = launch_batch_iteration(live, bt, s);
          he = hipStreamEndCapture(s, &graph);
          if (cst != FA_OK) {
            st = cst;
            if (graph) (void)hipGraphDestroy(graph);
            break;
          }
        }
        if (he == hipSuccess) he = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (he != hipSuccess) {
          gexec = nullptr;
          st = fail(FA_EHIP, std::string("capturing the batched iteration: ") + hipGetErrorString(he));
          break;
        }
      }
    }
    for (fa_pair P : live) {
      P->cur_iter += 1;
      P->t_done += 1;
      P->iters_done += 1;
    }
  }
  if (bt.dev) {
    // the queued launches read the tables
    const hipError_t e1 = hipStreamSynchronize(s);
    const hipError_t e2 = hipFree(bt.dev);
    if (st == FA_OK && e1 != hipSuccess) st = fail(FA_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e1));
    if (st == FA_OK && e2 != hipSuccess) st = fail(FA_EHIP, std::string("hipFree: ") + hipGetErrorString(e2));
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  return st;
}

}  // namespace

namespace fa {

fa_status fail(fa_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

fa_status check_shape(const fa_shape& s) {
  if (s.n0 < 2 || s.n1 < 2 || s.n2 < 2) return fail(FA_ESHAPE, "every dimension must be >= 2");
  // gathers address one volume with 32-bit signed byte offsets
  if ((double)s.n0 * s.n1 * s.n2 > 536870911.0)
    return fail(FA_ESHAPE, "volume too large: n0*n1*n2 must be < 2^29");
  // the gradient kernel addresses the padded moving image with 32-bit byte offsets
  if ((double)(s.n0 + 2 * kPad) * (s.n1 + 2 * kPad) * (s.n2 + 2 * kPad) > 1073741823.0)
    return fail(FA_ESHAPE, "volume too large: the padded volume (n+4 per axis) must hold < 2^30 voxels");
  return FA_OK;
}

// In-plane tile and n0 chunking of one streaming launch: 16x32 tiles (8x32
// when n1 is smaller) and the longest chunk that keeps the launch within a
// number of workgroups the GPU holds resident at once, so that no workgroup
// waits for another to finish, and at least a minimum chunk.  The gradient
// kernel holds two workgroups per CU (512 on 256 CUs); the sigma_grad
// smoothing kernel, with fewer registers, holds four.  The 2R-plane halos of
// the two smoothing kernels make chunks below 4 planes wasteful.  (Measured
// on the 160x192x224 pyramid: each level's time over chunks of 1 to 40
// planes.)
Tiling choose_tiling(const fa_shape& s, KernelKind kind, const Tuning& tu, bool cube_ok) {
  static const int kSlots[4] = {512, 1024, 512, 512};
  static const int kMinChunk[4] = {1, 4, 4, 1};
  // Small volumes take bricks: there a launch is bound by the length of its
  // chain of dependent steps, not by throughput.  (Measured at 40x48x56:
  // gradient 34.3 -> 22.5 us, sigma_grad smoothing 16.0 -> 11.9, composition
  // 7.3 -> 6.7, warp smoothing 14.0 -> 11.7; at 80x96x112 every brick form
  // loses to the march.)  Tuning variant: 1 forces the march, 2 (kinds 1 to
  // 3) or 3 (kind 0) the bricks.
  constexpr int64_t kCubeMaxVoxels = 300000;
  const int cube_variant = kind == KIND_GRAD ? 3 : 2;
  const bool cube = cube_ok && (tu.variant == cube_variant ||
                                (tu.variant == 0 && voxels(s) <= kCubeMaxVoxels));
  if (cube) {
    Tiling t;
    t.cube = true;
    t.ty = kCubeY;
    t.tx = kCubeX;
    t.zc = kCubeZ;
    t.tiles_y = (s.n1 + kCubeY - 1) / kCubeY;
    t.tiles_x = (s.n2 + kCubeX - 1) / kCubeX;
    t.chunks = (s.n0 + kCubeZ - 1) / kCubeZ;
    return t;
  }
  Tiling t;
  t.tx = 32;
  t.ty = s.n1 >= 16 ? 16 : 8;
  if (tu.ty > 0 && tu.tx > 0) {
    t.ty = tu.ty;
    t.tx = tu.tx;
  }
  t.variant = tu.variant;
  t.tiles_y = (s.n1 + t.ty - 1) / t.ty;
  t.tiles_x = (s.n2 + t.tx - 1) / t.tx;
  const int plane_tiles = t.tiles_y * t.tiles_x;
  int zc = (int)(((int64_t)s.n0 * plane_tiles + kSlots[kind] - 1) / kSlots[kind]);
  zc = std::max(zc, kMinChunk[kind]);
  if (tu.zc > 0) zc = tu.zc;
  zc = std::min(zc, s.n0);
  t.zc = zc;
  t.chunks = (s.n0 + zc - 1) / zc;
  return t;
}

// Chunk lengths along n0 for a batched march launch, whose entries share the
// GPU's resident workgroup slots.  Cost model: rounds of resident workgroups
// (ceil(workgroups / slots)) times the plane steps of one chunk (its planes
// plus the halo planes it recomputes); the common chunk that minimises it,
// then evened out per entry (the same number of chunks, each as short as that
// allows).  A launch of one entry keeps choose_tiling's chunk (the longest
// that keeps the launch within the resident slots, which the model also
// favours).  Entries with a chunk set by fa_pair_set_tuning keep it.
void batch_chunks(KernelKind kind, int halo, const std::vector<Tiling*>& ts, const std::vector<int>& n0s,
                  const std::vector<char>& pinned) {
  static const int kSlots[4] = {512, 1024, 512, 512};
  static const int kMinChunk[4] = {1, 4, 4, 1};
  if (ts.size() < 2 || ts[0]->cube) return;
  int zmax = 1;
  for (size_t i = 0; i < ts.size(); ++i) zmax = std::max(zmax, n0s[i]);
  double best = 0.0;
  int best_zc = 0;
  for (int zc = kMinChunk[kind]; zc <= std::max(zmax, kMinChunk[kind]); ++zc) {
    int64_t blocks = 0;
    int steps = 0;
    for (size_t i = 0; i < ts.size(); ++i) {
      const int z = pinned[i] ? ts[i]->zc : std::min(zc, n0s[i]);
      blocks += (int64_t)ts[i]->tiles_y * ts[i]->tiles_x * ((n0s[i] + z - 1) / z);
      steps = std::max(steps, z + halo);
    }
    const double cost = (double)((blocks + kSlots[kind] - 1) / kSlots[kind]) * steps;
    if (best_zc == 0 || cost < best) {
      best = cost;
      best_zc = zc;
    }
  }
  for (size_t i = 0; i < ts.size(); ++i) {
    if (pinned[i]) continue;
    const int z = std::min(best_zc, n0s[i]);
    const int chunks = (n0s[i] + z - 1) / z;
    ts[i]->zc = (n0s[i] + chunks - 1) / chunks;
    ts[i]->chunks = (n0s[i] + ts[i]->zc - 1) / ts[i]->zc;
  }
}

}  // namespace fa

extern "C" {

const char* fa_last_error(void) { return g_err.c_str(); }

fa_status fa_params_default(fa_params* out) {
  if (!out) return fail(FA_EINVAL, "out is NULL");
  out->eta = 0.5f;
  out->sigma_grad = 1.0f;
  out->sigma_warp = 0.5f;
  out->cc_window = 5;
  out->cc_eps = 1e-5f;
  out->adam_beta1 = 0.9f;
  out->adam_beta2 = 0.999f;
  out->adam_eps = 1e-8f;
  out->use_jac = 0;
  return FA_OK;
}

fa_status fa_pair_create(const float* fixed_dev, const float* moving_dev, fa_shape shape,
                         const fa_params* p, void* hip_stream, fa_pair* out) {
  if (!out) return fail(FA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!fixed_dev || !moving_dev) return fail(FA_EINVAL, "fixed and moving must be device pointers");
  FA_TRY(check_shape(shape));
  FA_TRY(check_params(p));
  fa_pair P = new (std::nothrow) fa_pair_s();
  if (!P) return fail(FA_ENOMEM, "host allocation failed");
  P->stream = (hipStream_t)hip_stream;
  P->shape = shape;
  P->n = voxels(shape);
  P->p = *p;
  (void)hipGetDevice(&P->device);
  fa_status st = FA_OK;
  const size_t bytes = (size_t)P->n * sizeof(float);
  if ((st = dalloc(&P->in_fixed, P->n, "fixed")) != FA_OK ||
      (st = dalloc(&P->in_moving, P->n, "moving")) != FA_OK ||
      (st = dalloc(&P->ctl, 1, "control block")) != FA_OK ||
      (st = dalloc(&P->scratch, fa::kMeanBlocks + 1, "scratch")) != FA_OK) {
    free_all(P);
    delete P;
    return st;
  }
  hipError_t e = hipMemcpyAsync(P->in_fixed, fixed_dev, bytes, hipMemcpyDeviceToDevice, P->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(P->in_moving, moving_dev, bytes, hipMemcpyDeviceToDevice, P->stream);
  if (e != hipSuccess) {
    free_all(P);
    delete P;
    return fail(FA_EHIP, std::string("copying the input volumes: ") + hipGetErrorString(e));
  }
  *out = P;
  return FA_OK;
}

fa_status fa_pair_set_schedule(fa_pair P, int n_levels, const float* scales, const int* iters) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (n_levels < 1 || n_levels > 16) return fail(FA_EINVAL, "n_levels must be in [1, 16]");
  if (!scales || !iters) return fail(FA_EINVAL, "scales and iters must not be NULL");
  std::vector<Level> lv(n_levels);
  int64_t total_iters = 0, nmax = 0;
  int pmax = 1;
  P->rg = tap_radius(P->p.sigma_grad);
  P->rw = tap_radius(P->p.sigma_warp);
  for (int i = 0; i < n_levels; ++i) {
    if (!(scales[i] >= 1.0f) || !(scales[i] <= 20.0f))
      return fail(FA_EINVAL, "scales must be in [1, 20]");
    if (iters[i] < 0) return fail(FA_EINVAL, "iters must be >= 0");
    lv[i].scale = scales[i];
    lv[i].iters = iters[i];
    lv[i].shape = level_shape(P->shape, scales[i]);
    lv[i].n = voxels(lv[i].shape);
    if (lv[i].shape.n0 < 2 || lv[i].shape.n1 < 2 || lv[i].shape.n2 < 2)
      return fail(FA_ESHAPE, "level " + std::to_string(i) + " has a dimension < 2");
    lv[i].tg = choose_tiling(lv[i].shape, fa::KIND_GRAD, P->tune[0], fa::grad_cube_supported(P->p.cc_window));
    lv[i].tsg = choose_tiling(lv[i].shape, fa::KIND_SMOOTH_MAX, P->tune[1],
                              fa::gauss_cube_supported(P->rg, fa::EPI_SMOOTH_MAX));
    lv[i].tsw = choose_tiling(lv[i].shape, fa::KIND_WARP_SMOOTH, P->tune[2],
                              fa::gauss_cube_supported(P->rw, fa::EPI_STORE));
    lv[i].tsc = choose_tiling(lv[i].shape, fa::KIND_COMPOSE, P->tune[3],
                              P->p.eta <= 2.0f && fa::gauss_cube_supported(0, fa::EPI_COMPOSE_LDS));
    {
      // shapes tuned earlier in this process for this grid and form (unless overridden)
      std::lock_guard<std::mutex> lk(tune_mutex());
      Tiling* slots[4] = {&lv[i].tg, &lv[i].tsg, &lv[i].tsw, &lv[i].tsc};
      for (int k = 0; k < 4; ++k) {
        const fa::Tuning& tu = P->tune[k];
        if (tu.ty || tu.tx || tu.zc || tu.variant) continue;
        auto it = tune_cache().find(TuneKey(P->device, k, lv[i].shape.n0, lv[i].shape.n1, lv[i].shape.n2,
                                            tune_form(P, k)));
        if (it != tune_cache().end()) {
          *slots[k] = it->second;
          lv[i].tuned[k] = true;
        }
      }
    }
    total_iters += iters[i];
    nmax = std::max(nmax, lv[i].n);
    pmax = std::max(pmax, lv[i].tg.blocks());
  }
  if (total_iters > (int64_t)1 << 30) return fail(FA_EINVAL, "too many iterations");

  // A previous schedule with the same level grids keeps its pyramid buffers
  // (its images are rebuilt below all the same), and nothing waits: the new
  // schedule's work queues behind the old one's on the stream.  Otherwise the
  // old pyramid is released first, which waits for the work still using it.
  bool reuse = P->levels.size() == (size_t)n_levels;
  for (int i = 0; reuse && i < n_levels; ++i) {
    const Level& o = P->levels[i];
    reuse = o.scale == lv[i].scale && o.shape.n0 == lv[i].shape.n0 && o.shape.n1 == lv[i].shape.n1 &&
            o.shape.n2 == lv[i].shape.n2;
  }
  if (reuse) {
    for (int i = 0; i < n_levels; ++i) {
      const Level& o = P->levels[i];
      lv[i].fixed = o.fixed;
      lv[i].moving = o.moving;
      lv[i].owns = o.owns;
      lv[i].moving_pad = o.moving_pad;
      lv[i].moving_quad = o.moving_quad;
    }
    P->levels = lv;   // owned by the pair while the rest of the call may fail
  } else {
    (void)hipStreamSynchronize(P->stream);
    free_levels(P);
  }
  P->scheduled = false;

  // Tap tables: sigma_grad, sigma_warp, then one per level for the blur.
  P->wts_host.clear();
  auto push = [&](const std::vector<float>& t) {
    const int off = (int)P->wts_host.size();
    P->wts_host.insert(P->wts_host.end(), t.begin(), t.end());
    while (P->wts_host.size() % 16) P->wts_host.push_back(0.0f);
    return off;
  };
  P->off_g = push(gaussian_taps(P->p.sigma_grad));
  P->off_w = push(gaussian_taps(P->p.sigma_warp));
  P->off_one = push(std::vector<float>{1.0f});
  P->off_blur.assign(n_levels, 0);
  for (int i = 0; i < n_levels; ++i) P->off_blur[i] = push(gaussian_taps(lv[i].scale / 2.0f));
  if (!P->wts || P->wts_dev != P->wts_host) {
    if (P->wts && P->wts_dev.size() < P->wts_host.size()) {
      (void)hipStreamSynchronize(P->stream);
      (void)hipFree(P->wts);
      P->wts = nullptr;
    }
    if (!P->wts) {
      P->wts_dev.clear();
      FA_TRY(dalloc(&P->wts, std::max(P->wts_host.size(), (size_t)256), "tap tables"));
    }
    // stream-ordered: queued kernels still read the previous table
    FA_HIP(hipMemcpyAsync(P->wts, P->wts_host.data(), P->wts_host.size() * sizeof(float),
                          hipMemcpyHostToDevice, P->stream));
    P->wts_dev = P->wts_host;
  }

  const bool wide = P->rg > fa::kMaxRadius || P->rw > fa::kMaxRadius;
  if (nmax > P->cap || (wide && !P->wide)) {
    (void)hipStreamSynchronize(P->stream);
    float** bufs[] = {&P->d, &P->m, &P->v, &P->a, &P->tmp, &P->wide};
    for (float** b : bufs) {
      if (*b) (void)hipFree(*b);
      *b = nullptr;
    }
    P->cap = 0;
    const int nb = wide ? 6 : 5;
    for (int k = 0; k < nb; ++k) FA_TRY(dalloc(bufs[k], (size_t)3 * nmax, "state"));
    P->cap = nmax;
  }
  if (total_iters > P->loss_cap) {
    (void)hipStreamSynchronize(P->stream);
    if (P->loss_hist) (void)hipFree(P->loss_hist);
    P->loss_hist = nullptr;
    P->loss_cap = 0;
    FA_TRY(dalloc(&P->loss_hist, (size_t)total_iters, "loss history"));
    P->loss_cap = (int)total_iters;
  }
  if (pmax > P->partials_cap) {
    (void)hipStreamSynchronize(P->stream);
    if (P->partials) (void)hipFree(P->partials);
    P->partials = nullptr;
    P->partials_cap = 0;
    FA_TRY(dalloc(&P->partials, (size_t)pmax, "loss partials"));
    P->partials_cap = pmax;
  }

  // Pyramid.
  bool need_blur = false;
  for (auto& L : lv) need_blur |= !(L.scale == 1.0f);
  if (need_blur && !P->blur0) {
    FA_TRY(dalloc(&P->blur0, (size_t)P->n, "pyramid scratch"));
    FA_TRY(dalloc(&P->blur1, (size_t)P->n, "pyramid scratch"));
  }
  P->levels = lv;
  for (int i = 0; i < n_levels; ++i) {
    Level& L = P->levels[i];
    if (L.scale == 1.0f) {
      L.fixed = P->in_fixed;
      L.moving = P->in_moving;
      L.owns = false;
      continue;
    }
    if (!L.fixed) {
      fa_status st;
      if ((st = dalloc(&L.fixed, (size_t)L.n, "pyramid")) != FA_OK) return st;
      if ((st = dalloc(&L.moving, (size_t)L.n, "pyramid")) != FA_OK) {
        (void)hipFree(L.fixed);
        L.fixed = nullptr;
        return st;
      }
      L.owns = true;
    }
    FA_TRY(build_level_image(P, P->in_fixed, L.fixed, L, P->off_blur[i]));
    FA_TRY(build_level_image(P, P->in_moving, L.moving, L, P->off_blur[i]));
  }
  for (auto& L : P->levels) {
    if (!L.moving_pad)
      FA_TRY(dalloc(&L.moving_pad, (size_t)fa::padded_voxels(L.shape.n0, L.shape.n1, L.shape.n2),
                    "padded moving"));
    FA_HIP(fa::launch_pad(L.moving, L.moving_pad, L.shape.n0, L.shape.n1, L.shape.n2, P->stream));
    if (fa::quad_supported(L.shape.n0, L.shape.n1, L.shape.n2)) {
      if (!L.moving_quad)
        FA_TRY(dalloc(&L.moving_quad, (size_t)4 * fa::padded_voxels(L.shape.n0, L.shape.n1, L.shape.n2),
                      "padded moving quads"));
      FA_HIP(fa::launch_pad_quad(L.moving_pad, L.moving_quad, L.shape.n0, L.shape.n1, L.shape.n2, P->stream));
    }
  }

  // State: phi = id, m = v = 0, t = 0.
  const int64_t n0 = P->levels[0].n;
  FA_HIP(fa::launch_fill(P->d, 0.0f, 3 * n0, P->stream));
  FA_HIP(fa::launch_fill(P->m, 0.0f, 3 * n0, P->stream));
  FA_HIP(fa::launch_fill(P->v, 0.0f, 3 * n0, P->stream));
  FA_HIP(fa::launch_fill(P->a, 0.0f, 3 * n0, P->stream));
  FA_HIP(fa::launch_ctl_init(P->ctl, P->p.adam_beta1, P->p.adam_beta2, 0, 0, P->stream));
  FA_HIP(fa::launch_mean(P->in_fixed, P->n, P->scratch, &P->ctl->shift_i, P->stream));
  FA_HIP(fa::launch_mean(P->in_moving, P->n, P->scratch, &P->ctl->shift_j, P->stream));
  P->cur_level = 0;
  P->cur_iter = 0;
  P->t_done = 0;
  P->iters_done = 0;
  P->scheduled = true;
  return FA_OK;
}

fa_status fa_pair_step(fa_pair P, int max_iters, int* iters_done, int* finished) {
  if (iters_done) *iters_done = 0;
  if (finished) *finished = 0;
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  if (max_iters < 0) return fail(FA_EINVAL, "max_iters must be >= 0");
  int done = 0;
  while (done < max_iters) {
    FA_TRY(advance_levels(P));
    if (schedule_done(P)) break;
    const Level& L = P->levels[P->cur_level];
    FA_TRY(launch_iteration(P, L));
    P->cur_iter += 1;
    P->t_done += 1;
    P->iters_done += 1;
    done += 1;
  }
  if (iters_done) *iters_done = done;
  if (finished) *finished = schedule_done(P) ? 1 : 0;
  return FA_OK;
}

fa_status fa_batch_step(fa_pair* pairs, int n, int max_iters, int* n_finished) {
  if (n_finished) *n_finished = 0;
  FA_TRY(check_batch(pairs, n, max_iters));
  // one iteration per pair in turn: each stream always has work queued
  std::vector<char> live(n, 1);
  for (int k = 0; k < max_iters; ++k) {
    int active = 0;
    for (int i = 0; i < n; ++i) {
      if (!live[i]) continue;
      int done = 0, fin = 0;
      FA_TRY(fa_pair_step(pairs[i], 1, &done, &fin));
      if (fin || done == 0) live[i] = 0;
      active += live[i];
    }
    if (active == 0) break;
  }
  if (n_finished) *n_finished = count_finished(pairs, n);
  return FA_OK;
}

void fa_batch_use_graphs(int enable) { g_batch_graphs = enable != 0; }

fa_status fa_batch_step_fused(fa_pair* pairs, int n, int max_iters, int* n_finished) {
  if (n_finished) *n_finished = 0;
  FA_TRY(check_batch(pairs, n, max_iters));
  for (int i = 1; i < n; ++i)
    if (pairs[i]->device != pairs[0]->device) return fail(FA_EINVAL, "the pairs of a batch must share a device");
  if (n > 0 && max_iters > 0) {
    // Every pair's work goes to one stream for the duration of the call:
    // pairs[0]'s, or with graphs a private one (the default stream cannot be
    // captured).  That stream first waits for the pairs' queued work, and
    // their streams wait for it at the end.
    hipStream_t priv = nullptr;
    if (g_batch_graphs) FA_HIP(hipStreamCreateWithFlags(&priv, hipStreamNonBlocking));
    const hipStream_t s = priv ? priv : pairs[0]->stream;
    std::vector<hipStream_t> saved(n);
    std::vector<hipEvent_t> evs;
    fa_status st = FA_OK;
    for (int i = 0; i < n && st == FA_OK; ++i) {
      saved[i] = pairs[i]->stream;
      if (saved[i] == s) continue;
      bool seen = false;   // join each distinct stream once
      for (int j = 0; j < i; ++j) seen |= saved[j] == saved[i];
      if (seen) continue;
      hipEvent_t e = nullptr;
      hipError_t he = hipEventCreateWithFlags(&e, hipEventDisableTiming);
      if (he == hipSuccess) {
        evs.push_back(e);
        he = hipEventRecord(e, saved[i]);
      }
      if (he == hipSuccess) he = hipStreamWaitEvent(s, e, 0);
      if (he != hipSuccess) st = fail(FA_EHIP, std::string("joining the pairs' streams: ") + hipGetErrorString(he));
    }
    if (st == FA_OK) {
      for (int i = 0; i < n; ++i) pairs[i]->stream = s;
      st = run_batch_fused(pairs, n, max_iters, s);
      for (int i = 0; i < n; ++i) pairs[i]->stream = saved[i];
    }
    hipEvent_t done = nullptr;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess) {
      evs.push_back(done);
      if (hipEventRecord(done, s) == hipSuccess)
        for (int i = 0; i < n; ++i)
          if (saved[i] != s) (void)hipStreamWaitEvent(saved[i], done, 0);
    }
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    if (priv) (void)hipStreamDestroy(priv);   // its queued work still completes
    if (st != FA_OK) return st;
  }
  if (n_finished) *n_finished = count_finished(pairs, n);
  return FA_OK;
}

fa_status fa_pair_get_loss(fa_pair P, float* host_out, int capacity, int* n_written) {
  if (n_written) *n_written = 0;
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!host_out && capacity > 0) return fail(FA_EINVAL, "host_out is NULL");
  const int cnt = std::min(std::max(capacity, 0), P->scheduled ? std::min(P->iters_done, P->loss_cap) : 0);
  FA_HIP(hipStreamSynchronize(P->stream));
  if (cnt > 0) FA_HIP(hipMemcpy(host_out, P->loss_hist, (size_t)cnt * sizeof(float), hipMemcpyDeviceToHost));
  if (n_written) *n_written = cnt;
  return FA_OK;
}

fa_status fa_pair_get_field(fa_pair P, float* dev_out, int layout, int* level, fa_shape* shape) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  if (layout != 0 && layout != 1) return fail(FA_EINVAL, "layout must be 0 (SoA) or 1 (AoS)");
  const Level& L = P->levels[P->cur_level];
  if (level) *level = P->cur_level;
  if (shape) *shape = L.shape;
  if (!dev_out) return FA_OK;
  if (layout == 0)
    FA_HIP(hipMemcpyAsync(dev_out, P->d, (size_t)3 * L.n * sizeof(float), hipMemcpyDeviceToDevice, P->stream));
  else
    FA_HIP(fa::launch_soa_to_aos(P->d, dev_out, L.n, P->stream));
  return FA_OK;
}

fa_status fa_pair_get_warped(fa_pair P, float* dev_out) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!dev_out) return fail(FA_EINVAL, "dev_out is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  const Level& L = P->levels[P->cur_level];
  FA_HIP(fa::launch_warp(L.moving, P->d, dev_out, L.shape.n0, L.shape.n1, L.shape.n2, P->stream));
  return FA_OK;
}

void fa_pair_destroy(fa_pair P) {
  if (!P) return;
  (void)hipStreamSynchronize(P->stream);
  for (auto& pe : P->pending)
    for (int k = 0; k < 5; ++k) P->ev_pool.push_back(pe.e[k]);
  for (hipEvent_t e : P->ev_pool) (void)hipEventDestroy(e);
  free_all(P);
  delete P;
}

// ---- fa_inspect.h ---------------------------------------------------------

fa_status fa_pair_get_progress(fa_pair P, int* level, int* iter_in_level, int* t_done) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (level) *level = P->cur_level;
  if (iter_in_level) *iter_in_level = P->cur_iter;
  if (t_done) *t_done = P->t_done;
  return FA_OK;
}

fa_status fa_pair_set_state(fa_pair P, const float* d, const float* m, const float* v, int t_done) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  if (t_done < 0 || t_done > (1 << 30)) return fail(FA_EINVAL, "t_done out of range");
  const Level& L = P->levels[P->cur_level];
  const size_t bytes = (size_t)3 * L.n * sizeof(float);
  if (d) FA_HIP(hipMemcpyAsync(P->d, d, bytes, hipMemcpyDeviceToDevice, P->stream));
  if (m) FA_HIP(hipMemcpyAsync(P->m, m, bytes, hipMemcpyDeviceToDevice, P->stream));
  if (v) FA_HIP(hipMemcpyAsync(P->v, v, bytes, hipMemcpyDeviceToDevice, P->stream));
  FA_HIP(fa::launch_ctl_init(P->ctl, P->p.adam_beta1, P->p.adam_beta2, t_done, -1, P->stream));
  P->t_done = t_done;
  return FA_OK;
}

fa_status fa_pair_get_state(fa_pair P, float* d, float* m, float* v) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  const Level& L = P->levels[P->cur_level];
  const size_t bytes = (size_t)3 * L.n * sizeof(float);
  if (d) FA_HIP(hipMemcpyAsync(d, P->d, bytes, hipMemcpyDeviceToDevice, P->stream));
  if (m) FA_HIP(hipMemcpyAsync(m, P->m, bytes, hipMemcpyDeviceToDevice, P->stream));
  if (v) FA_HIP(hipMemcpyAsync(v, P->v, bytes, hipMemcpyDeviceToDevice, P->stream));
  return FA_OK;
}

fa_status fa_pair_eval_gradient(fa_pair P, float* g_dev, float* loss_host) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  const Level& L = P->levels[P->cur_level];
  fa::GradArgs ga{};
  ga.fixed = L.fixed;
  ga.moving_pad = L.moving_pad;
  ga.moving_quad = L.moving_quad;
  ga.d = P->d;
  ga.out = g_dev ? g_dev : P->tmp;
  ga.partials = P->partials;
  ga.ctl = P->ctl;
  ga.n0 = L.shape.n0;
  ga.n1 = L.shape.n1;
  ga.n2 = L.shape.n2;
  ga.zc = L.tg.zc;
  ga.tiles_y = L.tg.tiles_y;
  ga.tiles_x = L.tg.tiles_x;
  ga.eps_cc = P->p.cc_eps;
  ga.inv_n = (float)(1.0 / (double)L.n);
  ga.mode = 1;
  FA_HIP(fa::launch_grad(ga, P->p.cc_window, L.tg, P->stream));
  if (loss_host) {
    FA_HIP(fa::launch_sum_partials(P->partials, L.tg.blocks(), P->scratch + fa::kMeanBlocks, P->stream));
    double s = 0.0;
    FA_HIP(hipMemcpyAsync(&s, P->scratch + fa::kMeanBlocks, sizeof(double), hipMemcpyDeviceToHost, P->stream));
    FA_HIP(hipStreamSynchronize(P->stream));
    *loss_host = (float)(-s / (double)L.n);
  }
  return FA_OK;
}

fa_status fa_pair_get_direction(fa_pair P, float* dev_out) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!dev_out) return fail(FA_EINVAL, "dev_out is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  const Level& L = P->levels[P->cur_level];
  FA_HIP(hipMemcpyAsync(dev_out, P->a, (size_t)3 * L.n * sizeof(float), hipMemcpyDeviceToDevice, P->stream));
  return FA_OK;
}

fa_status fa_pair_get_step_norm(fa_pair P, float* m_host) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!m_host) return fail(FA_EINVAL, "m_host is NULL");
  Ctl c;
  FA_HIP(hipMemcpyAsync(&c, P->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, P->stream));
  FA_HIP(hipStreamSynchronize(P->stream));
  unsigned m = 0u;   // M is the largest slot (fa_internal.h)
  for (int j = 0; j < fa::kMSlots; ++j) m = std::max(m, c.mslot[j * fa::kMStride]);
  std::memcpy(m_host, &m, sizeof(float));
  return FA_OK;
}

fa_status fa_pair_get_level_image(fa_pair P, int level, int which, float* dev_out, fa_shape* shape) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  if (level < 0 || level >= (int)P->levels.size()) return fail(FA_EINVAL, "level out of range");
  if (which != 0 && which != 1) return fail(FA_EINVAL, "which must be 0 (fixed) or 1 (moving)");
  const Level& L = P->levels[level];
  if (shape) *shape = L.shape;
  if (!dev_out) return FA_OK;
  FA_HIP(hipMemcpyAsync(dev_out, which ? L.moving : L.fixed, (size_t)L.n * sizeof(float),
                        hipMemcpyDeviceToDevice, P->stream));
  return FA_OK;
}

fa_status fa_plan_tiling(int kind, int n, const fa_shape* shapes, int halo, int batched, int* zc_out,
                         int* blocks_out) {
  if (kind < 0 || kind > 3) return fail(FA_EINVAL, "kind must be in [0, 3]");
  if (n < 1 || !shapes) return fail(FA_EINVAL, "shapes is NULL or n < 1");
  if (halo < 0) return fail(FA_EINVAL, "halo must be >= 0");
  std::vector<Tiling> ts(n);
  std::vector<Tiling*> tp(n);
  std::vector<int> n0s(n);
  for (int i = 0; i < n; ++i) {
    FA_TRY(check_shape(shapes[i]));
    ts[i] = choose_tiling(shapes[i], (fa::KernelKind)kind);
    tp[i] = &ts[i];
    n0s[i] = shapes[i].n0;
  }
  if (batched) fa::batch_chunks((fa::KernelKind)kind, halo, tp, n0s, std::vector<char>(n, 0));
  for (int i = 0; i < n; ++i) {
    if (zc_out) zc_out[i] = ts[i].zc;
    if (blocks_out) blocks_out[i] = ts[i].blocks();
  }
  return FA_OK;
}

fa_status fa_pair_set_tuning(fa_pair P, int kind, int ty, int tx, int zc, int variant) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (kind < 0 || kind > 3) return fail(FA_EINVAL, "kind must be 0, 1, 2 or 3");
  const bool autotile = ty == 0 && tx == 0;
  if (!autotile && !(kind == 0 ? fa::grad_tile_supported(ty, tx) : fa::gauss_tile_supported(ty, tx)))
    return fail(FA_EINVAL, "unsupported tile shape");
  if (zc < 0 || variant < 0 || variant > (kind == 0 ? 3 : 2))
    return fail(FA_EINVAL, "zc must be >= 0 and variant in [0, 3] (kind 0) or [0, 2] (kinds 1 to 3)");
  P->tune[kind].ty = ty;
  P->tune[kind].tx = tx;
  P->tune[kind].zc = zc;
  P->tune[kind].variant = variant;
  return FA_OK;
}

fa_status fa_pair_profile(fa_pair P, int enable) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  FA_TRY(drain_profile(P));
  P->profiling = enable != 0;
  if (P->profiling) {
    P->prof_ms.assign((size_t)16 * 4, 0.0);
    P->prof_n.assign((size_t)16 * 4, 0);
  }
  return FA_OK;
}

fa_status fa_pair_get_profile(fa_pair P, int level, int kind, double* total_ms, int* launches) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (level < 0 || level >= 16 || kind < 0 || kind > 3) return fail(FA_EINVAL, "level or kind out of range");
  FA_TRY(drain_profile(P));
  const size_t slot = (size_t)level * 4 + kind;
  if (total_ms) *total_ms = slot < P->prof_ms.size() ? P->prof_ms[slot] : 0.0;
  if (launches) *launches = slot < P->prof_n.size() ? P->prof_n[slot] : 0;
  return FA_OK;
}

// ---- fa_pair_autotune ---------------------------------------------------------

}  // extern "C"

namespace {

// Candidate march tilings of kernel `kind` at shape s around the automatic
// one: both in-plane tiles (8x64 too for the smoothing kinds), and chunk
// lengths giving 1/2, 2/3, 1, 3/2 and 2 times the automatic number of chunks;
// plus the brick form where it exists and the volume is small enough for it
// to have a chance.
std::vector<Tiling> tiling_candidates(const fa_shape& s, fa::KernelKind kind, const Tiling& t0, bool cube_ok) {
  std::vector<Tiling> out;
  auto add = [&](const Tiling& t) {
    for (const Tiling& u : out)
      if (u.cube == t.cube && u.ty == t.ty && u.tx == t.tx && u.zc == t.zc) return;
    out.push_back(t);
  };
  add(t0);
  std::vector<std::pair<int, int>> tiles = {{16, 32}, {8, 32}};
  if (kind != fa::KIND_GRAD) tiles.push_back({8, 64});
  for (auto [ty, tx] : tiles) {
    if (ty == 16 && s.n1 < 16) continue;
    fa::Tuning tu;
    tu.ty = ty;
    tu.tx = tx;
    tu.variant = 1;
    const Tiling base = choose_tiling(s, kind, tu, false);
    const int chunks0 = base.chunks;
    for (int num_den : {12, 23, 11, 32, 21}) {   // chunk-count factors 1/2, 2/3, 1, 3/2, 2
      const int num = num_den / 10, den = num_den % 10;
      const int ch = std::max(1, (chunks0 * num + den - 1) / den);
      fa::Tuning tz = tu;
      tz.zc = std::max(1, (s.n0 + ch - 1) / ch);
      add(choose_tiling(s, kind, tz, false));
    }
  }
  if (cube_ok && voxels(s) <= 1200000) {
    fa::Tuning tc;
    tc.variant = kind == fa::KIND_GRAD ? 3 : 2;
    add(choose_tiling(s, kind, tc, true));
  }
  return out;
}

}  // namespace

extern "C" {

fa_status fa_pair_autotune(fa_pair P, int trials) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  if (trials < 1 || trials > 100) return fail(FA_EINVAL, "trials must be in [1, 100]");
  FA_HIP(hipStreamSynchronize(P->stream));
  // scratch control block: the timing launches update M and the step count there
  Ctl* sctl = nullptr;
  FA_TRY(dalloc(&sctl, 1, "scratch control block"));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fa_status st = FA_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    st = fail(FA_EHIP, "hipEventCreate failed");
  // the fastest of three timed runs of `trials` launches each, after a warm-up
  auto time_it = [&](auto&& launch, double* us) -> fa_status {
    FA_HIP(launch());
    *us = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      FA_HIP(hipEventRecord(e0, P->stream));
      for (int r = 0; r < trials; ++r) FA_HIP(launch());
      FA_HIP(hipEventRecord(e1, P->stream));
      FA_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      FA_HIP(hipEventElapsedTime(&ms, e0, e1));
      *us = std::min(*us, 1e3 * ms / trials);
    }
    return FA_OK;
  };
  if (st == FA_OK) {
    const hipError_t he = fa::launch_ctl_init(sctl, P->p.adam_beta1, P->p.adam_beta2, 0, 0, P->stream);
    if (he != hipSuccess) st = fail(FA_EHIP, hipGetErrorString(he));
  }
  for (size_t li = 0; li < P->levels.size() && st == FA_OK; ++li) {
    Level& L = P->levels[li];
    const int w = P->p.cc_window;
    // the gradient: mode 0 with m, v and the direction all in the scratch buffer tmp
    std::vector<Tiling> cg = tiling_candidates(L.shape, fa::KIND_GRAD, L.tg, fa::grad_cube_supported(w));
    int need = 0;
    for (const Tiling& t : cg) need = std::max(need, t.blocks());
    if (need > P->partials_cap) {
      if (P->partials) (void)hipFree(P->partials);
      P->partials = nullptr;
      P->partials_cap = 0;
      if ((st = dalloc(&P->partials, (size_t)need, "loss partials")) != FA_OK) break;
      P->partials_cap = need;
    }
    IterPlan it;
    plan_iteration(P, L, it);
    fa::GradArgs ga = it.ga;
    ga.m = ga.v = ga.out = P->tmp;
    ga.ctl = sctl;
    ga.mode = 0;
    double best = 1e30;
    Tiling bt = L.tg;
    for (const Tiling& t : cg) {
      fa::GradArgs a = ga;
      a.zc = t.zc;
      a.tiles_y = t.tiles_y;
      a.tiles_x = t.tiles_x;
      double us = 0.0;
      if ((st = time_it([&]() { return fa::launch_grad(a, w, t, P->stream); }, &us)) != FA_OK) break;
      if (us < best) {
        best = us;
        bt = t;
      }
    }
    if (st != FA_OK) break;
    L.tg = bt;
    L.tuned[fa::KIND_GRAD] = true;
    {
      std::lock_guard<std::mutex> lk(tune_mutex());
      tune_cache()[TuneKey(P->device, fa::KIND_GRAD, L.shape.n0, L.shape.n1, L.shape.n2,
                           tune_form(P, fa::KIND_GRAD))] = bt;
    }
    // the smoothing and composition launches, on scratch buffers a and tmp
    const fa::KernelKind kinds[3] = {fa::KIND_SMOOTH_MAX, fa::KIND_COMPOSE, fa::KIND_WARP_SMOOTH};
    Tiling* slots[3] = {&L.tsg, &L.tsc, &L.tsw};
    for (int k = 0; k < 3 && st == FA_OK; ++k) {
      const bool cube_ok = k == 0   ? fa::gauss_cube_supported(P->rg, fa::EPI_SMOOTH_MAX)
                           : k == 1 ? (P->p.eta <= 2.0f && fa::gauss_cube_supported(0, fa::EPI_COMPOSE_LDS))
                                    : fa::gauss_cube_supported(P->rw, fa::EPI_STORE);
      std::vector<Tiling> cs = tiling_candidates(L.shape, kinds[k], *slots[k], cube_ok);
      fa::GaussArgs g = it.g[k];
      g.ctl = sctl;
      if (k == 0) {
        g.in = P->a;
        g.out = P->tmp;
      } else if (k == 1) {
        g.in = g.out = P->tmp;
      } else {
        g.in = P->tmp;
        g.out = P->a;
      }
      if (g.partials) {   // the record runs (on the scratch control block) but stores no loss
        g.loss_hist = nullptr;
        g.n_partials = std::min(L.tg.blocks(), P->partials_cap);
      }
      double bestk = 1e30;
      Tiling btk = *slots[k];
      for (const Tiling& t : cs) {
        fa::GaussArgs a = g;
        a.zc = t.zc;
        a.tiles_y = t.tiles_y;
        a.tiles_x = t.tiles_x;
        double us = 0.0;
        if ((st = time_it([&]() { return fa::launch_gauss(a, it.radius[k], it.epi[k], t, P->stream); }, &us)) != FA_OK)
          break;
        if (us < bestk) {
          bestk = us;
          btk = t;
        }
      }
      if (st == FA_OK) {
        *slots[k] = btk;
        L.tuned[kinds[k]] = true;
        std::lock_guard<std::mutex> lk(tune_mutex());
        tune_cache()[TuneKey(P->device, kinds[k], L.shape.n0, L.shape.n1, L.shape.n2, tune_form(P, kinds[k]))] = btk;
      }
    }
  }
  (void)hipStreamSynchronize(P->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sctl);
  return st;
}

void fa_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(tune_mutex());
  tune_cache().clear();
}

fa_status fa_pair_get_tiling(fa_pair P, int level, int kind, int* ty, int* tx, int* zc, int* brick) {
  if (!P) return fail(FA_EINVAL, "pair is NULL");
  if (!P->scheduled) return fail(FA_ESTATE, "fa_pair_set_schedule has not been called");
  if (level < 0 || level >= (int)P->levels.size()) return fail(FA_EINVAL, "level out of range");
  if (kind < 0 || kind > 3) return fail(FA_EINVAL, "kind must be in [0, 3]");
  const Level& L = P->levels[level];
  const Tiling& t = kind == 0 ? L.tg : kind == 1 ? L.tsg : kind == 2 ? L.tsw : L.tsc;
  if (ty) *ty = t.ty;
  if (tx) *tx = t.tx;
  if (zc) *zc = t.zc;
  if (brick) *brick = t.cube ? 1 : 0;
  return FA_OK;
}

}  // extern "C"

// ---- fa_symmetric.h ---------------------------------------------------------
// Two pairs share the handle's stream: M registers I_M (its moving image)
// toward I_F o phi_F, F registers I_F toward I_M o phi_M.  Each pair's
// level-l fixed image is the other side's level-l image; the warped images
// replace it as the fixed image of every iteration.
struct fa_sym_s {
  fa_pair F = nullptr;
  fa_pair M = nullptr;
  float* wf = nullptr;   // I_F o phi_F at the current level
  float* wm = nullptr;   // I_M o phi_M
  int64_t wcap = 0;
  hipStream_t stream = nullptr;
  fa_shape shape{};
};

extern "C" {

fa_status fa_sym_create(const float* fixed, const float* moving, fa_shape shape, const fa_params* params,
                        void* stream, fa_sym* out) {
  if (!out) return fail(FA_EINVAL, "out is NULL");
  *out = nullptr;
  fa_sym H = new (std::nothrow) fa_sym_s();
  if (!H) return fail(FA_ENOMEM, "host allocation failed");
  H->stream = (hipStream_t)stream;
  H->shape = shape;
  fa_status st = fa_pair_create(moving, fixed, shape, params, stream, &H->F);
  if (st == FA_OK) st = fa_pair_create(fixed, moving, shape, params, stream, &H->M);
  if (st != FA_OK) {
    fa_pair_destroy(H->F);
    delete H;
    return st;
  }
  *out = H;
  return FA_OK;
}

fa_status fa_sym_set_schedule(fa_sym H, int n_levels, const float* scales, const int* iters) {
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  FA_TRY(fa_pair_set_schedule(H->F, n_levels, scales, iters));
  FA_TRY(fa_pair_set_schedule(H->M, n_levels, scales, iters));
  int64_t nmax = 0;
  for (const Level& L : H->M->levels) nmax = std::max(nmax, L.n);
  if (nmax > H->wcap) {
    FA_HIP(hipStreamSynchronize(H->stream));
    if (H->wf) (void)hipFree(H->wf);
    if (H->wm) (void)hipFree(H->wm);
    H->wf = H->wm = nullptr;
    H->wcap = 0;
    FA_TRY(dalloc(&H->wf, (size_t)nmax, "warped image"));
    FA_TRY(dalloc(&H->wm, (size_t)nmax, "warped image"));
    H->wcap = nmax;
  }
  return FA_OK;
}

fa_status fa_sym_step(fa_sym H, int max_iters, int* iters_done, int* finished) {
  if (iters_done) *iters_done = 0;
  if (finished) *finished = 0;
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  if (!H->F->scheduled || !H->M->scheduled) return fail(FA_ESTATE, "fa_sym_set_schedule has not been called");
  if (max_iters < 0) return fail(FA_EINVAL, "max_iters must be >= 0");
  fa_pair F = H->F, M = H->M;
  M->fixed_override = H->wf;
  F->fixed_override = H->wm;
  // the two halves share every template parameter: each kernel of an
  // iteration is one batched launch over both
  const std::vector<fa_pair> both = {M, F};
  BatchTables bt;
  int level = -1;
  int done = 0;
  fa_status st = FA_OK;
  while (done < max_iters && st == FA_OK) {
    if ((st = advance_levels(F)) != FA_OK || (st = advance_levels(M)) != FA_OK) break;
    if (schedule_done(M)) break;
    if (M->cur_level != level) {
      if ((st = build_batch_tables(both, bt)) != FA_OK) break;
      if ((st = upload_batch_tables(bt, H->stream)) != FA_OK) break;
      level = M->cur_level;
    }
    const Level& LF = F->levels[F->cur_level];
    const Level& LM = M->levels[M->cur_level];
    const fa_shape& s = LM.shape;
    // both warped images first: the two halves step from the same pair of warps
    hipError_t he = fa::launch_warp(LF.moving, F->d, H->wf, s.n0, s.n1, s.n2, H->stream);
    if (he == hipSuccess) he = fa::launch_warp(LM.moving, M->d, H->wm, s.n0, s.n1, s.n2, H->stream);
    if (he != hipSuccess) {
      st = fail(FA_EHIP, std::string("warp: ") + hipGetErrorString(he));
      break;
    }
    if ((st = launch_batch_iteration(both, bt, H->stream)) != FA_OK) break;
    for (fa_pair P : both) {
      P->cur_iter += 1;
      P->t_done += 1;
      P->iters_done += 1;
    }
    done += 1;
  }
  if (bt.dev) {
    const hipError_t e1 = hipStreamSynchronize(H->stream);
    const hipError_t e2 = hipFree(bt.dev);
    if (st == FA_OK && e1 != hipSuccess) st = fail(FA_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e1));
    if (st == FA_OK && e2 != hipSuccess) st = fail(FA_EHIP, std::string("hipFree: ") + hipGetErrorString(e2));
  }
  if (st != FA_OK) return st;
  if (iters_done) *iters_done = done;
  if (finished) *finished = schedule_done(M) ? 1 : 0;
  return FA_OK;
}

fa_status fa_sym_get_halfway(fa_sym H, float* dF_dev, float* dM_dev, int* level, fa_shape* shape) {
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  FA_TRY(fa_pair_get_field(H->F, dF_dev, 0, nullptr, nullptr));
  return fa_pair_get_field(H->M, dM_dev, 0, level, shape);
}

fa_status fa_sym_get_loss(fa_sym H, float* host_out, int capacity, int* n_written) {
  if (n_written) *n_written = 0;
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  return fa_pair_get_loss(H->M, host_out, capacity, n_written);
}

fa_status fa_sym_finish(fa_sym H, const fa_params* inv_params, int n_levels, const float* scales,
                        const int* iters, float* d_out, float* inv_cost) {
  if (!H) return fail(FA_EINVAL, "handle is NULL");
  if (!d_out) return fail(FA_EINVAL, "d_out is NULL");
  if (!H->M->scheduled || !schedule_done(H->M) || !schedule_done(H->F))
    return fail(FA_ESTATE, "the half-way schedule is not complete");
  const Level& L = H->M->levels[H->M->cur_level];
  if (L.shape.n0 != H->shape.n0 || L.shape.n1 != H->shape.n1 || L.shape.n2 != H->shape.n2)
    return fail(FA_ESTATE, "the schedule's last level must be the input grid (scale 1)");
  fa_inverse inv = nullptr;
  FA_TRY(fa_inverse_create(H->F->d, H->shape, inv_params, H->stream, &inv));
  fa_status st = fa_inverse_set_schedule(inv, n_levels, scales, iters);
  if (st == FA_OK) st = fa_inverse_step(inv, 1 << 30, nullptr, nullptr);
  int lvl = 0;
  fa_shape es{};
  if (st == FA_OK) st = fa_inverse_get_field(inv, nullptr, &lvl, &es);
  if (st == FA_OK && (es.n0 != H->shape.n0 || es.n1 != H->shape.n1 || es.n2 != H->shape.n2))
    st = fail(FA_EINVAL, "the inverse schedule's last level must be the input grid (scale 1)");
  // e goes to pair M's scratch field (3 n floats, idle once the schedule is done)
  float* e = H->M->tmp;
  if (st == FA_OK) st = fa_inverse_get_field(inv, e, nullptr, nullptr);
  if (st == FA_OK) {
    const hipError_t he = fa::launch_compose_fields(e, H->M->d, d_out, H->shape.n0, H->shape.n1, H->shape.n2,
                                                    H->stream);
    if (he != hipSuccess) st = fail(FA_EHIP, std::string("compose: ") + hipGetErrorString(he));
  }
  if (st == FA_OK && inv_cost) {
    int total = 0;
    for (int i = 0; i < n_levels; ++i) total += iters[i];
    std::vector<float> hist((size_t)std::max(total, 1));
    int got = 0;
    st = fa_inverse_get_loss(inv, hist.data(), total, &got);
    *inv_cost = got > 0 ? hist[(size_t)got - 1] : 0.0f;
  }
  fa_inverse_destroy(inv);
  if (st == FA_OK) {
    const hipError_t he = hipStreamSynchronize(H->stream);
    if (he != hipSuccess) st = fail(FA_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(he));
  }
  return st;
}

void fa_sym_destroy(fa_sym H) {
  if (!H) return;
  (void)hipStreamSynchronize(H->stream);
  if (H->wf) (void)hipFree(H->wf);
  if (H->wm) (void)hipFree(H->wm);
  fa_pair_destroy(H->F);
  fa_pair_destroy(H->M);
  delete H;
}

}  // extern "C"
