// Host runtime of the salprior C-ABI: parameter validation, geometry, device memory
// layout, job tables, Kalman gain bookkeeping, the adjoint driver and the batched
// graph-replayed step.  Every device buffer is allocated in sp_create /
// sp_batch_create; the per-frame calls only enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "salprior.h"
#include "sp_internal.h"
#include "sp_kernels.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                                  \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail(SP_EHIP, "%s: %s (%d)", #expr, hipGetErrorString(e_), (int)e_); \
  } while (0)

constexpr int kTile = 16;   // tile edge of every tiled phase

// ---------------------------------------------------------------- geometry
struct Geo {
  int H = 0, W = 0, depth = 0, top = 0, c_min = 0, c_max = 0, n_pairs = 0;
  int pc[SP_MAXP] = {}, ps[SP_MAXP] = {};
  int Hl[SP_MAXL] = {}, Wl[SP_MAXL] = {};
  unsigned used = 0;   // bit l: level l is a centre or surround
};

bool is_fin(double v) { return std::isfinite(v); }

constexpr size_t kMaxDynLds = 150 * 1024;   // dynamic LDS of the across-scale-sum job (gfx950: 160 KB per CU)

// Reduced-map path: every pair has its centre at c_max or one level below.
bool gpath_ok(const Geo& g) {
  if (g.n_pairs < 1) return false;
  for (int p = 0; p < g.n_pairs; ++p)
    if (g.c_max - g.pc[p] > 1) return false;
  return true;
}

// Pair set the reduced-map kernel is compiled for (see cg_set1_r/d): 1 when the
// geometry's pairs are, in order, (c_max - c, s - c) = (1,2), (1,3), (0,2), (0,3); 0 reads
// the pairs at run time.
int csg_set(const Geo& g) {
  if (!gpath_ok(g) || g.n_pairs != CG_SET1_N) return 0;
  for (int p = 0; p < g.n_pairs; ++p)
    if (g.c_max - g.pc[p] != cg_set1_r(p) || g.ps[p] - g.pc[p] != cg_set1_d(p)) return 0;
  return 1;
}

size_t csg_lds_bytes(const Geo& g) {
  return sizeof(float) * (size_t)csg_layout(g.pc, g.ps, g.n_pairs, g.c_max).total;
}

size_t csapply_lds_bytes(const Geo& g) {
  return sizeof(float) * (size_t)csapply_layout(g.pc, g.ps, g.n_pairs, g.c_max).total;
}

int validate_params(const sp_params* p) {
  if (!p) return fail(SP_EINVAL, "params is NULL");
  if (p->n_centers < 1 || p->n_centers > 4) return fail(SP_EINVAL, "n_centers must be 1..4 (got %d)", p->n_centers);
  if (p->n_deltas < 1 || p->n_deltas > 4) return fail(SP_EINVAL, "n_deltas must be 1..4 (got %d)", p->n_deltas);
  for (int i = 0; i < p->n_centers; ++i)
    if (p->centers[i] < 1 || p->centers[i] > SP_MAX_LEVELS)
      return fail(SP_EINVAL, "centre levels must be 1..%d (got %d)", SP_MAX_LEVELS, p->centers[i]);
  for (int i = 0; i < p->n_deltas; ++i)
    if (p->deltas[i] < 1 || p->deltas[i] > SP_MAX_LEVELS)
      return fail(SP_EINVAL, "centre-surround offsets must be 1..%d (got %d)", SP_MAX_LEVELS, p->deltas[i]);
  for (int k = 0; k < SP_NCH; ++k)
    if (!is_fin(p->weights[k])) return fail(SP_EINVAL, "weight %d is not finite", k);
  if (!is_fin(p->q) || !is_fin(p->r) || p->q < 0 || p->r < 0 || !(p->q + p->r > 0))
    return fail(SP_EINVAL, "Kalman variances must be finite, >= 0 and not both 0 (q=%g r=%g)", p->q, p->r);
  if (!is_fin(p->eps) || !(p->eps > 0.f) || !(p->eps < 0.5f)) return fail(SP_EINVAL, "eps must be in (0, 0.5)");
  if (p->border < 0) return fail(SP_EINVAL, "border must be >= 0");
  if (!is_fin(p->lambda) || p->lambda < 0 || !is_fin(p->potts) || p->potts < 0)
    return fail(SP_EINVAL, "lambda and potts must be finite and >= 0");
  if (p->lm_block != 8) return fail(SP_EINVAL, "lm_block must be 8 (got %d)", p->lm_block);
  if (!is_fin(p->flat_tol) || p->flat_tol < 0) return fail(SP_EINVAL, "flat_tol must be finite and >= 0");
  if (!is_fin(p->gabor_lambda) || !(p->gabor_lambda > 0) || !is_fin(p->gabor_sigma) || !(p->gabor_sigma > 0))
    return fail(SP_EINVAL, "Gabor wavelength and sigma must be finite and > 0");
  if (p->gabor_radius < 1 || p->gabor_radius > SP_MAXR) return fail(SP_EINVAL, "gabor_radius must be 1..%d", SP_MAXR);
  if (p->record_tape < 0 || p->record_tape > (1 << 20)) return fail(SP_EINVAL, "record_tape must be 0..2^20");
  if (p->f_mode != 0 && p->f_mode != 1) return fail(SP_EINVAL, "f_mode must be 0 (blur) or 1 (distance transform)");
  if (!is_fin(p->dt_sigma) || !(p->dt_sigma > 0.f) || p->dt_sigma > 4.f)
    return fail(SP_EINVAL, "dt_sigma must be in (0, 4]");
  if (!is_fin(p->ssm_q) || !is_fin(p->ssm_r) || p->ssm_q < 0 || p->ssm_r < 0)
    return fail(SP_EINVAL, "ssm_q and ssm_r must be finite and >= 0");
  if (p->gmm_components < 0 || p->gmm_components > SP_GMM_MAXM)
    return fail(SP_EINVAL, "gmm_components must be 0..%d", SP_GMM_MAXM);
  if (p->gmm_iters < 0 || p->gmm_iters > 100) return fail(SP_EINVAL, "gmm_iters must be 0..100");
  if (!is_fin(p->gmm_reg) || p->gmm_reg < 0) return fail(SP_EINVAL, "gmm_reg must be finite and >= 0");
  if (p->record_tape > 0 && (p->f_mode != 0 || p->ssm_r > 0))
    return fail(SP_EINVAL, "the adjoint covers the default prior only: record_tape needs f_mode 0 and ssm_r 0");
  return SP_OK;
}

int make_geo(const sp_params& p, int H, int W, Geo& g) {
  if (H < 1 || W < 1) return fail(SP_ESHAPE, "frame must be at least 1x1 (got %dx%d)", H, W);
  if ((long long)H * W > (1LL << 28) || H > 65535 || W > 65535)
    return fail(SP_ESHAPE, "frame %dx%d exceeds the 2^28-pixel / 65535-edge limit", H, W);
  g.H = H;
  g.W = W;
  int D = p.depth;
  if (D <= 0) {
    int m = std::min(H, W), lg = 0;
    while ((2 << lg) <= m) ++lg;   // floor(log2 m)
    D = lg - 1;
  }
  if (D < 1) return fail(SP_ESHAPE, "frame %dx%d too small for a pyramid", H, W);
  if (D > SP_MAX_LEVELS) return fail(SP_ESHAPE, "pyramid depth %d exceeds %d", D, SP_MAX_LEVELS);
  g.depth = D;
  g.Hl[0] = H;
  g.Wl[0] = W;
  for (int l = 1; l <= D; ++l) {
    g.Hl[l] = (g.Hl[l - 1] + 1) / 2;
    g.Wl[l] = (g.Wl[l - 1] + 1) / 2;
  }
  g.n_pairs = 0;
  g.c_min = 1 << 30;
  g.c_max = -1;
  g.top = 0;
  for (int i = 0; i < p.n_centers; ++i)
    for (int j = 0; j < p.n_deltas; ++j) {
      const int c = p.centers[i], s = c + p.deltas[j];
      if (s > D) continue;
      if (g.n_pairs >= SP_MAXP) return fail(SP_EINVAL, "more than %d centre-surround pairs", SP_MAXP);
      g.pc[g.n_pairs] = c;
      g.ps[g.n_pairs] = s;
      ++g.n_pairs;
      g.c_min = std::min(g.c_min, c);
      g.c_max = std::max(g.c_max, c);
      g.top = std::max(g.top, s);
      g.used |= (1u << c) | (1u << s);
    }
  if (g.n_pairs == 0) return fail(SP_ESHAPE, "no centre-surround pair fits pyramid depth %d", D);
  if (g.c_max - g.c_min > 2)
    return fail(SP_ESHAPE, "centre levels may span at most 2 octaves (got %d..%d)", g.c_min, g.c_max);
  for (int a = 0; a < g.n_pairs; ++a)
    for (int b = 0; b < a; ++b)
      if (g.pc[a] == g.pc[b] && g.ps[a] == g.ps[b]) return fail(SP_EINVAL, "duplicate centre-surround pair");
  const size_t ca_lds = gpath_ok(g) ? csg_lds_bytes(g) : csapply_lds_bytes(g);
  if (ca_lds > kMaxDynLds)
    return fail(SP_ESHAPE, "centre-surround configuration needs %zu bytes of LDS per workgroup (max %zu)", ca_lds,
                kMaxDynLds);
  return SP_OK;
}

int ntiles(int h, int w) { return ((h + kTile - 1) / kTile) * ((w + kTile - 1) / kTile); }

void add_tiles(std::vector<Job>& v, int stream, int a, int h, int w, int kind = 0) {
  int tid = 0;
  for (int y0 = 0; y0 < h; y0 += kTile)
    for (int x0 = 0; x0 < w; x0 += kTile)
      v.push_back(Job{stream, a, y0, x0, std::min(kTile, h - y0), std::min(kTile, w - x0), tid++, kind});
}

void add_tiles_wh(std::vector<Job>& v, int stream, int a, int h, int w, int th, int tw, int kind) {
  int tid = 0;
  for (int y0 = 0; y0 < h; y0 += th)
    for (int x0 = 0; x0 < w; x0 += tw)
      v.push_back(Job{stream, a, y0, x0, std::min(th, h - y0), std::min(tw, w - x0), tid++, kind});
}

// Tuning knobs that never change results: the width of the level-0 update tiles and
// the XCD-aware order of the job tables.
struct Tune {
  int kalman_tw = 32;   // 16, 32 or 64
  bool xcd = false;
  int ca_nc = 2;        // channels per workgroup of the across-scale sum: 1, 2, 4 or 8
};

// Choices of the autotuner per resolution, reused by later contexts and batches.
std::map<std::pair<int, int>, int>& tune_cache_tw() {
  static std::map<std::pair<int, int>, int> m;
  return m;
}
bool& tune_cache_xcd() {
  static bool x = false;
  return x;
}
int& tune_cache_nc() {
  static int nc = 2;
  return nc;
}
std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
Tune cached_tune(int H, int W) {
  std::lock_guard<std::mutex> lk(tune_mutex());
  Tune t;
  auto it = tune_cache_tw().find({H, W});
  if (it != tune_cache_tw().end()) t.kalman_tw = it->second;
  t.xcd = tune_cache_xcd();
  t.ca_nc = tune_cache_nc();
  return t;
}

// Channels per workgroup of the across-scale sum: the largest power of two up to the
// preference whose LDS (one block per channel) fits the dynamic limit.
int csapply_nc(const Geo& g, int pref) {
  const size_t per = gpath_ok(g) ? csg_lds_bytes(g) : csapply_lds_bytes(g);
  int nc = 8;
  while (nc > 1 && (nc > pref || nc * per > kMaxDynLds)) nc /= 2;
  return nc;
}

// Reorders a launch's jobs so that workgroups dispatched round-robin over the 8 XCDs
// get contiguous runs of tiles (neighbouring tiles share halos in that XCD's L2).
void xcd_order(std::vector<Job>& v) {
  const size_t n = v.size();
  if (n < 16) return;
  std::vector<Job> out;
  out.reserve(n);
  std::vector<size_t> start(9);
  for (int x = 0; x <= 8; ++x) start[x] = n * x / 8;
  for (size_t k = 0;; ++k) {
    bool any = false;
    for (int x = 0; x < 8; ++x)
      if (start[x] + k < start[x + 1]) {
        out.push_back(v[start[x] + k]);
        any = true;
      }
    if (!any) break;
  }
  v.swap(out);
}

// Source level of the tail job: the first level >= lo from which every higher level
// (and the Gabor maps of the used ones) fits the LDS buffers of one workgroup.
int tail_source(const Geo& g, int lo) {
  auto sz = [&](int l) { return (long long)g.Hl[l] * g.Wl[l]; };
  for (int L0 = lo; L0 < g.top; ++L0) {
    bool ok = sz(L0) <= SP_TAIL_SRC;
    for (int l = L0 + 1; ok && l <= g.top; ++l) {
      const bool odd = (l - L0) & 1;   // level l in the second buffer, level l-1 in the first
      ok &= sz(l) <= (odd ? SP_TAIL_ALT : SP_TAIL_SRC);
      ok &= (long long)g.Hl[l - 1] * g.Wl[l] <= SP_TAIL_HB;
      if (g.used & (1u << l)) ok &= 4 * sz(l) <= (odd ? SP_TAIL_SRC : SP_TAIL_ALT);
    }
    if (ok) return L0;
  }
  return g.top;
}

// Pyramid stages of one stream above level lo (level lo already computed):
// DOWN(j -> j+1) + GABOR(j) for j < L0, then TAIL(L0) + GABOR(L0).
// Returns the middle stages and the final stage; *big says whether it has tail jobs.
void pyramid_stages(const Geo& g, int s, int lo, std::vector<std::vector<Job>>& mid, std::vector<Job>& fin,
                    bool* big) {
  const int L0 = tail_source(g, lo);
  mid.clear();
  fin.clear();
  for (int j = lo; j < L0; ++j) {
    std::vector<Job> v;   // Gabor tiles (the longer jobs) first, then the next level's tiles
    if (g.used & (1u << j)) add_tiles_wh(v, s, j, g.Hl[j], g.Wl[j], 16, 32, JOB_GABOR);
    add_tiles(v, s, j, g.Hl[j + 1], g.Wl[j + 1], JOB_DOWN);
    mid.push_back(std::move(v));
  }
  *big = L0 < g.top;
  if (*big) {
    for (int l = g.top; l > L0; --l)   // Gabor maps of the small used levels, in row bands of ~256 pixels
      if (g.used & (1u << l)) {
        const int nb = std::max(1, std::min(8, g.Hl[l] * g.Wl[l] / 256));
        const int rows = (g.Hl[l] + nb - 1) / nb;
        for (int y0 = 0; y0 < g.Hl[l]; y0 += rows)
          fin.push_back(Job{s, L0, y0, 0, std::min(rows, g.Hl[l] - y0), g.Wl[l], l, JOB_TAILGAB});
      }
    for (int ch = 0; ch < 4; ++ch) fin.push_back(Job{s, L0, 0, 0, g.Hl[L0], g.Wl[L0], ch, JOB_TAIL});
  }
  if (g.used & (1u << L0)) add_tiles_wh(fin, s, L0, g.Hl[L0], g.Wl[L0], 16, 32, JOB_GABOR);
}

// ---------------------------------------------------------------- device memory layout
struct Bump {
  char* base = nullptr;   // null during the sizing pass
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Colour-statistics tiles: rows x columns, at most SP_RGB_TR x SP_RGB_TC, with the
// row count lowered (down to 2) while a frame would give fewer than min_tiles workgroups.
struct RgbTiling {
  int tr, tc, nrt, nct;
  int count() const { return nrt * nct; }
};

RgbTiling rgb_tiling(const Geo& g, int min_tiles = 192) {
  RgbTiling t;
  t.nct = (g.W + SP_RGB_TC - 1) / SP_RGB_TC;
  t.tc = (((g.W + t.nct - 1) / t.nct) + 3) & ~3;   // tiles start at multiples of 4 columns
  t.nct = (g.W + t.tc - 1) / t.tc;
  t.tr = SP_RGB_TR;
  while (t.tr > 2 && ((g.H + t.tr - 1) / t.tr) * t.nct < min_tiles) t.tr /= 2;
  t.nrt = (g.H + t.tr - 1) / t.tr;
  return t;
}

void fill_taps(StreamDesc& sd, const sp_params& p) {
  const int R = p.gabor_radius;
  const double s2 = 2.0 * (double)p.gabor_sigma * (double)p.gabor_sigma;
  const double k = 2.0 * M_PI / (double)p.gabor_lambda;
  const double alpha = k * std::cos(M_PI / 4.0);
  double g[2 * SP_MAXR + 1], sg = 0, sgc = 0;
  for (int u = -R; u <= R; ++u) {
    g[u + R] = std::exp(-(double)(u * u) / s2);
    sg += g[u + R];
    sgc += g[u + R] * std::cos(k * u);
  }
  const double c0 = sgc / sg;
  double sc = 0, ss = 0;
  for (int u = -R; u <= R; ++u) {
    sc += g[u + R] * std::cos(alpha * u);
    ss += g[u + R] * std::sin(alpha * u);
  }
  for (int u = -R; u <= R; ++u) {
    const double gu = g[u + R];
    sd.gf[0][u + R] = (float)gu;
    sd.gf[1][u + R] = (float)(gu * (std::cos(k * u) - c0));
    sd.gf[2][u + R] = (float)(gu * std::cos(alpha * u));
    sd.gf[3][u + R] = (float)(gu * std::sin(alpha * u));
  }
  sd.c45 = (float)((sc * sc - ss * ss) / (sg * sg));
  sd.gr = R;
}

// Fills the geometry/parameter part of a stream description and takes its scratch
// from `bump`.  Levels below `first_level` get no base storage (level c_min of a
// recompute stream reads its checkpoint instead).
void layout_stream(StreamDesc& sd, const Geo& g, const sp_params& p, Bump& bump, int first_level, bool rgb_parts,
                   int rgb_min_tiles = 192) {
  std::memset(&sd, 0, sizeof sd);
  sd.H = g.H;
  sd.W = g.W;
  sd.top = g.top;
  sd.c_min = g.c_min;
  sd.c_max = g.c_max;
  sd.n_pairs = g.n_pairs;
  sd.border = p.border;
  for (int i = 0; i < g.n_pairs; ++i) {
    sd.pc[i] = g.pc[i];
    sd.ps[i] = g.ps[i];
  }
  for (int l = 0; l < SP_MAXL; ++l) {
    sd.Hl[l] = g.Hl[l];
    sd.Wl[l] = g.Wl[l];
    sd.ntiles_lvl[l] = (l <= g.depth) ? ntiles(g.Hl[l], g.Wl[l]) : 0;
  }
  sd.n_cmax_tiles = sd.ntiles_lvl[g.c_max];
  sd.gpath = gpath_ok(g) ? 1 : 0;
  int off = 0;
  for (int i = 0; i < g.n_pairs; ++i) {
    // partials per map: one per c_max tile (reduced-map path) or per centre-level tile
    sd.cs_nt[i] = sd.gpath ? sd.n_cmax_tiles : sd.ntiles_lvl[g.pc[i]];
    sd.cs_off[i] = off;
    off += SP_NCH * sd.cs_nt[i];
  }
  sd.used = g.used;
  for (int k = 0; k < SP_NCH; ++k) sd.w[k] = p.weights[k];
  sd.eps = p.eps;
  sd.flat_tol = p.flat_tol;
  sd.lam = p.lambda;
  sd.potts = p.potts;
  sd.dt_r = std::min(SP_DT_RMAX, (int)std::ceil(std::sqrt(176.0) * (double)p.dt_sigma));
  sd.dt_k = (float)(-1.0 / (2.0 * (double)p.dt_sigma * (double)p.dt_sigma * std::log(2.0)));
  fill_taps(sd, p);
  for (int l = std::max(1, first_level); l <= g.top; ++l)
    sd.base[l] = bump.take<float>((size_t)4 * g.Hl[l] * g.Wl[l]);
  for (int l = 1; l <= g.top; ++l)
    if (g.used & (1u << l)) sd.gab[l] = bump.take<float>((size_t)4 * g.Hl[l] * g.Wl[l]);
  if (rgb_parts) {
    const RgbTiling t = rgb_tiling(g, rgb_min_tiles);
    sd.n_rgb = t.count();
    sd.rgb_tr = t.tr;
    sd.rgb_max_part = bump.take<uint32_t>(sd.n_rgb);
    sd.rgb_d2_part = bump.take<unsigned long long>(sd.n_rgb);
  }
  sd.cs_part = bump.take<float>((size_t)3 * off);
  sd.fbar = bump.take<float>((size_t)SP_NCH * g.Hl[g.c_max] * g.Wl[g.c_max]);
  sd.fbar_part = bump.take<float>((size_t)3 * SP_NCH * sd.n_cmax_tiles);
  sd.s_part = bump.take<float>((size_t)2 * sd.n_cmax_tiles);
  sd.cs_np = bump.take<float>((size_t)4 * SP_NCH * std::max(1, g.n_pairs));
  if (sd.gpath) sd.gmap = bump.take<float>((size_t)g.n_pairs * SP_NCH * g.Hl[g.c_max] * g.Wl[g.c_max]);
}

void rgb_jobs(std::vector<Job>& v, int s, const StreamDesc& sd, const Geo& g) {
  RgbTiling t = rgb_tiling(g);
  t.tr = sd.rgb_tr;   // the tiling chosen when the partials were laid out
  t.nrt = (g.H + t.tr - 1) / t.tr;
  if (t.count() != sd.n_rgb) throw std::logic_error("colour tiling and partial buffer disagree");
  for (int i = 0; i < t.nrt; ++i)
    for (int j = 0; j < t.nct; ++j) {
      const int y0 = i * t.tr, x0 = j * t.tc;
      v.push_back(Job{s, i * t.nct + j, y0, x0, std::min(t.tr, g.H - y0), std::min(t.tc, g.W - x0),
                      i * t.nct + j, JOB_RGB});
    }
}

// ---------------------------------------------------------------- job tables
struct Phase {
  int kind = 0, flag = 0;
  size_t lds = 0;             // dynamic LDS bytes of the launch
  size_t off = 0;             // first job in the device table
  int n = 0;                  // jobs
  std::vector<int> upto;      // upto[s]: jobs of streams < s (stream-major tables)
};

struct JobStore {
  std::vector<Job> host;
  Job* dev = nullptr;
  size_t cap = 0;   // jobs the device buffer holds
  Phase add(int kind, int flag, const std::vector<Job>& jobs, int n_streams) {
    Phase ph;
    ph.kind = kind;
    ph.flag = flag;
    ph.off = host.size();
    ph.n = (int)jobs.size();
    ph.upto.assign(n_streams + 1, 0);
    for (const Job& j : jobs) ph.upto[j.stream + 1]++;
    for (int s = 0; s < n_streams; ++s) ph.upto[s + 1] += ph.upto[s];
    host.insert(host.end(), jobs.begin(), jobs.end());
    return ph;
  }
};

// Uploads the host job table, growing the device buffer when needed (set-up calls only).
int upload_jobs(JobStore& js, hipStream_t st) {
  const size_t n = std::max<size_t>(1, js.host.size());
  if (n > js.cap) {
    if (js.dev) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(js.dev);
      js.dev = nullptr;
      js.cap = 0;
    }
    if (hipMalloc(&js.dev, sizeof(Job) * n) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SP_ENOMEM, "hipMalloc of the job tables failed");
    }
    js.cap = n;
  }
  HIPCHK(hipMemcpyAsync(js.dev, js.host.data(), sizeof(Job) * js.host.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return SP_OK;
}

// Per-stream phase program of the forward saliency map.
enum ProgPart { PROG_ALL, PROG_RECOMPUTE };

double now_gain(int64_t t, double Pprev, double Q, double R, double* P) {
  if (t == 0) {
    *P = R;
    return 1.0;
  }
  const double a = Pprev + Q;
  const double K = a / (a + R);
  *P = R * K;
  return K;
}

}  // namespace

// ---------------------------------------------------------------- measurement hook
// One pair of events per launch, recorded on the launch stream.
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> ev;   // pairs
  std::vector<int> kind;
  size_t used = 0;
  int enable(bool en) {
    if (en && ev.empty()) {
      const size_t pairs = 65536;
      ev.assign(2 * pairs, nullptr);
      for (size_t i = 0; i < ev.size(); ++i) HIPCHK(hipEventCreate(&ev[i]));
      kind.assign(pairs, 0);
    }
    on = en;
    used = 0;
    return SP_OK;
  }
  template <class F>
  hipError_t timed(hipStream_t st, int k, F&& launch) {
    const bool rec = on && used < kind.size();
    if (rec) (void)hipEventRecord(ev[2 * used], st);
    hipError_t e = launch();
    if (rec) {
      (void)hipEventRecord(ev[2 * used + 1], st);
      kind[used++] = k;
    }
    return e;
  }
  int read(hipStream_t st, int n, float* total_ms, int32_t* launches) {
    if (!total_ms || !launches) return fail(SP_EINVAL, "NULL argument");
    if (n < SP_NKINDS) return fail(SP_EINVAL, "arrays must hold %d kinds", SP_NKINDS);
    for (int k = 0; k < n; ++k) {
      total_ms[k] = 0.f;
      launches[k] = 0;
    }
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < used; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      if (kind[i] >= 0 && kind[i] < n) {
        total_ms[kind[i]] += ms;
        launches[kind[i]] += 1;
      }
    }
    used = 0;
    return SP_OK;
  }
  void destroy() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  }
};

// ---------------------------------------------------------------- context
struct sp_ctx {
  sp_params p{};
  Geo g;
  hipStream_t stream = nullptr;
  int device = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  StreamDesc h_sd{};
  StreamDesc* d_sd = nullptr;
  JobStore jobs;
  std::vector<Phase> fwd, prior, mrf, bwd;
  // Kalman state
  int64_t t = 0;
  double P = 0.0;
  float* pi_state[2] = {nullptr, nullptr};
  int cur = 0;
  // tape
  int cap = 0;
  int64_t tape_valid_from = 0;   // tape covers steps since the last reset only
  bool tape_ok = true;
  int64_t tape_gen = 0;           // bumped whenever the recorded clip stops being the current one
  float* ckpt = nullptr;          // [cap][4][Hcmin][Wcmin]
  float* S_tape = nullptr;        // [cap][Hc][Wc]
  float* f_tape = nullptr;        // [cap][H][W]
  float* ms_tape = nullptr;       // [cap][2]
  double* K_tape = nullptr;       // [cap]
  double* P_tape = nullptr;       // [cap]
  std::vector<float> Kf;          // host copy of K_t (float) per recorded step
  std::vector<char> uses_pi;      // step t read the previous prior
  // adjoint workspace
  float* nu[2] = {nullptr, nullptr};
  float* gu = nullptr;
  float* gs_all = nullptr;        // [cap][Hc][Wc]
  float* gk_part = nullptr;       // [cap][n_lvl0_tiles]
  float* dot_part = nullptr;      // [cap][n_cmax_tiles][8]
  float* cx = nullptr;            // [cap][8]
  double* gK_scratch = nullptr;   // [cap] dL/dK_t, then [cap][8] the steps' shares of dL/dw
  int n_lvl0_tiles = 0;
  int CH = 0;                     // frames per recompute chunk
  StreamDesc* d_rsd = nullptr;    // [CH] recompute streams
  StepIO* d_rio = nullptr;        // [cap] io of every tape frame (checkpoint and adjoint buffers)
  std::vector<Phase> rec;         // recompute phases (stream-major, CH streams)
  float* S_scratch = nullptr;     // [Hc][Wc] saliency map of the autotuner's steps
  // variants of the prior
  float* f_map = nullptr;         // [H][W] distance-transform prediction (f_mode 1)
  std::vector<Phase> dt;          // its launch
  float* ssm[2] = {nullptr, nullptr};   // [Hc][Wc] stochastic saliency means (ping-pong)
  int ssm_cur = 0;
  int64_t ssm_t = 0;              // maps filtered since the reset
  double ssm_P = 0.0;             // variance of the stochastic map
  // pixel-level adjoint (contexts with a tape): workspace planes and static launch tables
  struct PixAdj {
    float* gS = nullptr;                 // [Hc][Wc] dL/dS of the frame
    float* gfbar = nullptr;              // [8][Hc][Wc]
    double* gs_part = nullptr;           // per-workgroup partials of sum gs S
    float* gN[SP_MAXL] = {};             // [8][H_l][W_l] dL/dN(F) at centre levels below c_max
    float* F[SP_MAXP] = {};              // [8][H_c][W_c] per pair: F, then dL/dF, then sign(D) dL/dF
    float* gX[SP_MAXL] = {};             // [8][H_l][W_l] dL/d(channel maps) per level 0..top
    size_t gX_floats = 0;                // floats of gX, followed by amax
    uint32_t* amax = nullptr;            // [n_pairs][8][SP_PA_AMAX] scale of each centre-surround pair (float bits)
    float* taps = nullptr;               // [4][2R+1][2R+1] Gabor taps
    PaMap* maps_fbar = nullptr;          // [8]
    PaMap* maps_F = nullptr;             // [8 n_pairs]
    PaPlane* tab_gn[SP_MAXL] = {};       // [8] per centre level below c_max
    PaPlane* tab_cs[SP_MAXP] = {};       // [8] per pair: centre-surround map and adjoint
    PaPlane* tab_up[SP_MAXP] = {};       // [8] per pair: up-sample transpose
    PaPlane* tab_gab[SP_MAXL] = {};      // [1] per used level
    PaPlane* tab_pyr[SP_MAXL] = {};      // [4] per level 1..top: to the level below
    float** gc[SP_MAXP] = {};            // [8] per pair: dL/dX(c) planes
    // pairs grouped so that no two of a group share a centre level (cs: the adjoint adds to
    // dL/dX(c)) or a surround level (up: the transpose adds to dL/dX(s)); each group's
    // tables are contiguous, the cs groups one after another, so one launch covers a group
    // (cs maps: every pair)
    int cs_first[SP_MAXP] = {}, cs_count[SP_MAXP] = {}, n_cs = 0;   // pair index of the first table, pairs
    int up_first[SP_MAXP] = {}, up_count[SP_MAXP] = {}, n_up = 0;
    int cs_order[SP_MAXP] = {}, up_order[SP_MAXP] = {};              // pairs in table order
    int64_t gen = -1;                    // tape generation of the last saliency_backward
    int T = 0;                           // and its clip length
  } pa;
  int32_t* pa_bpos = nullptr;     // block-maximum positions of every N(.) adjoint map
  float* pa_sc = nullptr;         // [maps][8] scalars of every N(.) adjoint map
  float2* pa_mm = nullptr;        // [maps][mm] (min, max) partials of every N(.) adjoint map
  PaStrip* pa_strip = nullptr;    // [maps][strips] strip partials of every N(.) adjoint map
  // colour likelihood
  GmmState* gmm_state = nullptr;
  double* gmm_part = nullptr;     // [2 M 10][gmm_tiles] FP64 moments per tile
  int gmm_tiles = 0;
  // loss helper
  float* loss_part = nullptr;
  int loss_nblk = 1024;
  Profiler prof;
  Tune tune;
};

namespace {

int ctx_build_tables(sp_ctx* c);

// Brackets a launch with a pair of events when the measurement hook is on.
template <class F>
hipError_t timed(sp_ctx* c, int kind, F&& launch) {
  return c->prof.timed(c->stream, kind, launch);
}

int run_phase(sp_ctx* c, const Phase& ph, const StreamDesc* sds, const StepIO* ios, const StepIO* io0, int n_jobs,
              const float* aux = nullptr) {
  hipError_t e = timed(c, ph.kind, [&] {
    return sp_launch(ph.kind, c->jobs.dev + ph.off, n_jobs, sds, ios, io0, ph.flag, aux, c->stream, ph.lds);
  });
  if (e != hipSuccess) return fail(SP_EHIP, "kernel launch (phase kind %d): %s", ph.kind, hipGetErrorString(e));
  return SP_OK;
}

void build_forward_jobs(std::vector<std::vector<Job>>& parts, std::vector<int>& kinds, const StreamDesc& sd,
                        const Geo& g, int s, ProgPart which, int nc) {
  auto push = [&](int kind, std::vector<Job> v) {
    parts.push_back(std::move(v));
    kinds.push_back(kind);
  };
  if (which == PROG_ALL) {
    std::vector<Job> v;
    rgb_jobs(v, s, sd, g);
    push(JOB_RGB, v);
    v.clear();
    add_tiles(v, s, 1, g.Hl[1], g.Wl[1], JOB_FEAT);
    push(JOB_FEAT, v);
  }
  const int from = (which == PROG_ALL) ? 1 : g.c_min;
  std::vector<std::vector<Job>> mid;
  std::vector<Job> fin;
  bool big = false;
  pyramid_stages(g, s, from, mid, fin, &big);
  for (auto& m : mid) push(JOB_DOWN, m);
  if (!fin.empty()) push(big ? JOB_TAIL : JOB_DOWN, fin);
  std::vector<Job> v;
  const bool gp = gpath_ok(g);
  if (gp) {
    for (int k = 0; k < SP_NCH; k += nc) add_tiles(v, s, k, g.Hl[g.c_max], g.Wl[g.c_max], JOB_CSG);
    push(JOB_CSG, v);
  } else {
    for (int c = 0; c <= g.top; ++c) {
      bool has = false;
      for (int i = 0; i < g.n_pairs; ++i) has |= (g.pc[i] == c);
      if (has) add_tiles(v, s, c, g.Hl[c], g.Wl[c]);
    }
    push(JOB_CSSTATS, v);
  }
  v.clear();
  if (!gp) {   // the reduced-map path's mix computes the N parameters itself
    for (int p = 0; p < g.n_pairs; ++p) v.push_back(Job{s, p, 0, 0, 1, 1, p, JOB_CSFINAL});
    push(JOB_CSFINAL, v);
  }
  v.clear();
  if (gp) {
    add_tiles(v, s, 0, g.Hl[g.c_max], g.Wl[g.c_max], JOB_CSMIX);
    push(JOB_CSMIX, v);
  } else {
    for (int k = 0; k < SP_NCH; k += nc) add_tiles(v, s, k, g.Hl[g.c_max], g.Wl[g.c_max]);
    push(JOB_CSAPPLY, v);
  }
  v.clear();
  add_tiles(v, s, 0, g.Hl[g.c_max], g.Wl[g.c_max]);
  push(which == PROG_ALL ? JOB_CONSP : JOB_CONSP_DOT, v);
}

// 8x8 blocks of every map of the N(.) adjoint: the 8 across-scale sums and every pair's 8
// centre-surround maps.
size_t pixadj_nblocks(const Geo& g) {
  auto nblk = [&](int l) { return (size_t)((g.Hl[l] + 7) / 8) * ((g.Wl[l] + 7) / 8); };
  size_t n = SP_NCH * nblk(g.c_max);
  for (int p = 0; p < g.n_pairs; ++p) n += SP_NCH * nblk(g.pc[p]);
  return n;
}

// Largest N(.) adjoint map (pixels, rows) and the partials each map gets.
struct PaDims {
  int maxn, maxh;
  size_t mm, strips;
};
PaDims pixadj_dims(const Geo& g) {
  PaDims D{g.Hl[g.c_max] * g.Wl[g.c_max], g.Hl[g.c_max], 0, 0};
  for (int p = 0; p < g.n_pairs; ++p) {
    D.maxn = std::max(D.maxn, g.Hl[g.pc[p]] * g.Wl[g.pc[p]]);
    D.maxh = std::max(D.maxh, g.Hl[g.pc[p]]);
  }
  D.mm = (size_t)(D.maxn + SP_PA_MMT - 1) / SP_PA_MMT;
  D.strips = (size_t)(D.maxh + 7) / 8;
  return D;
}

// Workspace of the pixel-level adjoint, taken from the context's arena (both layout passes).
void pixadj_layout(sp_ctx* c, Bump& b) {
  const Geo& g = c->g;
  auto& A = c->pa;
  auto n_l = [&](int l) { return (size_t)g.Hl[l] * g.Wl[l]; };
  const int Hc = g.Hl[g.c_max], Wc = g.Wl[g.c_max];
  A.gS = b.take<float>((size_t)Hc * Wc);
  A.gs_part = b.take<double>(((size_t)Hc * Wc + SP_BLOCK - 1) / SP_BLOCK);
  A.gfbar = b.take<float>((size_t)SP_NCH * Hc * Wc);
  for (int l = g.c_min; l < g.c_max; ++l) A.gN[l] = b.take<float>(SP_NCH * n_l(l));
  for (int p = 0; p < g.n_pairs; ++p) A.F[p] = b.take<float>(SP_NCH * n_l(g.pc[p]));
  A.gX_floats = 0;
  for (int l = 0; l <= g.top; ++l) A.gX_floats += SP_NCH * n_l(l);
  float* gx = b.take<float>(A.gX_floats + (size_t)SP_NCH * g.n_pairs * SP_PA_AMAX);
  for (int l = 0; l <= g.top; ++l) {
    A.gX[l] = gx;
    if (gx) gx += SP_NCH * n_l(l);
  }
  A.amax = reinterpret_cast<uint32_t*>(gx);
  const int K = 2 * SP_PA_R + 1;
  A.taps = b.take<float>((size_t)4 * K * K);
  A.maps_fbar = b.take<PaMap>(SP_NCH);
  A.maps_F = b.take<PaMap>((size_t)SP_NCH * g.n_pairs);
  for (int l = g.c_min; l < g.c_max; ++l) A.tab_gn[l] = b.take<PaPlane>(SP_NCH);
  {
    // group round r: the pairs that are the r-th of their centre (surround) level
    auto groups = [&](bool by_surround, int* order, int* first, int* count, int& ng) {
      int round[SP_MAXP], nr = 0, k = 0;
      for (int p = 0; p < g.n_pairs; ++p) {
        int r = 0;
        for (int q = 0; q < p; ++q) r += (by_surround ? g.ps[q] == g.ps[p] : g.pc[q] == g.pc[p]) ? 1 : 0;
        round[p] = r;
        nr = std::max(nr, r + 1);
      }
      ng = nr;
      for (int r = 0; r < nr; ++r) {
        first[r] = k;
        count[r] = 0;
        for (int p = 0; p < g.n_pairs; ++p)
          if (round[p] == r) {
            order[k++] = p;
            ++count[r];
          }
      }
    };
    groups(false, A.cs_order, A.cs_first, A.cs_count, A.n_cs);
    groups(true, A.up_order, A.up_first, A.up_count, A.n_up);
    PaPlane* cs = b.take<PaPlane>((size_t)SP_NCH * g.n_pairs);
    PaPlane* up = b.take<PaPlane>((size_t)SP_NCH * g.n_pairs);
    float** gc = b.take<float*>((size_t)SP_NCH * g.n_pairs);
    for (int k = 0; k < g.n_pairs; ++k) {
      const int pc = A.cs_order[k], pu = A.up_order[k];
      A.tab_cs[pc] = cs ? cs + (size_t)k * SP_NCH : nullptr;
      A.gc[pc] = gc ? gc + (size_t)k * SP_NCH : nullptr;
      A.tab_up[pu] = up ? up + (size_t)k * SP_NCH : nullptr;
    }
  }
  for (int l = 1; l <= g.top; ++l) {
    if (g.used & (1u << l)) A.tab_gab[l] = b.take<PaPlane>(1);
    A.tab_pyr[l] = b.take<PaPlane>(4);
  }
  c->pa_bpos = b.take<int32_t>(pixadj_nblocks(g) + 64);
  c->pa_sc = b.take<float>((size_t)SP_PA_SC * SP_NCH * (1 + g.n_pairs));
  const size_t nmaps = (size_t)SP_NCH * (1 + g.n_pairs);
  const PaDims D = pixadj_dims(g);
  c->pa_mm = b.take<float2>(nmaps * D.mm);
  c->pa_strip = b.take<PaStrip>(nmaps * D.strips);
}

// Static launch tables of the pixel-level adjoint (pointers into the forward's own maps and
// the workspace; every frame reuses them).
hipError_t pixadj_upload(sp_ctx* c) {
  const Geo& g = c->g;
  const StreamDesc& sd = c->h_sd;
  auto& A = c->pa;
  auto n_l = [&](int l) { return (size_t)g.Hl[l] * g.Wl[l]; };
  const int cm = g.c_max;
  // channel k of level l in the forward's maps (I, RG, BY, O0..O135, M)
  auto chan = [&](int k, int l) -> const float* {
    if (k == 0) return sd.base[l];
    if (k == 1 || k == 2) return sd.base[l] + (size_t)k * n_l(l);
    if (k == 7) return sd.base[l] + (size_t)BASE_M * n_l(l);
    return sd.gab[l] + (size_t)(k - 3) * n_l(l);
  };
  std::vector<char> blob;
  std::vector<std::pair<void*, std::vector<char>>> ups;
  auto put = [&](void* dst, const void* src, size_t bytes) {
    ups.emplace_back(dst, std::vector<char>((const char*)src, (const char*)src + bytes));
  };
  // Gabor taps, the 2-D kernel of each orientation in FP64, stored FP32
  {
    const int R = c->p.gabor_radius, K = 2 * SP_PA_R + 1;
    std::vector<float> taps((size_t)4 * K * K, 0.f);
    const double s2 = 2.0 * (double)c->p.gabor_sigma * (double)c->p.gabor_sigma;
    for (int th = 0; th < 4; ++th) {
      const double a = th * M_PI / 4.0;
      double se = 0, sec = 0;
      for (int v = -R; v <= R; ++v)
        for (int u = -R; u <= R; ++u) {
          const double e = std::exp(-(double)(u * u + v * v) / s2);
          se += e;
          sec += e * std::cos(2.0 * M_PI * (u * std::cos(a) + v * std::sin(a)) / (double)c->p.gabor_lambda);
        }
      const double c0 = sec / se;
      for (int v = -R; v <= R; ++v)
        for (int u = -R; u <= R; ++u) {
          const double e = std::exp(-(double)(u * u + v * v) / s2);
          const double h = e * std::cos(2.0 * M_PI * (u * std::cos(a) + v * std::sin(a)) / (double)c->p.gabor_lambda) - c0 * e;
          taps[((size_t)th * K + (v + R)) * K + (u + R)] = (float)h;
        }
    }
    put(A.taps, taps.data(), taps.size() * sizeof(float));
  }
  // N(.) adjoint maps: the 8 across-scale sums, then every pair's 8 centre-surround maps
  int32_t* bpos = c->pa_bpos;
  float* sc = c->pa_sc;
  float2* mm = c->pa_mm;
  PaStrip* strip = c->pa_strip;
  const PaDims D = pixadj_dims(g);
  auto nblk = [&](int l) { return ((g.Hl[l] + 7) / 8) * ((g.Wl[l] + 7) / 8); };
  {
    std::vector<PaMap> m(SP_NCH);
    const size_t pl = n_l(cm);
    for (int k = 0; k < SP_NCH; ++k) {
      m[k] = PaMap{sd.fbar + k * pl, A.gS, A.gfbar + k * pl, bpos, sc, mm, strip, g.Hl[cm], g.Wl[cm], c->p.weights[k], 0};
      bpos += nblk(cm);
      sc += SP_PA_SC;
      mm += D.mm;
      strip += D.strips;
    }
    put(A.maps_fbar, m.data(), m.size() * sizeof(PaMap));
  }
  {
    std::vector<PaMap> m((size_t)SP_NCH * g.n_pairs);
    for (int p = 0; p < g.n_pairs; ++p) {
      const int cl = g.pc[p];
      const size_t pl = n_l(cl);
      for (int k = 0; k < SP_NCH; ++k) {
        const float* gn = cl == cm ? A.gfbar + k * pl : A.gN[cl] + k * pl;
        m[(size_t)p * SP_NCH + k] = PaMap{A.F[p] + k * pl, gn, A.F[p] + k * pl, bpos, sc, mm, strip, g.Hl[cl], g.Wl[cl],
                                          1.f, 0};
        bpos += nblk(cl);
        sc += SP_PA_SC;
        mm += D.mm;
        strip += D.strips;
      }
    }
    put(A.maps_F, m.data(), m.size() * sizeof(PaMap));
  }
  // dL/dN at centre levels below c_max: pyramid-step transposes from c_max down
  for (int l = cm - 1; l >= g.c_min; --l) {
    std::vector<PaPlane> t(SP_NCH);
    for (int k = 0; k < SP_NCH; ++k) {
      const float* src = (l + 1 == cm) ? A.gfbar + k * n_l(cm) : A.gN[l + 1] + k * n_l(l + 1);
      t[k] = PaPlane{src, nullptr, A.gN[l] + k * n_l(l), nullptr, g.Hl[l], g.Wl[l], g.Hl[l + 1], g.Wl[l + 1], 0, 0};
    }
    put(A.tab_gn[l], t.data(), t.size() * sizeof(PaPlane));
  }
  // centre-surround maps, their adjoint and the up-sample transpose, per pair
  for (int p = 0; p < g.n_pairs; ++p) {
    const int cl = g.pc[p], sl = g.ps[p];
    std::vector<PaPlane> cs(SP_NCH), up(SP_NCH);
    std::vector<float*> gc(SP_NCH);
    for (int k = 0; k < SP_NCH; ++k) {
      float* Fk = A.F[p] + k * n_l(cl);
      cs[k] = PaPlane{chan(k, cl), chan(k, sl), Fk, A.amax + ((size_t)p * SP_NCH + k) * SP_PA_AMAX, g.Hl[cl], g.Wl[cl],
                      g.Hl[sl], g.Wl[sl], sl - cl, 0};
      up[k] = PaPlane{Fk, nullptr, A.gX[sl] + k * n_l(sl), nullptr, g.Hl[cl], g.Wl[cl], g.Hl[sl], g.Wl[sl], sl - cl, 0};
      gc[k] = A.gX[cl] + k * n_l(cl);
    }
    put(A.tab_cs[p], cs.data(), cs.size() * sizeof(PaPlane));
    put(A.tab_up[p], up.data(), up.size() * sizeof(PaPlane));
    put(A.gc[p], gc.data(), gc.size() * sizeof(float*));
  }
  // Gabor transposes at the used levels; pyramid-step transposes of the base channels
  for (int l = 1; l <= g.top; ++l) {
    if (A.tab_gab[l]) {
      PaPlane t{A.gX[l] + 3 * n_l(l), nullptr, A.gX[l], nullptr, g.Hl[l], g.Wl[l], 0, 0, c->p.gabor_radius, 0};
      put(A.tab_gab[l], &t, sizeof t);
    }
    const int ks[4] = {0, 1, 2, 7};
    std::vector<PaPlane> t(4);
    for (int j = 0; j < 4; ++j)
      t[j] = PaPlane{A.gX[l] + ks[j] * n_l(l), nullptr, A.gX[l - 1] + ks[j] * n_l(l - 1), nullptr, g.Hl[l - 1],
                     g.Wl[l - 1], g.Hl[l], g.Wl[l], 0, 0};
    put(A.tab_pyr[l], t.data(), t.size() * sizeof(PaPlane));
  }
  for (auto& u : ups) {
    const hipError_t e = hipMemcpyAsync(u.first, u.second.data(), u.second.size(), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
  }
  return hipStreamSynchronize(c->stream);
}

// Phases of one stream's forward saliency map (stream index 0), appended to `js` with
// their launch flags and LDS sizes; *nc_out receives the channels per across-scale
// workgroup.  Contexts and the allocation-free entry point build identical tables.
int forward_phases(const Geo& g, const sp_params& p, const StreamDesc& sd, const Tune& tune, JobStore& js,
                   std::vector<Phase>& out, int* nc_out) {
  std::vector<std::vector<Job>> parts;
  std::vector<int> kinds;
  const int nc = csapply_nc(g, tune.ca_nc);
  const size_t ca_lds = nc * (gpath_ok(g) ? csg_lds_bytes(g) : csapply_lds_bytes(g));
  if (sp_csapply_reserve_lds(ca_lds) != hipSuccess)
    return fail(SP_EHIP, "cannot reserve %zu bytes of LDS for the across-scale sum", ca_lds);
  build_forward_jobs(parts, kinds, sd, g, 0, PROG_ALL, nc);
  for (size_t i = 0; i < parts.size(); ++i) {
    const bool grp = kinds[i] == JOB_CSAPPLY || kinds[i] == JOB_CSG;
    const bool pyr = kinds[i] == JOB_DOWN || kinds[i] == JOB_TAIL;   // flag: Gabor radius
    const int gflag = nc | (kinds[i] == JOB_CSG ? csg_set(g) << 8 : 0);
    if (tune.xcd) xcd_order(parts[i]);
    out.push_back(js.add(kinds[i], grp ? gflag : (pyr ? p.gabor_radius : 0), parts[i], 1));
    if (grp) out.back().lds = ca_lds;
  }
  *nc_out = nc;
  return SP_OK;
}

}  // namespace

extern "C" {

const char* sp_last_error(void) { return g_err.c_str(); }

void sp_default_params(sp_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->depth = 0;
  p->n_centers = 2;
  p->centers[0] = 1;
  p->centers[1] = 2;
  p->n_deltas = 2;
  p->deltas[0] = 2;
  p->deltas[1] = 3;
  for (int k = 0; k < 8; ++k) p->weights[k] = 1.f;
  p->q = 1e-3;
  p->r = 1e-1;
  p->eps = 1e-4f;
  p->border = 1;
  p->lambda = 1.f;
  p->potts = 0.f;
  p->lm_block = 8;
  p->flat_tol = 1e-5f;
  p->gabor_lambda = 4.f;
  p->gabor_sigma = 2.f;
  p->gabor_radius = 6;
  p->record_tape = 0;
  p->f_mode = 0;
  p->dt_sigma = 2.f;
  p->ssm_q = 0.0;
  p->ssm_r = 0.0;
  p->gmm_components = 3;
  p->gmm_iters = 10;
  p->gmm_reg = 1e-4f;
}

int sp_destroy(sp_ctx* c) {
  g_err.clear();
  if (!c) return SP_OK;
  if (c->stream || c->arena) (void)hipStreamSynchronize(c->stream);
  c->prof.destroy();
  if (c->arena) (void)hipFree(c->arena);
  if (c->jobs.dev) (void)hipFree(c->jobs.dev);
  delete c;
  return SP_OK;
}

int sp_create(const sp_params* p, int32_t H, int32_t W, void* hip_stream, sp_ctx** out) {
  g_err.clear();
  if (!out) return fail(SP_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_params(p);
  if (rc) return rc;
  Geo g;
  rc = make_geo(*p, H, W, g);
  if (rc) return rc;
  sp_ctx* c = new (std::nothrow) sp_ctx();
  if (!c) return fail(SP_ENOMEM, "host allocation failed");
  c->p = *p;
  c->g = g;
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(SP_EHIP, "hipGetDevice failed (no GPU?)");
  }
  c->cap = p->record_tape;
  c->n_lvl0_tiles = ntiles(H, W);
  const int Hc = g.Hl[g.c_max], Wc = g.Wl[g.c_max];
  const size_t HW = (size_t)H * W;
  c->CH = c->cap > 0 ? std::min(c->cap, 32) : 0;
  // two passes over the layout: size, then place
  for (int pass = 0; pass < 2; ++pass) {
    Bump b;
    b.base = c->arena;
    layout_stream(c->h_sd, g, *p, b, 1, true);
    c->d_sd = b.take<StreamDesc>(1);
    c->pi_state[0] = b.take<float>(HW);
    c->pi_state[1] = b.take<float>(HW);
    c->loss_part = b.take<float>(c->loss_nblk);
    c->S_scratch = b.take<float>((size_t)Hc * Wc);
    if (p->f_mode == 1) c->f_map = b.take<float>(HW);
    if (p->gmm_components > 0) {
      c->gmm_tiles = (int)((HW + SP_GMM_TILE - 1) / SP_GMM_TILE);
      c->gmm_state = b.take<GmmState>(1);
      c->gmm_part = b.take<double>((size_t)2 * p->gmm_components * 10 * c->gmm_tiles);
    }
    if (p->ssm_r > 0) {
      c->ssm[0] = b.take<float>((size_t)Hc * Wc);
      c->ssm[1] = b.take<float>((size_t)Hc * Wc);
    }
    std::vector<StreamDesc> rsd(c->CH);
    if (c->cap > 0) {
      c->ckpt = b.take<float>((size_t)c->cap * 4 * g.Hl[g.c_min] * g.Wl[g.c_min]);
      c->S_tape = b.take<float>((size_t)c->cap * Hc * Wc);
      c->f_tape = b.take<float>((size_t)c->cap * HW);
      c->ms_tape = b.take<float>((size_t)c->cap * 2);
      c->K_tape = b.take<double>(c->cap);
      c->P_tape = b.take<double>(c->cap);
      c->nu[0] = b.take<float>(HW);
      c->nu[1] = b.take<float>(HW);
      c->gu = b.take<float>(HW);
      c->gs_all = b.take<float>((size_t)c->cap * Hc * Wc);
      c->gk_part = b.take<float>((size_t)c->cap * c->n_lvl0_tiles);
      c->dot_part = b.take<float>((size_t)c->cap * c->h_sd.n_cmax_tiles * SP_NCH);
      c->cx = b.take<float>((size_t)c->cap * SP_NCH);
      c->gK_scratch = b.take<double>((size_t)c->cap * (1 + SP_NCH));
      c->d_rsd = b.take<StreamDesc>(c->CH);
      c->d_rio = b.take<StepIO>(c->cap);
      for (int i = 0; i < c->CH; ++i) layout_stream(rsd[i], g, *p, b, g.c_min + 1, false);
      pixadj_layout(c, b);
    }
    if (pass == 0) {
      c->arena_bytes = b.off + 256;
      if (hipMalloc(&c->arena, c->arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return fail(SP_ENOMEM, "hipMalloc of %zu bytes failed", c->arena_bytes);
      }
    } else {
      // upload static tables
      hipError_t e = hipMemcpyAsync(c->d_sd, &c->h_sd, sizeof(StreamDesc), hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess && c->cap > 0) {
        e = hipMemcpyAsync(c->d_rsd, rsd.data(), sizeof(StreamDesc) * c->CH, hipMemcpyHostToDevice, c->stream);
        std::vector<StepIO> rio(c->cap);
        const size_t cstride = (size_t)4 * g.Hl[g.c_min] * g.Wl[g.c_min];
        const size_t plane = (size_t)Hc * Wc;
        for (int t = 0; t < c->cap; ++t) {
          std::memset(&rio[t], 0, sizeof(StepIO));
          rio[t].ckpt = c->ckpt + (size_t)t * cstride;
          rio[t].gs = c->gs_all + (size_t)t * plane;
          rio[t].ms_tape = c->ms_tape + 2 * (size_t)t;
          rio[t].dot = c->dot_part + (size_t)t * c->h_sd.n_cmax_tiles * SP_NCH;
          rio[t].cx = c->cx + (size_t)t * SP_NCH;
        }
        if (e == hipSuccess)
          e = hipMemcpyAsync(c->d_rio, rio.data(), sizeof(StepIO) * c->cap, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = pixadj_upload(c);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) {
        sp_destroy(c);
        return fail(SP_EHIP, "uploading stream tables: %s", hipGetErrorString(e));
      }
    }
  }
  if (sp_csapply_reserve_lds(csapply_lds_bytes(g)) != hipSuccess) {
    sp_destroy(c);
    return fail(SP_EHIP, "cannot reserve %zu bytes of LDS for the across-scale sum", csapply_lds_bytes(g));
  }
  c->tune = cached_tune(H, W);
  int rc2 = ctx_build_tables(c);
  if (rc2) {
    std::string msg = g_err;
    sp_destroy(c);
    g_err = msg;
    return rc2;
  }
  *out = c;
  return SP_OK;
}

}  // extern "C"

namespace {

// (Re)builds every job table of a context from its geometry and tuning knobs.
int ctx_build_tables(sp_ctx* c) {
  const Geo& g = c->g;
  const int H = g.H, W = g.W, Hc = g.Hl[g.c_max], Wc = g.Wl[g.c_max];
  c->jobs.host.clear();
  c->fwd.clear();
  c->prior.clear();
  c->mrf.clear();
  c->bwd.clear();
  c->rec.clear();
  c->dt.clear();
  {
    int nc = 0;
    int rc = forward_phases(g, c->p, c->h_sd, c->tune, c->jobs, c->fwd, &nc);
    if (rc) return rc;
    const size_t ca_lds = nc * (gpath_ok(g) ? csg_lds_bytes(g) : csapply_lds_bytes(g));
    auto order = [&](std::vector<Job> v) {
      if (c->tune.xcd) xcd_order(v);
      return v;
    };
    std::vector<Job> v;
    add_tiles(v, 0, 0, Hc, Wc);
    c->prior.push_back(c->jobs.add(JOB_SMAX, 0, v, 1));
    v.clear();
    add_tiles_wh(v, 0, 0, H, W, SP_KAL_ROWS, c->tune.kalman_tw, JOB_KALMAN);
    c->prior.push_back(c->jobs.add(JOB_KALMAN, 0, order(v), 1));
    v.clear();
    rgb_jobs(v, 0, c->h_sd, g);
    c->mrf.push_back(c->jobs.add(JOB_RGB, 1, v, 1));
    v.clear();
    add_tiles(v, 0, 0, H, W);
    c->mrf.push_back(c->jobs.add(JOB_MRF, 0, v, 1));
    v.clear();
    add_tiles_wh(v, 0, 0, H, W, SP_DT_T, SP_DT_T, JOB_DT);
    c->dt.push_back(c->jobs.add(JOB_DT, 0, order(v), 1));
    v.clear();
    add_tiles(v, 0, 0, H, W);
    c->bwd.push_back(c->jobs.add(JOB_BWD_NU, 0, v, 1));
    v.clear();
    add_tiles(v, 0, 0, Hc, Wc);
    c->bwd.push_back(c->jobs.add(JOB_BWD_GS, 0, v, 1));
    if (c->CH > 0) {
      std::vector<std::vector<Job>> all;
      std::vector<int> kk;
      for (int s = 0; s < c->CH; ++s) {
        std::vector<std::vector<Job>> ps;
        std::vector<int> ks;
        build_forward_jobs(ps, ks, c->h_sd, g, s, PROG_RECOMPUTE, nc);
        if (all.empty()) {
          all.resize(ps.size());
          kk = ks;
        }
        for (size_t i = 0; i < ps.size(); ++i) all[i].insert(all[i].end(), ps[i].begin(), ps[i].end());
      }
      for (size_t i = 0; i < all.size(); ++i) {
        const bool grp = kk[i] == JOB_CSAPPLY || kk[i] == JOB_CSG;
        const bool pyr = kk[i] == JOB_DOWN || kk[i] == JOB_TAIL;
        const int gflag = nc | (kk[i] == JOB_CSG ? csg_set(g) << 8 : 0);
        c->rec.push_back(c->jobs.add(kk[i], grp ? gflag : (pyr ? c->p.gabor_radius : 0), all[i], c->CH));
        if (grp) c->rec.back().lds = ca_lds;
      }
    }
  }
  return upload_jobs(c->jobs, c->stream);
}

}  // namespace

extern "C" {

int sp_set_stream(sp_ctx* c, void* hip_stream) {
  g_err.clear();
  if (!c) return fail(SP_EINVAL, "ctx is NULL");
  c->stream = (hipStream_t)hip_stream;
  return SP_OK;
}

int sp_get_geometry(const sp_ctx* c, sp_geometry* out) {
  g_err.clear();
  if (!c || !out) return fail(SP_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  const Geo& g = c->g;
  out->H = g.H;
  out->W = g.W;
  out->depth = g.depth;
  out->top = g.top;
  out->c_min = g.c_min;
  out->c_max = g.c_max;
  out->n_pairs = g.n_pairs;
  for (int i = 0; i < g.n_pairs; ++i) {
    out->pair_c[i] = g.pc[i];
    out->pair_s[i] = g.ps[i];
  }
  for (int l = 0; l <= g.depth && l <= SP_MAX_LEVELS; ++l) {
    out->level_h[l] = g.Hl[l];
    out->level_w[l] = g.Wl[l];
  }
  out->Hc = g.Hl[g.c_max];
  out->Wc = g.Wl[g.c_max];
  return SP_OK;
}

int sp_set_weights(sp_ctx* c, const float* w, double q, double r) {
  g_err.clear();
  if (!c || !w) return fail(SP_EINVAL, "NULL argument");
  for (int k = 0; k < SP_NCH; ++k)
    if (!std::isfinite(w[k])) return fail(SP_EINVAL, "weight %d is not finite", k);
  if (!is_fin(q) || !is_fin(r) || q < 0 || r < 0 || !(q + r > 0))
    return fail(SP_EINVAL, "Kalman variances must be finite, >= 0 and not both 0");
  for (int k = 0; k < SP_NCH; ++k) {
    c->p.weights[k] = w[k];
    c->h_sd.w[k] = w[k];
  }
  c->p.q = q;
  c->p.r = r;
  // steps already recorded used the old weights and variances: their tape no longer
  // matches what the adjoint would rebuild
  if (c->t > 0) c->tape_ok = false;
  c->tape_gen += 1;
  HIPCHK(hipMemcpyAsync(c->d_sd, &c->h_sd, sizeof(StreamDesc), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SP_OK;
}

int sp_reset(sp_ctx* c) {
  g_err.clear();
  if (!c) return fail(SP_EINVAL, "ctx is NULL");
  c->t = 0;
  c->P = 0.0;
  c->cur = 0;
  c->ssm_t = 0;
  c->ssm_P = 0.0;
  c->ssm_cur = 0;
  c->tape_ok = true;
  c->tape_gen += 1;
  c->Kf.clear();
  c->uses_pi.clear();
  return SP_OK;
}

int64_t sp_step_index(const sp_ctx* c) { return c ? c->t : -1; }

int64_t sp_tape_generation(const sp_ctx* c) { return c ? c->tape_gen : -1; }

int sp_manual_prior(sp_ctx* c, const uint8_t* labels, float* prior_out) {
  g_err.clear();
  if (!c || !labels) return fail(SP_EINVAL, "ctx and labels must not be NULL");
  if (c->cap > 0) return fail(SP_ESTATE, "a context that records a tape starts from the saliency observation");
  int rc = sp_reset(c);
  if (rc) return rc;
  const Geo& g = c->g;
  float* pnext = c->pi_state[c->cur ^ 1];
  const hipError_t e = c->prof.timed(c->stream, JOB_MANUAL, [&] {
    return sp_launch_manual(labels, pnext, prior_out, (size_t)g.H * g.W, c->p.eps, c->stream);
  });
  if (e != hipSuccess) return fail(SP_EHIP, "manual prior launch: %s", hipGetErrorString(e));
  (void)now_gain(0, 0.0, c->p.q, c->p.r, &c->P);   // P_0 = R, as after a first observation
  c->cur ^= 1;
  c->t = 1;
  return SP_OK;
}

int sp_colour_likelihood(sp_ctx* c, const uint8_t* rgb_t, const float* prior, float* unary_inout, float* gmm_out) {
  g_err.clear();
  if (!c || !rgb_t || !prior || !unary_inout) return fail(SP_EINVAL, "ctx, rgb_t, prior and unary_inout must not be NULL");
  const int M = c->p.gmm_components;
  if (M < 1 || !c->gmm_state) return fail(SP_ESTATE, "the context was created with gmm_components = 0");
  GmmIO io{};
  io.rgb = rgb_t;
  io.prior = prior;
  io.unary = unary_inout;
  io.n = c->g.H * c->g.W;
  io.ntiles = c->gmm_tiles;
  io.reg = c->p.gmm_reg;
  const int iters = c->p.gmm_iters;
  io.part_out = c->gmm_part;
  io.part_in = c->gmm_part;
  io.st_prev = c->gmm_state;
  io.st_next = c->gmm_state;
  auto launch = [&](int phase, int kind, float* out) -> int {
    io.out = out;
    const hipError_t e = c->prof.timed(c->stream, kind, [&] { return sp_launch_gmm(phase, M, io, c->stream); });
    if (e != hipSuccess) return fail(SP_EHIP, "colour likelihood launch (phase %d): %s", phase, hipGetErrorString(e));
    return SP_OK;
  };
  int rc = launch(0, JOB_GMM_ACC, nullptr);
  if (!rc) rc = launch(1, JOB_GMM_FIT, iters == 0 ? gmm_out : nullptr);
  for (int it = 0; it < iters && !rc; ++it) {
    rc = launch(2, JOB_GMM_ACC, nullptr);
    if (!rc) rc = launch(3, JOB_GMM_FIT, it == iters - 1 ? gmm_out : nullptr);
  }
  if (!rc) rc = launch(4, JOB_GMM_PSI, nullptr);
  return rc;
}

int sp_stochastic_saliency(const sp_ctx* c, const float** mean, double* var) {
  g_err.clear();
  if (!c || !mean || !var) return fail(SP_EINVAL, "NULL argument");
  if (!c->ssm[0]) return fail(SP_ESTATE, "the stochastic saliency map is off (ssm_r = 0)");
  if (c->ssm_t == 0) return fail(SP_ESTATE, "no prior update since the reset");
  *mean = c->ssm[c->ssm_cur];
  *var = c->ssm_P;
  return SP_OK;
}

int saliency_forward(sp_ctx* c, const uint8_t* rgb_t, const uint8_t* rgb_prev, float* S_out, float* C_out) {
  g_err.clear();
  if (!c || !rgb_t || !S_out) return fail(SP_EINVAL, "ctx, rgb_t and S_out must not be NULL");
  StepIO io;
  std::memset(&io, 0, sizeof io);
  io.rgb = rgb_t;
  io.rgb_prev = rgb_prev;
  io.S_out = S_out;
  io.C_out = C_out;
  if (c->cap > 0) {
    if (c->t >= c->cap) return fail(SP_ESTATE, "tape holds %d frames; call sp_reset before frame %lld", c->cap,
                                    (long long)c->t);
    const Geo& g = c->g;
    io.ckpt = c->ckpt + (size_t)c->t * 4 * g.Hl[g.c_min] * g.Wl[g.c_min];
    io.S_tape = c->S_tape + (size_t)c->t * g.Hl[g.c_max] * g.Wl[g.c_max];
  }
  for (const Phase& ph : c->fwd) {
    int rc = run_phase(c, ph, c->d_sd, nullptr, &io, ph.n);
    if (rc) return rc;
  }
  return SP_OK;
}

}  // extern "C"

namespace {

// The variant phases of a prior update, before its Kalman phase: the stochastic saliency
// map (which then replaces S as the observation, with its max partials) and the
// distance-transform prediction.  `smax` says whether the max partials of the observation
// must still be taken (the fused step has them from the conspicuity pass).
int prior_variants(sp_ctx* c, StepIO& io, bool smax) {
  double Ps = 0.0;
  if (c->ssm[0]) {
    const double Ks = now_gain(c->ssm_t, c->ssm_P, c->p.ssm_q, c->p.ssm_r, &Ps);
    io.ssm_prev = c->ssm_t == 0 ? nullptr : c->ssm[c->ssm_cur];
    io.ssm_next = c->ssm[c->ssm_cur ^ 1];
    io.Ks = (float)Ks;
  }
  if (smax || c->ssm[0]) {
    int rc = run_phase(c, c->prior.front(), c->d_sd, nullptr, &io, c->prior.front().n);   // the max partials
    if (rc) return rc;
  }
  if (c->ssm[0]) {
    io.S_in = io.ssm_next;
    c->ssm_P = Ps;
    c->ssm_cur ^= 1;
    c->ssm_t += 1;
  }
  if (c->f_map && io.t > 0) {
    io.f_map = c->f_map;
    int rc = run_phase(c, c->dt.front(), c->d_sd, nullptr, &io, c->dt.front().n);
    if (rc) return rc;
  }
  return SP_OK;
}

}  // namespace

extern "C" {

int prior_update(sp_ctx* c, const float* S, const uint8_t* seg_prev, float* prior_out) {
  g_err.clear();
  if (!c || !S) return fail(SP_EINVAL, "ctx and S must not be NULL");
  if (c->cap > 0 && c->t >= c->cap)
    return fail(SP_ESTATE, "tape holds %d frames; call sp_reset first", c->cap);
  StepIO io;
  std::memset(&io, 0, sizeof io);
  io.S_in = S;
  io.seg_prev = seg_prev;
  io.pi_prev = c->pi_state[c->cur];
  io.pi_next = c->pi_state[c->cur ^ 1];
  io.prior_out = prior_out;
  double Pn = 0.0;
  const double K = now_gain(c->t, c->P, c->p.q, c->p.r, &Pn);
  io.K = (float)K;
  io.t = (int32_t)std::min<int64_t>(c->t, 0x7fffffff);
  if (c->cap > 0) {
    const Geo& g = c->g;
    io.f_tape = c->f_tape + (size_t)c->t * g.H * g.W;
    io.ms_tape = c->ms_tape + (size_t)c->t * 2;
  }
  int rc = prior_variants(c, io, true);
  if (rc) return rc;
  rc = run_phase(c, c->prior.back(), c->d_sd, nullptr, &io, c->prior.back().n);   // the Kalman phase
  if (rc) return rc;
  if (c->cap > 0) {
    // gains and variances of the recorded steps (host -> device, from values that stay
    // alive in the context until the next reset)
    c->Kf.push_back((float)K);
    c->uses_pi.push_back(seg_prev == nullptr && c->t > 0);
  }
  c->P = Pn;
  c->cur ^= 1;
  c->t += 1;
  return SP_OK;
}

int sp_step(sp_ctx* c, const uint8_t* rgb_t, const uint8_t* rgb_prev, const uint8_t* seg_prev, float* S_out,
            float* C_out, float* prior_out, float* unary_out, float* pairwise_out, float* beta_out) {
  g_err.clear();
  if (!c || !rgb_t || !S_out) return fail(SP_EINVAL, "ctx, rgb_t and S_out must not be NULL");
  if ((unary_out == nullptr) != (pairwise_out == nullptr))
    return fail(SP_EINVAL, "unary_out and pairwise_out must be given together");
  if (c->cap > 0 && c->t >= c->cap)
    return fail(SP_ESTATE, "tape holds %d frames; call sp_reset first", c->cap);
  const bool mrf = unary_out != nullptr;
  const Geo& g = c->g;
  StepIO io;
  std::memset(&io, 0, sizeof io);
  io.rgb = rgb_t;
  io.rgb_prev = rgb_prev;
  io.S_out = S_out;
  io.C_out = C_out;
  io.S_in = S_out;
  io.seg_prev = seg_prev;
  io.pi_prev = c->pi_state[c->cur];
  io.pi_next = c->pi_state[c->cur ^ 1];
  io.prior_out = prior_out;
  if (mrf) {
    io.unary = unary_out;
    io.pairwise = pairwise_out;
    io.beta_out = beta_out;
  }
  double Pn = 0.0;
  const double K = now_gain(c->t, c->P, c->p.q, c->p.r, &Pn);
  io.K = (float)K;
  io.t = (int32_t)std::min<int64_t>(c->t, 0x7fffffff);
  if (c->cap > 0) {
    io.ckpt = c->ckpt + (size_t)c->t * 4 * g.Hl[g.c_min] * g.Wl[g.c_min];
    io.S_tape = c->S_tape + (size_t)c->t * g.Hl[g.c_max] * g.Wl[g.c_max];
    io.f_tape = c->f_tape + (size_t)c->t * g.H * g.W;
    io.ms_tape = c->ms_tape + (size_t)c->t * 2;
  }
  for (const Phase& ph0 : c->fwd) {
    Phase ph = ph0;
    if (ph.kind == JOB_RGB) ph.flag = mrf ? 1 : 0;
    int rc = run_phase(c, ph, c->d_sd, nullptr, &io, ph.n);
    if (rc) return rc;
  }
  int rc = prior_variants(c, io, false);
  if (rc) return rc;
  rc = run_phase(c, c->prior.back(), c->d_sd, nullptr, &io, c->prior.back().n);   // the Kalman phase
  if (rc) return rc;
  if (c->cap > 0) {
    c->Kf.push_back((float)K);
    c->uses_pi.push_back(seg_prev == nullptr && c->t > 0);
  }
  c->P = Pn;
  c->cur ^= 1;
  c->t += 1;
  return SP_OK;
}

int sp_saliency_noalloc(const sp_params* p, int32_t H, int32_t W, const uint8_t* rgb_t, const uint8_t* rgb_prev,
                        float* S_out, float* C_out, void* hip_stream) {
  g_err.clear();
  if (!rgb_t || !S_out) return fail(SP_EINVAL, "rgb_t and S_out must not be NULL");
  int rc = validate_params(p);
  if (rc) return rc;
  Geo g;
  rc = make_geo(*p, H, W, g);
  if (rc) return rc;
  const Tune tune = cached_tune(H, W);
  const int nc = csapply_nc(g, tune.ca_nc);
  // sizing pass (no device call): stream description, job table, then the stream's
  // pyramid, maps and partials, in the order the placing pass takes them
  StreamDesc sd;
  size_t n_jobs = 0;
  size_t need = 0;
  {
    Bump b;
    b.take<StreamDesc>(1);
    layout_stream(sd, g, *p, b, 1, true);
    std::vector<std::vector<Job>> parts;
    std::vector<int> kinds;
    build_forward_jobs(parts, kinds, sd, g, 0, PROG_ALL, nc);
    for (const auto& v : parts) n_jobs += v.size();
    b.take<Job>(n_jobs);
    need = b.off;
  }
  if (need > SP_NOALLOC_BYTES)
    return fail(SP_ESHAPE, "a %dx%d frame needs %zu bytes of scratch; the allocation-free entry point holds %zu "
                "(use a context)", H, W, need, (size_t)SP_NOALLOC_BYTES);
  void* base = nullptr;
  HIPCHK(sp_noalloc_scratch(&base));
  Bump b;
  b.base = static_cast<char*>(base);
  StreamDesc* d_sd = b.take<StreamDesc>(1);
  layout_stream(sd, g, *p, b, 1, true);
  Job* d_jobs = b.take<Job>(n_jobs);
  if (b.off != need) return fail(SP_EINVAL, "scratch layout changed between its passes");
  JobStore js;
  std::vector<Phase> phases;
  int nc2 = 0;
  rc = forward_phases(g, *p, sd, tune, js, phases, &nc2);
  if (rc) return rc;
  if (js.host.size() != n_jobs || nc2 != nc) return fail(SP_EINVAL, "job table changed between its passes");
  hipStream_t st = (hipStream_t)hip_stream;
  // The uploads are ordered after earlier work on this stream (which may still read the
  // scratch); the wait keeps the host tables alive until they are copied.
  HIPCHK(hipMemcpyAsync(d_sd, &sd, sizeof(StreamDesc), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_jobs, js.host.data(), sizeof(Job) * n_jobs, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  StepIO io;
  std::memset(&io, 0, sizeof io);
  io.rgb = rgb_t;
  io.rgb_prev = rgb_prev;
  io.S_out = S_out;
  io.C_out = C_out;
  for (const Phase& ph : phases) {
    const hipError_t e = sp_launch(ph.kind, d_jobs + ph.off, ph.n, d_sd, nullptr, &io, ph.flag, nullptr, st, ph.lds);
    if (e != hipSuccess) return fail(SP_EHIP, "kernel launch (phase kind %d): %s", ph.kind, hipGetErrorString(e));
  }
  return SP_OK;
}

int sp_autotune(sp_ctx* c, const uint8_t* rgb_t, const uint8_t* rgb_prev, int32_t steps, char* report,
                size_t report_len) {
  g_err.clear();
  if (!c || !rgb_t) return fail(SP_EINVAL, "ctx and rgb_t must not be NULL");
  if (steps < 1 || steps > 1000) return fail(SP_EINVAL, "steps must be 1..1000");
  if (c->cap > 0) return fail(SP_ESTATE, "autotune a context without a tape");
  const Geo& g = c->g;
  HIPCHK(hipStreamSynchronize(c->stream));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float* S_out = c->S_scratch;   // the state is reset at the end
  std::string rep;
  char line[160];
  auto time_it = [&](double* ms) -> int {
    int r = ctx_build_tables(c);
    if (r) return r;
    r = sp_step(c, rgb_t, rgb_prev, nullptr, S_out, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (r) return r;
    HIPCHK(hipEventRecord(e0, c->stream));
    for (int i = 0; i < steps && !r; ++i)
      r = sp_step(c, rgb_t, rgb_prev, nullptr, S_out, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (r) return r;
    HIPCHK(hipEventRecord(e1, c->stream));
    HIPCHK(hipEventSynchronize(e1));
    float f = 0.f;
    HIPCHK(hipEventElapsedTime(&f, e0, e1));
    *ms = f / steps;
    return SP_OK;
  };
  int rc = SP_OK;
  double best = 1e30, t = 0;
  Tune bt = c->tune;
  for (int x = 0; x < 2 && !rc; ++x)
    for (int tw : {16, 32, 64}) {
      c->tune.xcd = x != 0;
      c->tune.kalman_tw = tw;
      rc = time_it(&t);
      if (rc) break;
      snprintf(line, sizeof line, "%dx%d xcd_order=%d kalman tile %dx%d: %.4f ms/frame\n", g.H, g.W, x, SP_KAL_ROWS, tw, t);
      rep += line;
      if (t < best) {
        best = t;
        bt = c->tune;
      }
    }
  for (int nc : {1, 2, 4, 8}) {
    if (rc || nc == bt.ca_nc || csapply_nc(g, nc) != nc) continue;
    c->tune = bt;
    c->tune.ca_nc = nc;
    rc = time_it(&t);
    if (rc) break;
    snprintf(line, sizeof line, "%dx%d across-scale channels per workgroup %d: %.4f ms/frame\n", g.H, g.W, nc, t);
    rep += line;
    if (t < best) {
      best = t;
      bt = c->tune;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  c->tune = bt;
  rc = ctx_build_tables(c);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(tune_mutex());
    tune_cache_tw()[{g.H, g.W}] = bt.kalman_tw;
    tune_cache_xcd() = bt.xcd;
    tune_cache_nc() = bt.ca_nc;
  }
  if (report && report_len) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return sp_reset(c);
}

int sp_set_tune(sp_ctx* c, int32_t kalman_tw, int32_t xcd_order, int32_t channels) {
  g_err.clear();
  if (!c) return fail(SP_EINVAL, "ctx is NULL");
  if (kalman_tw != 16 && kalman_tw != 32 && kalman_tw != 64) return fail(SP_EINVAL, "kalman_tw must be 16, 32 or 64");
  if (channels != 1 && channels != 2 && channels != 4 && channels != 8) return fail(SP_EINVAL, "channels must be 1, 2, 4 or 8");
  if (csapply_nc(c->g, channels) != channels)
    return fail(SP_EINVAL, "%d channels per across-scale workgroup exceed the LDS limit for this geometry", channels);
  c->tune.kalman_tw = kalman_tw;
  c->tune.xcd = xcd_order != 0;
  c->tune.ca_nc = channels;
  HIPCHK(hipStreamSynchronize(c->stream));
  return ctx_build_tables(c);
}

int sp_tune_cache_clear(void) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(tune_mutex());
  tune_cache_tw().clear();
  tune_cache_xcd() = false;
  tune_cache_nc() = 2;
  return SP_OK;
}

int mrf_weights(sp_ctx* c, const uint8_t* rgb_t, const float* prior, float* unary_out, float* pairwise_out,
                float* beta_out) {
  g_err.clear();
  if (!c || !rgb_t || !prior || !unary_out || !pairwise_out)
    return fail(SP_EINVAL, "ctx, rgb_t, prior, unary_out and pairwise_out must not be NULL");
  StepIO io;
  std::memset(&io, 0, sizeof io);
  io.rgb = rgb_t;
  io.unary = unary_out;
  io.pairwise = pairwise_out;
  io.beta_out = beta_out;
  for (const Phase& ph : c->mrf) {
    int rc = run_phase(c, ph, c->d_sd, nullptr, &io, ph.n, prior);
    if (rc) return rc;
  }
  return SP_OK;
}

int saliency_backward(sp_ctx* c, const float* grad_prior, int32_t T, float* grad_w, float* grad_q, float* grad_r) {
  g_err.clear();
  if (!c || !grad_prior || !grad_w || !grad_q || !grad_r) return fail(SP_EINVAL, "NULL argument");
  if (c->cap <= 0) return fail(SP_ESTATE, "context was created without a tape (record_tape = 0)");
  if (!c->tape_ok)
    return fail(SP_ESTATE, "tape invalidated by sp_set_state or sp_set_weights after recorded steps; call sp_reset");
  if (T < 1 || T != c->t || (size_t)T != c->Kf.size())
    return fail(SP_ESTATE, "backward of %d steps, but %lld prior updates were recorded since the reset", T,
                (long long)c->t);
  const Geo& g = c->g;
  const size_t HW = (size_t)g.H * g.W;
  const int Hc = g.Hl[g.c_max], Wc = g.Wl[g.c_max];
  // host gains -> device tape (FP64), for the scalar sweep
  {
    std::vector<double> Kd(T), Pd(T);
    double P = 0.0;
    for (int t = 0; t < T; ++t) Kd[t] = now_gain(t, P, c->p.q, c->p.r, &P), Pd[t] = P;
    HIPCHK(hipMemcpyAsync(c->K_tape, Kd.data(), sizeof(double) * T, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->P_tape, Pd.data(), sizeof(double) * T, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  // reverse sweep over the steps
  for (int t = T - 1; t >= 0; --t) {
    BwdIO b;
    std::memset(&b, 0, sizeof b);
    b.grad = grad_prior + (size_t)t * HW;
    b.nu_next = (t + 1 < T) ? c->nu[(t + 1) & 1] : nullptr;
    b.nu_out = c->nu[t & 1];
    b.gu = c->gu;
    b.gs = c->gs_all + (size_t)t * Hc * Wc;
    b.gk_part = c->gk_part + (size_t)t * c->n_lvl0_tiles;
    b.f = (t > 0) ? c->f_tape + (size_t)t * HW : nullptr;
    b.S = c->S_tape + (size_t)t * Hc * Wc;
    b.ms = c->ms_tape + (size_t)t * 2;
    b.K = (t > 0) ? c->Kf[t] : 1.f;
    b.carry = (t + 1 < T && c->uses_pi[t + 1]) ? 1.f - c->Kf[t + 1] : 0.f;
    b.t = t;
    for (const Phase& ph : c->bwd) {
      hipError_t e = timed(c, ph.kind, [&] {
        return sp_launch_bwd(ph.kind, c->jobs.dev + ph.off, ph.n, c->d_sd, nullptr, &b, c->stream);
      });
      if (e != hipSuccess) return fail(SP_EHIP, "adjoint launch: %s", hipGetErrorString(e));
    }
  }
  // conspicuity maps recomputed from the checkpoints, dotted with the saliency adjoint
  for (int t0 = 0; t0 < T; t0 += c->CH) {
    const int n = std::min(c->CH, T - t0);
    const StepIO* ios = c->d_rio + t0;
    for (const Phase& ph : c->rec) {
      const int nj = ph.upto[n];
      hipError_t e = timed(c, ph.kind, [&] {
        if (ph.kind == JOB_CONSP_DOT) return sp_launch_consp_dot(c->jobs.dev + ph.off, nj, c->d_rsd, ios, c->stream);
        return sp_launch(ph.kind, c->jobs.dev + ph.off, nj, c->d_rsd, ios, nullptr, ph.flag, nullptr, c->stream, ph.lds);
      });
      if (e != hipSuccess) return fail(SP_EHIP, "recompute launch: %s", hipGetErrorString(e));
    }
  }
  const float* wdev = reinterpret_cast<const float*>(reinterpret_cast<const char*>(c->d_sd) + offsetof(StreamDesc, w));
  BwdFin fin{c->gk_part, c->dot_part, c->cx, c->ms_tape, wdev, c->gK_scratch, grad_w, grad_q, grad_r,
             c->n_lvl0_tiles, c->h_sd.n_cmax_tiles};
  hipError_t e = timed(c, JOB_BWD_FINAL, [&] {
    return sp_launch_bwd_final(nullptr, &fin, 1, T, c->K_tape, c->P_tape, c->p.q, c->p.r, c->p.flat_tol, c->stream);
  });
  if (e != hipSuccess) return fail(SP_EHIP, "adjoint reduction launch: %s", hipGetErrorString(e));
  c->pa.gen = c->tape_gen;
  c->pa.T = T;
  return SP_OK;
}

int saliency_backward_frames(sp_ctx* c, const uint8_t* frames, int32_t T, float* grad_frames) {
  g_err.clear();
  if (!c || !frames || !grad_frames) return fail(SP_EINVAL, "NULL argument");
  if (c->cap <= 0) return fail(SP_ESTATE, "context was created without a tape (record_tape = 0)");
  if (c->pa.gen != c->tape_gen || c->pa.T != T || T != c->t)
    return fail(SP_ESTATE, "saliency_backward of this %d-step clip must run first", T);
  const Geo& g = c->g;
  auto& A = c->pa;
  const size_t HW = (size_t)g.H * g.W, HW3 = 3 * HW;
  const int cm = g.c_max;
  const size_t plc = (size_t)g.Hl[cm] * g.Wl[cm];
  auto n_l = [&](int l) { return (int)((size_t)g.Hl[l] * g.Wl[l]); };
  auto ok = [&](hipError_t e, const char* what) -> int {
    if (e != hipSuccess) return fail(SP_EHIP, "pixel adjoint (%s): %s", what, hipGetErrorString(e));
    return SP_OK;
  };
  int maxF = 0;
  for (int p = 0; p < g.n_pairs; ++p) maxF = std::max(maxF, n_l(g.pc[p]));
  for (int t = 0; t < T; ++t) {
    // the frame's forward maps, recomputed into the context's buffers
    StepIO io;
    std::memset(&io, 0, sizeof io);
    io.rgb = frames + (size_t)t * HW3;
    io.rgb_prev = t ? frames + (size_t)(t - 1) * HW3 : nullptr;
    io.S_out = c->S_scratch;
    for (const Phase& ph0 : c->fwd) {
      Phase ph = ph0;
      if (ph.kind == JOB_RGB) ph.flag = 0;
      int rc = run_phase(c, ph, c->d_sd, nullptr, &io, ph.n);
      if (rc) return rc;
    }
    int rc = SP_OK;
    const hipError_t e = timed(c, JOB_PIX_ADJ, [&]() -> hipError_t {
      hipError_t r = sp_pa_gs(c->gs_all + (size_t)t * plc, c->S_tape + (size_t)t * plc, c->ms_tape + 2 * (size_t)t,
                              (int)plc, c->p.flat_tol, A.gS, A.gs_part, c->stream);
      if (r == hipSuccess) r = sp_pa_nadjoint(A.maps_fbar, SP_NCH, (int)plc, g.Hl[cm], c->p.flat_tol, c->stream);
      for (int l = cm - 1; l >= g.c_min && r == hipSuccess; --l)
        r = sp_pa_plane(0, A.tab_gn[l], SP_NCH, n_l(l), 0, nullptr, nullptr, c->stream);
      // dL/dX and the pairs' scales start at zero
      if (r == hipSuccess) r = sp_pa_zero(A.gX[0], A.gX_floats + (size_t)SP_NCH * g.n_pairs * SP_PA_AMAX, c->stream);
      // maps of every pair in one launch, then the adjoint and the up-sample transpose one
      // group at a time (a group's pairs write different levels)
      auto group_n = [&](const int* order, int first, int count, bool surround) {
        int mx = 0;
        for (int k = first; k < first + count; ++k) mx = std::max(mx, n_l(surround ? g.ps[order[k]] : g.pc[order[k]]));
        return mx;
      };
      if (r == hipSuccess)
        r = sp_pa_plane(1, A.tab_cs[A.cs_order[0]], SP_NCH * g.n_pairs, group_n(A.cs_order, 0, g.n_pairs, false), 0,
                        nullptr, nullptr, c->stream);
      if (r == hipSuccess)
        r = sp_pa_nadjoint(A.maps_F, SP_NCH * g.n_pairs, maxF, pixadj_dims(g).maxh, c->p.flat_tol, c->stream);
      for (int q = 0; q < A.n_cs && r == hipSuccess; ++q) {
        const int p0 = A.cs_order[A.cs_first[q]];
        r = sp_pa_plane(2, A.tab_cs[p0], SP_NCH * A.cs_count[q], group_n(A.cs_order, A.cs_first[q], A.cs_count[q], false),
                        0, A.gc[p0], nullptr, c->stream);
      }
      for (int q = 0; q < A.n_up && r == hipSuccess; ++q) {
        const int p0 = A.up_order[A.up_first[q]];
        r = sp_pa_plane(3, A.tab_up[p0], SP_NCH * A.up_count[q], group_n(A.up_order, A.up_first[q], A.up_count[q], true),
                        0, nullptr, nullptr, c->stream);
      }
      // the Gabor transposes of every used level at once (each reads its level's orientation
      // gradients, complete here, and adds into that level's intensity gradient), then the
      // pyramid-step transposes from the top level down
      if (r == hipSuccess) {
        PaGabLevels L{};
        int max_tiles = 0;
        for (int l = g.top; l >= 1; --l)
          if (A.tab_gab[l]) {
            L.tab[L.n++] = A.tab_gab[l];
            max_tiles = std::max(max_tiles, ((g.Hl[l] + 15) / 16) * ((g.Wl[l] + 15) / 16));
          }
        r = sp_pa_gabor(L, max_tiles, A.taps, c->stream, c->p.gabor_radius);
      }
      for (int l = g.top; l >= 1 && r == hipSuccess; --l)
        r = sp_pa_plane(0, A.tab_pyr[l], 4, n_l(l - 1), 1, nullptr, nullptr, c->stream);
      if (r == hipSuccess)
        r = sp_pa_feat(io.rgb, io.rgb_prev, c->h_sd.rgb_max_part, c->h_sd.n_rgb, A.gX[0], (int)HW,
                       grad_frames + (size_t)t * HW3, t ? grad_frames + (size_t)(t - 1) * HW3 : nullptr, c->stream);
      return r;
    });
    if ((rc = ok(e, "launch"))) return rc;
  }
  return SP_OK;
}

int sp_mse_mask_loss(sp_ctx* c, const float* prior, const uint8_t* mask, int32_t T, float* loss, float* grad_prior) {
  g_err.clear();
  if (!c || !prior || !mask || !loss) return fail(SP_EINVAL, "NULL argument");
  if (T < 1) return fail(SP_EINVAL, "T must be >= 1");
  const size_t n = (size_t)T * c->g.H * c->g.W;
  const int nblk = (int)std::min<size_t>(c->loss_nblk, (n + SP_BLOCK - 1) / SP_BLOCK);
  const LossIO L{prior, mask, grad_prior, c->loss_part, loss, (unsigned long long)n};
  hipError_t e = timed(c, JOB_LOSS, [&] { return sp_launch_loss(nullptr, &L, 1, nblk, c->stream); });
  if (e != hipSuccess) return fail(SP_EHIP, "loss launch: %s", hipGetErrorString(e));
  return SP_OK;
}

int sp_state_size(const sp_ctx* c, size_t* bytes) {
  g_err.clear();
  if (!c || !bytes) return fail(SP_EINVAL, "NULL argument");
  *bytes = (size_t)c->g.H * c->g.W * sizeof(float) + 2 * sizeof(double);
  return SP_OK;
}

int sp_get_state(sp_ctx* c, void* buf, size_t bytes) {
  g_err.clear();
  size_t need = 0;
  int rc = sp_state_size(c, &need);
  if (rc) return rc;
  if (!buf || bytes < need) return fail(SP_EINVAL, "state buffer needs %zu bytes", need);
  if (c->ssm[0]) return fail(SP_ESTATE, "the checkpoint does not hold the stochastic saliency map (ssm_r > 0)");
  const size_t HW = (size_t)c->g.H * c->g.W;
  HIPCHK(hipMemcpyAsync(buf, c->pi_state[c->cur], HW * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  double sc[2] = {(double)c->t, c->P};
  HIPCHK(hipMemcpyAsync((char*)buf + HW * sizeof(float), sc, sizeof sc, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SP_OK;
}

int sp_set_state(sp_ctx* c, const void* buf, size_t bytes) {
  g_err.clear();
  size_t need = 0;
  int rc = sp_state_size(c, &need);
  if (rc) return rc;
  if (!buf || bytes < need) return fail(SP_EINVAL, "state buffer needs %zu bytes", need);
  if (c->ssm[0]) return fail(SP_ESTATE, "the checkpoint does not hold the stochastic saliency map (ssm_r > 0)");
  const size_t HW = (size_t)c->g.H * c->g.W;
  double sc[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(sc, (const char*)buf + HW * sizeof(float), sizeof sc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  // the step count must be a whole number that an int64_t holds
  if (!(sc[0] >= 0 && sc[0] < 9.0e18) || sc[0] != std::floor(sc[0]) || !std::isfinite(sc[1]) || sc[1] < 0)
    return fail(SP_EINVAL, "state buffer holds an invalid header");
  HIPCHK(hipMemcpyAsync(c->pi_state[c->cur], buf, HW * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  c->t = (int64_t)sc[0];
  c->P = sc[1];
  c->tape_ok = false;
  c->tape_gen += 1;
  return SP_OK;
}

int sp_profile_enable(sp_ctx* c, int32_t enable) {
  g_err.clear();
  if (!c) return fail(SP_EINVAL, "ctx is NULL");
  return c->prof.enable(enable != 0);
}

static_assert(JOB_NKINDS == SP_NKINDS, "kernel kinds and the public SP_NKINDS disagree");
static_assert(SP_NOALLOC_BYTES == SP_NOALLOC_MAX_BYTES, "scratch size and the public SP_NOALLOC_MAX_BYTES disagree");

int sp_profile_read(sp_ctx* c, int32_t n, float* total_ms, int32_t* launches) {
  g_err.clear();
  if (!c) return fail(SP_EINVAL, "ctx is NULL");
  return c->prof.read(c->stream, n, total_ms, launches);
}

int sp_calibration_copy(const void* src, void* dst, size_t bytes, int32_t mode, void* hip_stream) {
  g_err.clear();
  if (!src || !dst) return fail(SP_EINVAL, "src and dst must not be NULL");
  if (bytes == 0 || bytes % 16 != 0 || bytes > (size_t(1) << 31))
    return fail(SP_EINVAL, "bytes must be a positive multiple of 16, at most 2 GiB");
  if (mode < 0 || mode > 2) return fail(SP_EINVAL, "mode must be 0, 1 or 2");
  hipError_t e = sp_launch_calib(static_cast<const float*>(src), static_cast<float*>(dst), bytes / 16, mode,
                                 (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(SP_EHIP, "calibration launch: %s", hipGetErrorString(e));
  return SP_OK;
}

const char* sp_kernel_name(int32_t k) {
  // launch kinds: a pyramid launch is timed under the kind of its phase (k_pyr small
  // for DOWN/GABOR stages, k_pyr tail for the final stage with tail jobs)
  static const char* names[SP_NKINDS] = {"k_rgb", "k_feat", "k_pyr", "k_pyr", "k_csstats", "k_csapply",
                                         "k_consp", "k_smax", "k_kalman", "k_mrf", "k_bwd_nu", "k_bwd_gs",
                                         "k_consp_dot", "k_loss", "k_pyr_tail", "k_pyr_tail", "k_csfinal", "k_csg", "k_csmix",
                                         "k_bwd_final", "k_dt", "k_manual", "k_gmm_acc", "k_gmm_fit",
                                         "k_gmm_psi", "k_cut_init", "k_cut_relabel", "k_cut_push",
                                         "k_pixel_adjoint"};
  return (k >= 0 && k < SP_NKINDS) ? names[k] : "";
}

}  // extern "C"

// ---------------------------------------------------------------- batched step
// Adjoint buffers of one stream of a batch with a tape.
struct BatchAdj {
  float* nu[2];        // [H][W] masked adjoint ping-pong
  float* gu;           // [H][W] adjoint of the unclamped observation
  float* gs_all;       // [cap][Hc][Wc]
  float* gk_part;      // [cap][n_lvl0_tiles]
  float* dot_part;     // [cap][n_cmax_tiles][8]
  float* cx;           // [cap][8]
  double* gK;          // [cap]
  float* loss_part;    // [loss_nblk]
  int n_lvl0_tiles;
};

// Pinned host buffer for a table uploaded asynchronously.  Refilling waits for the event
// recorded after the last upload, so the copy engine has consumed it first.
struct HostStage {
  char* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  int init(size_t n) {
    if (hipHostMalloc((void**)&host, std::max<size_t>(n, 256), 0) != hipSuccess) {
      (void)hipGetLastError();
      host = nullptr;
      return fail(SP_ENOMEM, "hipHostMalloc of %zu bytes failed", n);
    }
    bytes = n;
    HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    return SP_OK;
  }
  int acquire() {
    if (pending) HIPCHK(hipEventSynchronize(done));
    pending = false;
    return SP_OK;
  }
  int upload(void* dev, size_t n, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(dev, host, n, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(done, st));
    pending = true;
    return SP_OK;
  }
  void destroy() {
    if (done) (void)hipEventDestroy(done);
    if (host) (void)hipHostFree(host);
    done = nullptr;
    host = nullptr;
  }
};

struct sp_batch {
  sp_params p{};
  int n = 0;
  hipStream_t stream = nullptr;     // caller's stream: graph launches go here
  hipStream_t cap_stream = nullptr; // private stream used only to capture the graph
  char* arena = nullptr;
  std::vector<Geo> geo;
  std::vector<StreamDesc> h_sd;
  StreamDesc* d_sd = nullptr;
  StepIO* d_io = nullptr;
  BatchState* d_st = nullptr;
  std::vector<BatchState> h_st;
  const uint8_t* const* in_node = nullptr;   // frame table the captured graph reads
  hipGraphNode_t rgb_node = nullptr;         // its first node: colour statistics + step start
  RgbNodeArgs rgb_args{};
  JobStore jobs;
  std::vector<Phase> phases;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // several consecutive steps in one graph (sp_batch_steps): captured for mn steps, step k's
  // first node reading the frame table mtab[k]
  hipGraph_t mgraph = nullptr;
  hipGraphExec_t mexec = nullptr;
  int mn = 0;
  std::vector<hipGraphNode_t> mnodes;
  std::vector<const uint8_t* const*> mtab;
  std::vector<RgbNodeArgs> margs;
  long long steps = 0;
  Profiler prof;
  bool mrf = false;
  std::vector<Tune> tune;   // per stream
  bool xcd = false;
  int ca_nc = 2;            // preferred channels per across-scale workgroup (one value per launch)
  // tape and adjoint (record_tape > 0): every stream records the same steps
  int cap = 0;              // frames each stream's tape holds
  int CH = 0;               // frames of every stream per recompute chunk
  bool tape_ok = true;      // false once the weights changed after recorded steps
  long long tape_gen = 0;   // bumped whenever the recorded clip stops being the current one
  std::vector<BatchAdj> adj;                  // per stream: adjoint buffers
  std::vector<StreamDesc> h_rsd;              // [CH * n] recompute streams (v = j * n + i)
  StreamDesc* d_rsd = nullptr;
  StepIO* d_rio = nullptr;                    // [cap][n] checkpoint and adjoint buffers of each frame
  char* d_bstage = nullptr;                   // gains, variances, [cap][n] BwdIO, [n] BwdFin
  char* d_lstage = nullptr;                   // [n] LossIO
  HostStage bstage, lstage;                   // pinned host copies of the two tables
  std::vector<Phase> bwd, rec;                // adjoint sweep (2 launches per step), recompute program
  int loss_nblk = 1024;
};

namespace {

// Job tables of the batched adjoint: the level-0 sweep and the up-sample transpose over
// every stream (one launch each per reverse step), and the recompute program over the
// CH * n recompute streams of a chunk (recompute stream v = j * n + i takes frame t0 + j of
// stream i).  Each phase lists its jobs in recompute-stream order, so a chunk of rem < CH
// frames launches the prefix of rem * n streams.  Streams of different sizes may have
// different numbers of pyramid stages: middle stages are merged by index and every final
// stage goes to one last pyramid launch (its kernel handles every pyramid job kind).
void batch_adjoint_tables(sp_batch* b, int nc, size_t lds_a, size_t lds_g) {
  const int n = b->n, nv = b->CH * n;
  std::vector<Job> nu, gs;
  for (int i = 0; i < n; ++i) {
    const Geo& g = b->geo[i];
    add_tiles(nu, i, 0, g.H, g.W);
    add_tiles(gs, i, 0, g.Hl[g.c_max], g.Wl[g.c_max]);
  }
  b->bwd.clear();
  b->bwd.push_back(b->jobs.add(JOB_BWD_NU, 0, nu, n));
  b->bwd.push_back(b->jobs.add(JOB_BWD_GS, 0, gs, n));
  std::vector<std::vector<Job>> mids;
  std::vector<Job> fin, css, csg, csf, csa, csm, dot;
  bool any_tail = false;
  int set = 1;
  for (int v = 0; v < nv; ++v) {
    const int i = v % n;
    const Geo& g = b->geo[i];
    std::vector<std::vector<Job>> parts;
    std::vector<int> kinds;
    build_forward_jobs(parts, kinds, b->h_rsd[v], g, v, PROG_RECOMPUTE, nc);
    size_t np = 0;   // leading pyramid stages; the last of them is the final one
    while (np < parts.size() && (kinds[np] == JOB_DOWN || kinds[np] == JOB_TAIL)) ++np;
    for (size_t k = 0; k + 1 < np; ++k) {
      if (mids.size() <= k) mids.resize(k + 1);
      mids[k].insert(mids[k].end(), parts[k].begin(), parts[k].end());
    }
    if (np > 0) {
      fin.insert(fin.end(), parts[np - 1].begin(), parts[np - 1].end());
      any_tail |= kinds[np - 1] == JOB_TAIL;
    }
    for (size_t k = np; k < parts.size(); ++k) {
      std::vector<Job>* dst = nullptr;
      switch (kinds[k]) {
        case JOB_CSSTATS: dst = &css; break;
        case JOB_CSG: dst = &csg; set = std::min(set, csg_set(g)); break;
        case JOB_CSFINAL: dst = &csf; break;
        case JOB_CSAPPLY: dst = &csa; break;
        case JOB_CSMIX: dst = &csm; break;
        default: dst = &dot; break;
      }
      dst->insert(dst->end(), parts[k].begin(), parts[k].end());
    }
  }
  b->rec.clear();
  for (auto& m : mids) b->rec.push_back(b->jobs.add(JOB_DOWN, b->p.gabor_radius, m, nv));
  if (!fin.empty()) b->rec.push_back(b->jobs.add(any_tail ? JOB_TAIL : JOB_DOWN, b->p.gabor_radius, fin, nv));
  if (!css.empty()) b->rec.push_back(b->jobs.add(JOB_CSSTATS, 0, css, nv));
  if (!csg.empty()) {
    b->rec.push_back(b->jobs.add(JOB_CSG, nc | (set << 8), csg, nv));
    b->rec.back().lds = nc * lds_g;
  }
  if (!csf.empty()) b->rec.push_back(b->jobs.add(JOB_CSFINAL, 0, csf, nv));
  if (!csa.empty()) {
    b->rec.push_back(b->jobs.add(JOB_CSAPPLY, nc, csa, nv));
    b->rec.back().lds = nc * lds_a;
  }
  if (!csm.empty()) b->rec.push_back(b->jobs.add(JOB_CSMIX, 0, csm, nv));
  b->rec.push_back(b->jobs.add(JOB_CONSP_DOT, 0, dot, nv));
}

// Drops the graph of several steps (recaptured by the next sp_batch_steps).
void batch_drop_multi(sp_batch* b) {
  if (b->mexec) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(b->mexec);
    b->mexec = nullptr;
  }
  if (b->mgraph) {
    (void)hipGraphDestroy(b->mgraph);
    b->mgraph = nullptr;
  }
  b->mn = 0;
  b->mnodes.clear();
  b->mtab.clear();
  b->margs.clear();
}

// (Re)builds the batch's phase program: one launch per phase over every stream.  Drops
// the captured graphs, which are captured again on the next step.
int batch_build_tables(sp_batch* b) {
  const int n = b->n;
  if (b->exec) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  batch_drop_multi(b);
  b->rgb_node = nullptr;
  b->in_node = nullptr;
  b->jobs.host.clear();
  b->phases.clear();
  std::vector<Job> rgb, feat, fin, css, csf, csa, csg, csm, cons, kal;
  std::vector<std::vector<Job>> mids;
  bool any_big = false;
  int nc = 8;   // one channel-group size for the whole across-scale launch
  for (int i = 0; i < n; ++i) nc = std::min(nc, csapply_nc(b->geo[i], b->ca_nc));
  for (int i = 0; i < n; ++i) {
    const Geo& g = b->geo[i];
    if (!gpath_ok(g))   // the reduced-map path's mix computes the N parameters itself
      for (int p = 0; p < g.n_pairs; ++p) csf.push_back(Job{i, p, 0, 0, 1, 1, p, JOB_CSFINAL});
    rgb_jobs(rgb, i, b->h_sd[i], g);
    add_tiles(feat, i, 1, g.Hl[1], g.Wl[1], JOB_FEAT);
    std::vector<std::vector<Job>> mid;
    std::vector<Job> f;
    bool big = false;
    pyramid_stages(g, i, 1, mid, f, &big);
    any_big |= big;
    if (mids.size() < mid.size()) mids.resize(mid.size());
    for (size_t j = 0; j < mid.size(); ++j) mids[j].insert(mids[j].end(), mid[j].begin(), mid[j].end());
    fin.insert(fin.end(), f.begin(), f.end());
    if (gpath_ok(g)) {
      for (int k = 0; k < SP_NCH; k += nc) add_tiles(csg, i, k, g.Hl[g.c_max], g.Wl[g.c_max], JOB_CSG);
      add_tiles(csm, i, 0, g.Hl[g.c_max], g.Wl[g.c_max], JOB_CSMIX);
    } else {
      for (int c = 0; c <= g.top; ++c) {
        bool has = false;
        for (int k = 0; k < g.n_pairs; ++k) has |= (g.pc[k] == c);
        if (has) add_tiles(css, i, c, g.Hl[c], g.Wl[c]);
      }
      for (int k = 0; k < SP_NCH; k += nc) add_tiles(csa, i, k, g.Hl[g.c_max], g.Wl[g.c_max]);
    }
    add_tiles(cons, i, 0, g.Hl[g.c_max], g.Wl[g.c_max]);
    add_tiles_wh(kal, i, 0, g.H, g.W, SP_KAL_ROWS, b->tune[i].kalman_tw, JOB_KALMAN);
  }
  auto order = [&](std::vector<Job> v) {
    if (b->xcd) xcd_order(v);
    return v;
  };
  // tail jobs first in the final pyramid launch (they are the longest workgroups), each
  // group in its own XCD order so a stream's jobs stay on the XCD that produced its levels
  {
    std::vector<Job> tails, rest;
    for (const Job& jb : fin) (jb.kind == JOB_TAIL || jb.kind == JOB_TAILGAB ? tails : rest).push_back(jb);
    fin = order(tails);
    rest = order(rest);
    fin.insert(fin.end(), rest.begin(), rest.end());
  }
  b->phases.push_back(b->jobs.add(JOB_RGB, b->mrf ? 1 : 0, order(rgb), n));
  b->phases.push_back(b->jobs.add(JOB_FEAT, 0, order(feat), n));
  for (auto& d : mids) {
    if (d.empty()) continue;
    // every stream's Gabor tiles (the longer jobs) before the next level's tiles, each
    // group in its own XCD order
    std::vector<Job> gab, down;
    for (const Job& jb : d) (jb.kind == JOB_GABOR ? gab : down).push_back(jb);
    std::vector<Job> all = order(gab), rest = order(down);
    all.insert(all.end(), rest.begin(), rest.end());
    b->phases.push_back(b->jobs.add(JOB_DOWN, b->p.gabor_radius, all, n));
  }
  if (!fin.empty()) b->phases.push_back(b->jobs.add(any_big ? JOB_TAIL : JOB_DOWN, b->p.gabor_radius, fin, n));
  size_t lds_a = 0, lds_g = 0;
  for (const Geo& g : b->geo) {
    if (gpath_ok(g))
      lds_g = std::max(lds_g, csg_lds_bytes(g));
    else
      lds_a = std::max(lds_a, csapply_lds_bytes(g));
  }
  if (sp_csapply_reserve_lds(nc * std::max(lds_a, lds_g)) != hipSuccess)
    return fail(SP_EHIP, "cannot reserve %zu bytes of LDS for the across-scale sum", nc * std::max(lds_a, lds_g));
  if (!css.empty()) b->phases.push_back(b->jobs.add(JOB_CSSTATS, 0, order(css), n));
  if (!csg.empty()) {
    int set = 1;
    for (const Geo& g : b->geo)
      if (gpath_ok(g)) set = std::min(set, csg_set(g));
    b->phases.push_back(b->jobs.add(JOB_CSG, nc | (set << 8), order(csg), n));
    b->phases.back().lds = nc * lds_g;
  }
  if (!csf.empty()) b->phases.push_back(b->jobs.add(JOB_CSFINAL, 0, order(csf), n));
  if (!csa.empty()) {
    b->phases.push_back(b->jobs.add(JOB_CSAPPLY, nc, order(csa), n));
    b->phases.back().lds = nc * lds_a;
  }
  if (!csm.empty()) b->phases.push_back(b->jobs.add(JOB_CSMIX, 0, order(csm), n));
  b->phases.push_back(b->jobs.add(JOB_CONSP, 0, order(cons), n));
  b->phases.push_back(b->jobs.add(JOB_KALMAN, 0, order(kal), n));
  if (b->cap > 0) batch_adjoint_tables(b, nc, lds_a, lds_g);
  return upload_jobs(b->jobs, b->stream);
}

// One step's launches.  The first phase (colour statistics) also starts the step and
// reads the frames from in_ptrs; with node set (under capture) its graph node is kept so
// later steps can point it at their own frame tables.
int batch_enqueue(sp_batch* b, hipStream_t st, const uint8_t* const* in_ptrs, hipGraphNode_t* node = nullptr) {
  bool first = true;
  for (const Phase& ph : b->phases) {
    hipError_t e;
    if (first) {
      if (ph.kind != JOB_RGB) return fail(SP_ESTATE, "batched step must start with the colour statistics");
      const BatchBegin bb{in_ptrs, b->d_st, b->d_io, b->n, 0, b->p.q, b->p.r};
      e = b->prof.timed(st, ph.kind, [&] {
        return sp_launch_batch_rgb(b->jobs.dev + ph.off, ph.n, b->d_sd, b->d_io, ph.flag, bb, st);
      });
      if (e == hipSuccess && node) {
        hipStreamCaptureStatus cs;
        const hipGraphNode_t* deps = nullptr;
        size_t nd = 0;
        e = hipStreamGetCaptureInfo_v2(st, &cs, nullptr, nullptr, &deps, &nd);
        if (e == hipSuccess && (cs != hipStreamCaptureStatusActive || nd != 1))
          return fail(SP_EHIP, "graph capture: cannot find the first node");
        if (e == hipSuccess) *node = deps[0];
      }
      first = false;
    } else {
      e = b->prof.timed(st, ph.kind, [&] {
        return sp_launch(ph.kind, b->jobs.dev + ph.off, ph.n, b->d_sd, b->d_io, nullptr, ph.flag, nullptr, st, ph.lds);
      });
    }
    if (e != hipSuccess) return fail(SP_EHIP, "batch phase launch (kind %d): %s", ph.kind, hipGetErrorString(e));
  }
  return SP_OK;
}

// Points a step's first node (colour statistics + step start) of an instantiated graph at
// the frame table in_ptrs; a holds the node's arguments.
int point_rgb_node(sp_batch* b, hipGraphExec_t ex, hipGraphNode_t node, RgbNodeArgs& a,
                   const uint8_t* const* in_ptrs) {
  const Phase& ph = b->phases.front();
  a.jobs = b->jobs.dev + ph.off;
  a.sds = b->d_sd;
  a.ios = b->d_io;
  a.io0 = StepIO{};
  a.want_d2 = ph.flag;
  a.bb = BatchBegin{in_ptrs, b->d_st, b->d_io, b->n, 0, b->p.q, b->p.r};
  hipKernelNodeParams kp;
  sp_batch_rgb_node_params(&a, ph.n, &kp);
  HIPCHK(hipGraphExecKernelNodeSetParams(ex, node, &kp));
  return SP_OK;
}

// Points the captured graph's first node at this step's frame table.
int batch_point_graph(sp_batch* b, const uint8_t* const* in_ptrs) {
  if (in_ptrs == b->in_node) return SP_OK;
  const int rc = point_rgb_node(b, b->exec, b->rgb_node, b->rgb_args, in_ptrs);
  if (rc) return rc;
  b->in_node = in_ptrs;
  return SP_OK;
}

// Captures the whole step once on the private stream (graph kept until the tables change),
// reading the frames from in_ptrs until batch_point_graph points it elsewhere.
int batch_capture(sp_batch* b, const uint8_t* const* in_ptrs) {
  HIPCHK(hipStreamSynchronize(b->stream));
  HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  const bool was = b->prof.on;
  b->prof.on = false;
  hipGraphNode_t node = nullptr;
  int rc = batch_enqueue(b, b->cap_stream, in_ptrs, &node);
  b->prof.on = was;
  hipGraph_t gr = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &gr);
  if (rc) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  if (e != hipSuccess) return fail(SP_EHIP, "graph capture: %s", hipGetErrorString(e));
  b->graph = gr;
  HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->rgb_node = node;
  b->in_node = in_ptrs;
  return SP_OK;
}

// Captures n consecutive steps in one graph on the private stream, step k reading the
// frame table tabs[k] until point_rgb_node points its first node elsewhere.
int batch_capture_multi(sp_batch* b, int n, const uint8_t* const* const* tabs) {
  batch_drop_multi(b);
  HIPCHK(hipStreamSynchronize(b->stream));
  HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  const bool was = b->prof.on;
  b->prof.on = false;
  std::vector<hipGraphNode_t> nodes((size_t)n, nullptr);
  int rc = SP_OK;
  for (int k = 0; k < n && rc == SP_OK; ++k) rc = batch_enqueue(b, b->cap_stream, tabs[k], &nodes[(size_t)k]);
  b->prof.on = was;
  hipGraph_t gr = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &gr);
  if (rc) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  if (e != hipSuccess) return fail(SP_EHIP, "graph capture: %s", hipGetErrorString(e));
  b->mgraph = gr;
  HIPCHK(hipGraphInstantiate(&b->mexec, b->mgraph, nullptr, nullptr, 0));
  b->mn = n;
  b->mnodes = nodes;
  b->mtab.assign(tabs, tabs + n);
  b->margs.assign((size_t)n, RgbNodeArgs{});
  return SP_OK;
}

void batch_free(sp_batch* b) {
  if (!b) return;
  if (b->stream || b->arena) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->mexec) (void)hipGraphExecDestroy(b->mexec);
  if (b->mgraph) (void)hipGraphDestroy(b->mgraph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  b->prof.destroy();
  b->bstage.destroy();
  b->lstage.destroy();
  if (b->arena) (void)hipFree(b->arena);
  if (b->jobs.dev) (void)hipFree(b->jobs.dev);
  delete b;
}

}  // namespace

extern "C" {

int sp_batch_create(const sp_params* p, int32_t n, const int32_t* H, const int32_t* W, int32_t flags,
                    void* hip_stream, sp_batch** out) {
  g_err.clear();
  if (!out) return fail(SP_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > 4096) return fail(SP_EINVAL, "batch size must be 1..4096 (got %d)", n);
  if (!H || !W) return fail(SP_EINVAL, "H and W must not be NULL");
  int rc = validate_params(p);
  if (rc) return rc;
  if (flags & ~(SP_BATCH_MRF | SP_BATCH_CONSP)) return fail(SP_EINVAL, "unknown batch flags 0x%x", flags);
  if (p->f_mode != 0 || p->ssm_r > 0)
    return fail(SP_EINVAL, "the batched step runs the default prior (f_mode 0, no stochastic map)");
  const bool mrf = (flags & SP_BATCH_MRF) != 0;
  const bool consp = (flags & SP_BATCH_CONSP) != 0;
  sp_batch* b = new (std::nothrow) sp_batch();
  if (!b) return fail(SP_ENOMEM, "host allocation failed");
  b->p = *p;
  b->n = n;
  b->stream = (hipStream_t)hip_stream;
  b->geo.resize(n);
  for (int i = 0; i < n; ++i) {
    rc = make_geo(*p, H[i], W[i], b->geo[i]);
    if (rc) {
      batch_free(b);
      return fail(rc, "stream %d: %s", i, g_err.c_str());
    }
  }
  b->h_sd.resize(n);
  b->h_st.resize(n);
  b->cap = p->record_tape;
  // recompute chunks of about 64 recompute streams (at least one frame per stream)
  b->CH = b->cap > 0 ? std::max(1, std::min({b->cap, 32, (64 + n - 1) / n})) : 0;
  b->adj.resize(b->cap > 0 ? n : 0);
  b->h_rsd.resize((size_t)b->CH * n);
  const size_t bstage_bytes = b->cap > 0 ? 2 * sizeof(double) * b->cap + sizeof(BwdIO) * (size_t)b->cap * n +
                                               sizeof(BwdFin) * n : 0;
  const size_t lstage_bytes = b->cap > 0 ? sizeof(LossIO) * n : 0;
  size_t bytes = 0;
  for (int pass = 0; pass < 2; ++pass) {
    Bump bm;
    bm.base = b->arena;
    for (int i = 0; i < n; ++i) {
      // the colour-statistics launch holds every stream's tiles: aim at ~192 in total
      layout_stream(b->h_sd[i], b->geo[i], *p, bm, 1, true, std::max(1, 192 / n));
      const Geo& g = b->geo[i];
      BatchState& s = b->h_st[i];
      std::memset(&s, 0, sizeof s);
      s.pi[0] = bm.take<float>((size_t)g.H * g.W);
      s.pi[1] = bm.take<float>((size_t)g.H * g.W);
      s.S = bm.take<float>((size_t)g.Hl[g.c_max] * g.Wl[g.c_max]);
      if (mrf) {
        s.unary = bm.take<float>((size_t)2 * g.H * g.W);
        s.pairwise = bm.take<float>((size_t)4 * g.H * g.W);
        s.beta = bm.take<float>(1);
      }
      if (consp) s.C = bm.take<float>((size_t)SP_NCH * g.Hl[g.c_max] * g.Wl[g.c_max]);
      if (b->cap > 0) {
        const size_t cap = (size_t)b->cap, hw = (size_t)g.H * g.W, plane = (size_t)g.Hl[g.c_max] * g.Wl[g.c_max];
        s.tape_cap = b->cap;
        s.tape_ckpt = bm.take<float>(cap * 4 * g.Hl[g.c_min] * g.Wl[g.c_min]);
        s.tape_S = bm.take<float>(cap * plane);
        s.tape_f = bm.take<float>(cap * hw);
        s.tape_ms = bm.take<float>(cap * 2);
        s.tape_pi = bm.take<float>(cap * hw);
        BatchAdj& a = b->adj[i];
        a.n_lvl0_tiles = ntiles(g.H, g.W);
        a.nu[0] = bm.take<float>(hw);
        a.nu[1] = bm.take<float>(hw);
        a.gu = bm.take<float>(hw);
        a.gs_all = bm.take<float>(cap * plane);
        a.gk_part = bm.take<float>(cap * a.n_lvl0_tiles);
        a.dot_part = bm.take<float>(cap * b->h_sd[i].n_cmax_tiles * SP_NCH);
        a.cx = bm.take<float>(cap * SP_NCH);
        a.gK = bm.take<double>((size_t)cap * (1 + SP_NCH));
        a.loss_part = bm.take<float>(b->loss_nblk);
      }
    }
    b->d_sd = bm.take<StreamDesc>(n);
    b->d_io = bm.take<StepIO>(n);
    b->d_st = bm.take<BatchState>(n);
    if (b->cap > 0) {
      b->d_rsd = bm.take<StreamDesc>(b->h_rsd.size());
      b->d_rio = bm.take<StepIO>((size_t)b->cap * n);
      b->d_bstage = bm.take<char>(bstage_bytes);
      b->d_lstage = bm.take<char>(lstage_bytes);
      for (size_t v = 0; v < b->h_rsd.size(); ++v) {
        const Geo& g = b->geo[v % n];
        layout_stream(b->h_rsd[v], g, *p, bm, g.c_min + 1, false);
      }
    }
    if (pass == 0) {
      bytes = bm.off + 256;
      if (hipMalloc(&b->arena, bytes) != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return fail(SP_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
      }
    }
  }
  b->mrf = mrf;
  b->tune.resize(n);
  for (int i = 0; i < n; ++i) b->tune[i] = cached_tune(H[i], W[i]);
  b->xcd = n > 0 ? b->tune[0].xcd : false;
  b->ca_nc = n > 0 ? b->tune[0].ca_nc : 2;
  {
    size_t lds = 0;
    for (const Geo& g : b->geo) lds = std::max(lds, csapply_lds_bytes(g));
    if (sp_csapply_reserve_lds(lds) != hipSuccess) {
      batch_free(b);
      return fail(SP_EHIP, "cannot reserve %zu bytes of LDS for the across-scale sum", lds);
    }
  }
  rc = batch_build_tables(b);
  if (rc) {
    std::string msg = g_err;
    batch_free(b);
    g_err = msg;
    return rc;
  }
  hipError_t e = hipMemcpy(b->d_sd, b->h_sd.data(), sizeof(StreamDesc) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_st, b->h_st.data(), sizeof(BatchState) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess && b->cap > 0) {
    e = hipMemcpy(b->d_rsd, b->h_rsd.data(), sizeof(StreamDesc) * b->h_rsd.size(), hipMemcpyHostToDevice);
    std::vector<StepIO> rio((size_t)b->cap * n);
    for (int t = 0; t < b->cap; ++t)
      for (int i = 0; i < n; ++i) {
        const Geo& g = b->geo[i];
        const BatchState& s = b->h_st[i];
        const BatchAdj& a = b->adj[i];
        StepIO& io = rio[(size_t)t * n + i];
        std::memset(&io, 0, sizeof io);
        io.ckpt = s.tape_ckpt + (size_t)t * 4 * g.Hl[g.c_min] * g.Wl[g.c_min];
        io.gs = a.gs_all + (size_t)t * g.Hl[g.c_max] * g.Wl[g.c_max];
        io.ms_tape = s.tape_ms + 2 * (size_t)t;
        io.dot = a.dot_part + (size_t)t * b->h_sd[i].n_cmax_tiles * SP_NCH;
        io.cx = a.cx + (size_t)t * SP_NCH;
      }
    if (e == hipSuccess) e = hipMemcpy(b->d_rio, rio.data(), sizeof(StepIO) * rio.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    batch_free(b);
    return fail(SP_EHIP, "batch set-up: %s", hipGetErrorString(e));
  }
  if (b->cap > 0 && (b->bstage.init(bstage_bytes) || b->lstage.init(lstage_bytes))) {
    std::string msg = g_err;
    batch_free(b);
    g_err = msg;
    return SP_ENOMEM;
  }
  *out = b;
  return SP_OK;
}

int sp_batch_step(sp_batch* b, const uint8_t* const* rgb_ptrs, float* const* prior_ptrs) {
  g_err.clear();
  if (!b || !rgb_ptrs) return fail(SP_EINVAL, "batch and rgb_ptrs must not be NULL");
  if (b->cap > 0 && b->steps >= b->cap)
    return fail(SP_ESTATE, "the tape holds %d frames per stream; call sp_batch_reset before step %lld", b->cap,
                (long long)b->steps);
  if (b->prof.on) {
    // measurement: the same phases, launched one by one with events around each
    int rc = batch_enqueue(b, b->stream, rgb_ptrs);
    if (rc) return rc;
    b->steps += 1;
    if (prior_ptrs) {
      hipError_t e = sp_launch_batch_copy_out(b->n, b->d_st, b->d_sd, prior_ptrs, b->stream);
      if (e != hipSuccess) return fail(SP_EHIP, "copy-out launch: %s", hipGetErrorString(e));
    }
    return SP_OK;
  }
  if (!b->exec) {
    const int rc = batch_capture(b, rgb_ptrs);
    if (rc) return rc;
  } else {
    const int rc = batch_point_graph(b, rgb_ptrs);
    if (rc) return rc;
  }
  HIPCHK(hipGraphLaunch(b->exec, b->stream));
  b->steps += 1;
  if (prior_ptrs) {
    hipError_t e = sp_launch_batch_copy_out(b->n, b->d_st, b->d_sd, prior_ptrs, b->stream);
    if (e != hipSuccess) return fail(SP_EHIP, "copy-out launch: %s", hipGetErrorString(e));
  }
  return SP_OK;
}

int sp_batch_steps(sp_batch* b, int32_t n, const uint8_t* const* const* rgb_tables) {
  g_err.clear();
  if (!b || !rgb_tables) return fail(SP_EINVAL, "batch and rgb_tables must not be NULL");
  if (n < 1 || n > 1024) return fail(SP_EINVAL, "steps per call must be 1..1024 (got %d)", n);
  for (int k = 0; k < n; ++k)
    if (!rgb_tables[k]) return fail(SP_EINVAL, "frame table %d is NULL", k);
  if (b->cap > 0 && b->steps + n > b->cap)
    return fail(SP_ESTATE, "the tape holds %d frames per stream; %d steps after step %lld do not fit", b->cap, n,
                (long long)b->steps);
  if (b->prof.on) {   // measurement: every step's phases launched one by one with events
    for (int k = 0; k < n; ++k) {
      const int rc = batch_enqueue(b, b->stream, rgb_tables[k]);
      if (rc) return rc;
      b->steps += 1;
    }
    return SP_OK;
  }
  if (!b->mexec || b->mn != n) {
    const int rc = batch_capture_multi(b, n, rgb_tables);
    if (rc) return rc;
  } else {
    for (int k = 0; k < n; ++k)
      if (rgb_tables[k] != b->mtab[(size_t)k]) {
        const int rc = point_rgb_node(b, b->mexec, b->mnodes[(size_t)k], b->margs[(size_t)k], rgb_tables[k]);
        if (rc) return rc;
        b->mtab[(size_t)k] = rgb_tables[k];
      }
  }
  HIPCHK(hipGraphLaunch(b->mexec, b->stream));
  b->steps += n;
  return SP_OK;
}

int sp_batch_prior(sp_batch* b, int32_t i, const float** prior) {
  g_err.clear();
  if (!b || !prior) return fail(SP_EINVAL, "NULL argument");
  if (i < 0 || i >= b->n) return fail(SP_EINVAL, "stream index %d out of range", i);
  if (b->steps == 0) return fail(SP_ESTATE, "no step has run since the reset");
  *prior = b->h_st[i].pi[b->steps & 1];
  return SP_OK;
}

int sp_batch_outputs(sp_batch* b, int32_t i, const float** S, const float** unary, const float** pairwise,
                     const float** beta) {
  g_err.clear();
  if (!b) return fail(SP_EINVAL, "batch is NULL");
  if (i < 0 || i >= b->n) return fail(SP_EINVAL, "stream index %d out of range", i);
  if (S) *S = b->h_st[i].S;
  if (unary) *unary = b->h_st[i].unary;
  if (pairwise) *pairwise = b->h_st[i].pairwise;
  if (beta) *beta = b->h_st[i].beta;
  return SP_OK;
}

int sp_batch_consp(sp_batch* b, int32_t i, const float** C) {
  g_err.clear();
  if (!b || !C) return fail(SP_EINVAL, "NULL argument");
  if (i < 0 || i >= b->n) return fail(SP_EINVAL, "stream index %d out of range", i);
  *C = b->h_st[i].C;
  return SP_OK;
}

int sp_batch_reset(sp_batch* b) {
  g_err.clear();
  if (!b) return fail(SP_EINVAL, "batch is NULL");
  hipError_t e = sp_launch_batch_reset(b->n, b->d_st, b->stream);
  if (e != hipSuccess) return fail(SP_EHIP, "reset launch: %s", hipGetErrorString(e));
  b->steps = 0;
  b->tape_ok = true;
  b->tape_gen += 1;
  return SP_OK;
}

int sp_batch_profile_enable(sp_batch* b, int32_t enable) {
  g_err.clear();
  if (!b) return fail(SP_EINVAL, "batch is NULL");
  return b->prof.enable(enable != 0);
}

int sp_batch_profile_read(sp_batch* b, int32_t n, float* total_ms, int32_t* launches) {
  g_err.clear();
  if (!b) return fail(SP_EINVAL, "batch is NULL");
  return b->prof.read(b->stream, n, total_ms, launches);
}

int sp_batch_autotune(sp_batch* b, const uint8_t* const* rgb_ptrs, int32_t steps, char* report, size_t report_len) {
  g_err.clear();
  if (!b || !rgb_ptrs) return fail(SP_EINVAL, "batch and rgb_ptrs must not be NULL");
  if (steps < 1 || steps > 1000) return fail(SP_EINVAL, "steps must be 1..1000");
  HIPCHK(hipStreamSynchronize(b->stream));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const bool was = b->prof.on;
  b->prof.on = false;
  std::string rep;
  int rc = SP_OK;
  auto time_it = [&](double* ms) -> int {   // replays of the captured step, as deployed
    int r = batch_build_tables(b);
    if (r) return r;
    r = batch_capture(b, rgb_ptrs);
    if (r) return r;
    HIPCHK(hipGraphLaunch(b->exec, b->stream));   // warm-up
    HIPCHK(hipEventRecord(e0, b->stream));
    for (int i = 0; i < steps; ++i) HIPCHK(hipGraphLaunch(b->exec, b->stream));
    HIPCHK(hipEventRecord(e1, b->stream));
    HIPCHK(hipEventSynchronize(e1));
    float f = 0.f;
    HIPCHK(hipEventElapsedTime(&f, e0, e1));
    *ms = f / steps;
    return SP_OK;
  };
  char line[160];
  double best = 1e30, t = 0;
  bool best_x = b->xcd;
  for (int x = 0; x < 2 && !rc; ++x) {
    b->xcd = x != 0;
    rc = time_it(&t);
    snprintf(line, sizeof line, "xcd_order=%d: %.4f ms/step\n", x, t);
    rep += line;
    if (!rc && t < best) {
      best = t;
      best_x = b->xcd;
    }
  }
  b->xcd = best_x;
  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int i = 0; i < b->n; ++i) groups[{b->geo[i].H, b->geo[i].W}].push_back(i);
  for (auto& kv : groups) {
    if (rc) break;
    int best_tw = b->tune[kv.second[0]].kalman_tw;
    double bt = 1e30;
    for (int tw : {16, 32, 64}) {
      for (int i : kv.second) b->tune[i].kalman_tw = tw;
      rc = time_it(&t);
      if (rc) break;
      snprintf(line, sizeof line, "%dx%d kalman tile %dx%d: %.4f ms/step\n", kv.first.first, kv.first.second, SP_KAL_ROWS, tw, t);
      rep += line;
      if (t < bt) {
        bt = t;
        best_tw = tw;
      }
    }
    for (int i : kv.second) b->tune[i].kalman_tw = best_tw;
  }
  {
    int best_nc = b->ca_nc;
    double bt = 1e30;
    for (int nc : {1, 2, 4, 8}) {
      if (rc) break;
      bool ok = true;
      for (const Geo& g : b->geo) ok &= csapply_nc(g, nc) == nc;
      if (!ok) continue;
      b->ca_nc = nc;
      rc = time_it(&t);
      if (rc) break;
      snprintf(line, sizeof line, "across-scale channels per workgroup %d: %.4f ms/step\n", nc, t);
      rep += line;
      if (t < bt) {
        bt = t;
        best_nc = nc;
      }
    }
    b->ca_nc = best_nc;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->prof.on = was;
  if (rc) return rc;
  rc = batch_build_tables(b);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(tune_mutex());
    tune_cache_xcd() = b->xcd;
    tune_cache_nc() = b->ca_nc;
    for (int i = 0; i < b->n; ++i) tune_cache_tw()[{b->geo[i].H, b->geo[i].W}] = b->tune[i].kalman_tw;
  }
  snprintf(line, sizeof line, "chosen: xcd_order=%d, across-scale channels %d\n", (int)b->xcd, b->ca_nc);
  rep += line;
  if (report && report_len) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  hipError_t e = sp_launch_batch_reset(b->n, b->d_st, b->stream);
  if (e != hipSuccess) return fail(SP_EHIP, "reset launch: %s", hipGetErrorString(e));
  b->steps = 0;
  b->tape_ok = true;
  b->tape_gen += 1;
  HIPCHK(hipStreamSynchronize(b->stream));
  return SP_OK;
}

int sp_batch_set_tune(sp_batch* b, int32_t kalman_tw, int32_t xcd_order, int32_t channels) {
  g_err.clear();
  if (!b) return fail(SP_EINVAL, "batch is NULL");
  if (kalman_tw != 16 && kalman_tw != 32 && kalman_tw != 64) return fail(SP_EINVAL, "kalman_tw must be 16, 32 or 64");
  if (channels != 1 && channels != 2 && channels != 4 && channels != 8) return fail(SP_EINVAL, "channels must be 1, 2, 4 or 8");
  for (const Geo& g : b->geo)
    if (csapply_nc(g, channels) != channels)
      return fail(SP_EINVAL, "%d channels per across-scale workgroup exceed the LDS limit of a stream", channels);
  for (Tune& t : b->tune) t.kalman_tw = kalman_tw;
  b->xcd = xcd_order != 0;
  b->ca_nc = channels;
  return batch_build_tables(b);
}

int sp_batch_set_weights(sp_batch* b, const float* w, double q, double r) {
  g_err.clear();
  if (!b || !w) return fail(SP_EINVAL, "NULL argument");
  for (int k = 0; k < SP_NCH; ++k)
    if (!std::isfinite(w[k])) return fail(SP_EINVAL, "weight %d is not finite", k);
  if (!is_fin(q) || !is_fin(r) || q < 0 || r < 0 || !(q + r > 0))
    return fail(SP_EINVAL, "Kalman variances must be finite, >= 0 and not both 0");
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int k = 0; k < SP_NCH; ++k) b->p.weights[k] = w[k];
  b->p.q = q;
  b->p.r = r;
  for (StreamDesc& sd : b->h_sd)
    for (int k = 0; k < SP_NCH; ++k) sd.w[k] = w[k];
  for (StreamDesc& sd : b->h_rsd)
    for (int k = 0; k < SP_NCH; ++k) sd.w[k] = w[k];
  HIPCHK(hipMemcpy(b->d_sd, b->h_sd.data(), sizeof(StreamDesc) * b->n, hipMemcpyHostToDevice));
  if (b->d_rsd)
    HIPCHK(hipMemcpy(b->d_rsd, b->h_rsd.data(), sizeof(StreamDesc) * b->h_rsd.size(), hipMemcpyHostToDevice));
  // each step's first node carries Q and R: point every one of them again at its next launch
  b->in_node = nullptr;
  for (auto& t : b->mtab) t = nullptr;
  if (b->steps > 0) b->tape_ok = false;
  b->tape_gen += 1;
  return SP_OK;
}

int64_t sp_batch_tape_generation(const sp_batch* b) { return b ? b->tape_gen : -1; }

int64_t sp_batch_step_index(const sp_batch* b) { return b ? b->steps : -1; }

int sp_batch_tape_prior(sp_batch* b, int32_t i, const float** prior) {
  g_err.clear();
  if (!b || !prior) return fail(SP_EINVAL, "NULL argument");
  if (i < 0 || i >= b->n) return fail(SP_EINVAL, "stream index %d out of range", i);
  if (b->cap <= 0) return fail(SP_ESTATE, "the batch was created without a tape (record_tape = 0)");
  *prior = b->h_st[i].tape_pi;
  return SP_OK;
}

int sp_batch_mse_mask_loss(sp_batch* b, const uint8_t* const* masks, int32_t T, float* loss,
                           float* const* grad_prior) {
  g_err.clear();
  if (!b || !masks || !loss) return fail(SP_EINVAL, "NULL argument");
  if (b->cap <= 0) return fail(SP_ESTATE, "the batch was created without a tape (record_tape = 0)");
  if (T < 1 || T > b->steps || T > b->cap)
    return fail(SP_ESTATE, "loss over %d steps, but %lld are recorded since the reset", T, (long long)b->steps);
  const int n = b->n;
  size_t most = 0;
  for (int i = 0; i < n; ++i) {
    if (!masks[i]) return fail(SP_EINVAL, "mask of stream %d is NULL", i);
    if (grad_prior && !grad_prior[i]) return fail(SP_EINVAL, "grad_prior of stream %d is NULL", i);
    most = std::max(most, (size_t)T * b->geo[i].H * b->geo[i].W);
  }
  int rc = b->lstage.acquire();
  if (rc) return rc;
  LossIO* tab = reinterpret_cast<LossIO*>(b->lstage.host);
  for (int i = 0; i < n; ++i)
    tab[i] = LossIO{b->h_st[i].tape_pi, masks[i], grad_prior ? grad_prior[i] : nullptr, b->adj[i].loss_part, loss + i,
                    (unsigned long long)T * b->geo[i].H * b->geo[i].W};
  rc = b->lstage.upload(b->d_lstage, sizeof(LossIO) * n, b->stream);
  if (rc) return rc;
  const int nblk = (int)std::min<size_t>(b->loss_nblk, (most + SP_BLOCK - 1) / SP_BLOCK);
  hipError_t e = b->prof.timed(b->stream, JOB_LOSS, [&] {
    return sp_launch_loss(reinterpret_cast<const LossIO*>(b->d_lstage), nullptr, n, nblk, b->stream);
  });
  if (e != hipSuccess) return fail(SP_EHIP, "loss launch: %s", hipGetErrorString(e));
  return SP_OK;
}

int sp_batch_backward(sp_batch* b, const float* const* grad_prior, int32_t T, float* grad_w, float* grad_q,
                      float* grad_r) {
  g_err.clear();
  if (!b || !grad_prior || !grad_w || !grad_q || !grad_r) return fail(SP_EINVAL, "NULL argument");
  if (b->cap <= 0) return fail(SP_ESTATE, "the batch was created without a tape (record_tape = 0)");
  if (!b->tape_ok) return fail(SP_ESTATE, "tape invalidated by sp_batch_set_weights after recorded steps; reset");
  if (T < 1 || T != b->steps || T > b->cap)
    return fail(SP_ESTATE, "backward of %d steps, but %lld steps were recorded since the reset", T,
                (long long)b->steps);
  const int n = b->n;
  for (int i = 0; i < n; ++i)
    if (!grad_prior[i]) return fail(SP_EINVAL, "grad_prior of stream %d is NULL", i);
  // tables: the gains and variances (FP64, the device's own recursion), one BwdIO per
  // stream and step, one BwdFin per stream
  int rc = b->bstage.acquire();
  if (rc) return rc;
  char* h = b->bstage.host;
  double* Kd = reinterpret_cast<double*>(h);
  double* Pd = Kd + b->cap;
  BwdIO* bio = reinterpret_cast<BwdIO*>(Pd + b->cap);
  BwdFin* fin = reinterpret_cast<BwdFin*>(bio + (size_t)b->cap * n);
  {
    double P = 0.0;
    for (int t = 0; t < T; ++t) Kd[t] = now_gain(t, P, b->p.q, b->p.r, &P), Pd[t] = P;
  }
  const float* wdev0 = reinterpret_cast<const float*>(reinterpret_cast<const char*>(b->d_sd) + offsetof(StreamDesc, w));
  for (int i = 0; i < n; ++i) {
    const Geo& g = b->geo[i];
    const BatchState& s = b->h_st[i];
    const BatchAdj& a = b->adj[i];
    const size_t hw = (size_t)g.H * g.W, plane = (size_t)g.Hl[g.c_max] * g.Wl[g.c_max];
    for (int t = 0; t < T; ++t) {
      BwdIO& o = bio[(size_t)t * n + i];
      std::memset(&o, 0, sizeof o);
      o.grad = grad_prior[i] + (size_t)t * hw;
      o.nu_next = (t + 1 < T) ? a.nu[(t + 1) & 1] : nullptr;
      o.nu_out = a.nu[t & 1];
      o.gu = a.gu;
      o.gs = a.gs_all + (size_t)t * plane;
      o.gk_part = a.gk_part + (size_t)t * a.n_lvl0_tiles;
      o.f = (t > 0) ? s.tape_f + (size_t)t * hw : nullptr;
      o.S = s.tape_S + (size_t)t * plane;
      o.ms = s.tape_ms + 2 * (size_t)t;
      o.K = (t > 0) ? (float)Kd[t] : 1.f;
      o.carry = (t + 1 < T) ? 1.f - (float)Kd[t + 1] : 0.f;   // every later step read the previous prior
      o.t = t;
    }
    const float* wdev = reinterpret_cast<const float*>(reinterpret_cast<const char*>(wdev0) + sizeof(StreamDesc) * i);
    fin[i] = BwdFin{a.gk_part, a.dot_part, a.cx, s.tape_ms, wdev, a.gK, grad_w + (size_t)SP_NCH * i, grad_q + i,
                    grad_r + i, a.n_lvl0_tiles, b->h_sd[i].n_cmax_tiles};
  }
  rc = b->bstage.upload(b->d_bstage, b->bstage.bytes, b->stream);
  if (rc) return rc;
  const double* dKd = reinterpret_cast<const double*>(b->d_bstage);
  const double* dPd = dKd + b->cap;
  const BwdIO* dbio = reinterpret_cast<const BwdIO*>(dPd + b->cap);
  const BwdFin* dfin = reinterpret_cast<const BwdFin*>(dbio + (size_t)b->cap * n);
  // reverse sweep: per step one launch of the level-0 adjoint and one of the up-sample
  // transpose, each over every stream
  for (int t = T - 1; t >= 0; --t)
    for (const Phase& ph : b->bwd) {
      hipError_t e = b->prof.timed(b->stream, ph.kind, [&] {
        return sp_launch_bwd(ph.kind, b->jobs.dev + ph.off, ph.n, b->d_sd, dbio + (size_t)t * n, nullptr, b->stream);
      });
      if (e != hipSuccess) return fail(SP_EHIP, "adjoint launch: %s", hipGetErrorString(e));
    }
  // conspicuity maps recomputed from the checkpoints, CH frames of every stream at a time
  for (int t0 = 0; t0 < T; t0 += b->CH) {
    const int rem = std::min(b->CH, T - t0);
    const StepIO* ios = b->d_rio + (size_t)t0 * n;
    for (const Phase& ph : b->rec) {
      const int nj = ph.upto[(size_t)rem * n];
      hipError_t e = b->prof.timed(b->stream, ph.kind, [&] {
        if (ph.kind == JOB_CONSP_DOT) return sp_launch_consp_dot(b->jobs.dev + ph.off, nj, b->d_rsd, ios, b->stream);
        return sp_launch(ph.kind, b->jobs.dev + ph.off, nj, b->d_rsd, ios, nullptr, ph.flag, nullptr, b->stream,
                         ph.lds);
      });
      if (e != hipSuccess) return fail(SP_EHIP, "recompute launch: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = b->prof.timed(b->stream, JOB_BWD_FINAL, [&] {
    return sp_launch_bwd_final(dfin, nullptr, n, T, dKd, dPd, b->p.q, b->p.r, b->p.flat_tol, b->stream);
  });
  if (e != hipSuccess) return fail(SP_EHIP, "adjoint reduction launch: %s", hipGetErrorString(e));
  return SP_OK;
}

int sp_batch_destroy(sp_batch* b) {
  g_err.clear();
  batch_free(b);
  return SP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- minimum cut
struct sp_cut {
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  CutIO io{};   // buffers and the frame size
  Profiler prof;
};

extern "C" {

int sp_cut_create(int32_t H, int32_t W, void* hip_stream, sp_cut** out) {
  g_err.clear();
  if (!out) return fail(SP_EINVAL, "out is NULL");
  *out = nullptr;
  if (H < 1 || W < 1 || (long long)H * W > (1LL << 28)) return fail(SP_ESHAPE, "frame %dx%d out of range", H, W);
  sp_cut* c = new (std::nothrow) sp_cut();
  if (!c) return fail(SP_ENOMEM, "host allocation failed");
  c->stream = (hipStream_t)hip_stream;
  const size_t n = (size_t)H * W;
  size_t bytes = 0;
  for (int pass = 0; pass < 2; ++pass) {
    Bump b;
    b.base = c->arena;
    c->io.r = b.take<int32_t>(8 * n);
    c->io.e = b.take<int32_t>(n);
    c->io.h = b.take<int32_t>(n);
    c->io.rt = b.take<int32_t>(n);
    c->io.flow = b.take<unsigned long long>(2);
    c->io.flags = b.take<int32_t>(2);
    if (pass == 0) {
      bytes = b.off + 256;
      if (hipMalloc(&c->arena, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return fail(SP_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
      }
    }
  }
  c->io.H = H;
  c->io.W = W;
  *out = c;
  return SP_OK;
}

int sp_cut_destroy(sp_cut* c) {
  g_err.clear();
  if (!c) return SP_OK;
  (void)hipStreamSynchronize(c->stream);
  c->prof.destroy();
  if (c->arena) (void)hipFree(c->arena);
  delete c;
  return SP_OK;
}

int sp_mincut(sp_cut* c, const float* unary, const float* pairwise, float scale, uint8_t* labels, int64_t* flow_out) {
  g_err.clear();
  if (!c || !unary || !pairwise || !labels) return fail(SP_EINVAL, "cut, unary, pairwise and labels must not be NULL");
  if (!std::isfinite(scale) || !(scale > 0.f)) return fail(SP_EINVAL, "scale must be finite and > 0");
  CutIO io = c->io;
  io.unary = unary;
  io.pairwise = pairwise;
  io.labels = labels;
  io.flow_out = flow_out;
  io.scale = scale;
  io.cycles = 64;
  const long long tiles = (long long)((io.H + SP_CUT_T - 1) / SP_CUT_T) * ((io.W + SP_CUT_T - 1) / SP_CUT_T);
  const long long max_pass = std::max(64LL, 4 * tiles + (long long)io.H + io.W);
  auto launch = [&](int phase, int kind) -> int {
    const hipError_t e = c->prof.timed(c->stream, kind, [&] { return sp_launch_cut(phase, io, c->stream); });
    if (e != hipSuccess) return fail(SP_EHIP, "minimum cut launch (phase %d): %s", phase, hipGetErrorString(e));
    return SP_OK;
  };
  int rc = launch(0, JOB_CUT_INIT);
  if (rc) return rc;
  bool done = false;
  for (int round = 0; round < 65536 && !done; ++round) {
    // global relabel: exact distances to the sink, then the pixels with excess that reach it
    io.reset = 1;
    if ((rc = launch(1, JOB_CUT_RELABEL))) return rc;
    io.reset = 0;
    int32_t fl[2] = {1, 0};
    long long pass = 0;
    while (fl[0] != 0) {
      if (++pass > max_pass) return fail(SP_ESTATE, "minimum cut: relabelling did not settle");
      if ((rc = launch(1, JOB_CUT_RELABEL))) return rc;
      HIPCHK(hipMemcpyAsync(fl, io.flags, sizeof fl, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    }
    if (fl[1] == 0) {
      done = true;
      break;
    }
    for (int k = 0; k < 4; ++k)
      if ((rc = launch(2, JOB_CUT_PUSH))) return rc;
  }
  if (!done) return fail(SP_ESTATE, "minimum cut did not converge in 65536 rounds");
  return launch(3, JOB_CUT_INIT);
}

}  // extern "C"
