// Internal data structures shared by the HIP kernels and the host runtime.
//
// Every kernel consumes a table of jobs (one workgroup per job).  A job names the
// stream it belongs to and a rectangular tile of some map, so one launch can serve
// one stream (the plain per-frame calls) or many streams of uneven size (the
// batched step) with the same code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SP_MAXL 13          // pyramid levels 0..12
#define SP_MAXP 16          // centre-surround pairs
#define SP_MAXR 8           // largest Gabor radius
#define SP_NCH 8            // channels: I, RG, BY, O0, O45, O90, O135, M
#define SP_BLOCK 256        // threads per workgroup of every tiled kernel (4 wave64)
#define SP_KAL_ROWS 40      // rows of a prior-update tile (its width is tuned: 16, 32 or 64)
#define SP_RGB_TR 32        // most rows of a colour-statistics tile (four wavefront bands)
#define SP_RGB_TC 256       // most columns of a colour-statistics tile (4 pixels per lane)
#define SP_NOALLOC_BYTES (64u << 20)   // device scratch of the allocation-free saliency entry point
#define SP_NOALLOC_DEVICES 64          // devices whose scratch address is remembered
#define SP_DT_T 32          // tile edge of the distance-transform prediction
#define SP_DT_RMAX 54       // its largest search radius (decay length 4 pixels)

// Base channels are stored per level as [4][H_l][W_l] in the order I, RG, BY, M;
// orientation maps per used level as [4][H_l][W_l] in the order O0, O45, O90, O135.
enum { BASE_I = 0, BASE_RG = 1, BASE_BY = 2, BASE_M = 3 };

enum JobKind : int32_t {
  JOB_RGB = 0,      // colour max (+ colour-difference sums) partials over a tile of pixels
  JOB_FEAT,         // level-0 features -> level 1 (blur + decimate)
  JOB_DOWN,         // level a -> level a+1 for the 4 base channels
  JOB_GABOR,        // 4 orientation maps of level a
  JOB_CSSTATS,      // centre-surround maps of centre level a: min/max/block-max partials
  JOB_CSAPPLY,      // channel a: across-scale sum at c_max (+ its partials)
  JOB_CONSP,        // conspicuity, saliency, max/argmax partials at c_max
  JOB_SMAX,         // max/argmax partials of a given saliency map
  JOB_KALMAN,       // observation + Kalman update at level 0
  JOB_MRF,          // unary + pairwise capacities at level 0
  JOB_BWD_NU,       // adjoint sweep at level 0
  JOB_BWD_GS,       // upsample transpose at c_max
  JOB_CONSP_DOT,    // recomputed conspicuity dotted with the saliency adjoint
  JOB_LOSS,         // masked MSE partials
  JOB_TAIL,         // one channel: every level above a small source level, in LDS
  JOB_TAILGAB,      // Gabor maps of one level above the tail source (intensity chain in LDS)
  JOB_CSFINAL,      // pair a: N(.) parameters of its 8 centre-surround maps from the partials
  JOB_CSG,          // channels a..: centre-surround maps of a c_max tile, their partials and
                    // their reduction to c_max (pairs with c_max - c <= 1)
  JOB_CSMIX,        // c_max tile: F-bar as the sum of the normalised reduced maps (+ partials)
  JOB_BWD_FINAL,    // reduction of the adjoint partials (timing id only)
  JOB_DT,           // level-0 tile: prediction f from the distance to the previous object
  JOB_MANUAL,       // prior of the first frame from manual labels (timing id only)
  JOB_GMM_ACC,      // colour likelihood: prior-weighted moments of a pixel tile (timing id only)
  JOB_GMM_FIT,      // colour likelihood: mixture parameters from the moments (timing id only)
  JOB_GMM_PSI,      // colour likelihood: -log p(C | A) added to the unary costs (timing id only)
  JOB_CUT_INIT,     // minimum cut: integer capacities and the saturated t-link flow (timing id only)
  JOB_CUT_RELABEL,  // minimum cut: distances to the sink in the residual graph (timing id only)
  JOB_CUT_PUSH,     // minimum cut: push / relabel cycles (timing id only)
  JOB_PIX_ADJ,      // pixel-level adjoint of one frame (timing id only)
  JOB_NKINDS
};

// Capacities of the LDS buffers of the tail job (floats).  The levels alternate between
// the first two buffers; the four vertical Gabor passes of a level take the buffer of the
// level below it, no longer needed once the level is built.
#define SP_TAIL_SRC 8192   // source level and every second level above it
#define SP_TAIL_ALT 4096   // the other levels above it
#define SP_TAIL_HB 4096    // horizontal intermediate

struct Job {
  int32_t stream;   // index into the stream table
  int32_t a;        // kind-specific: level, channel or row band
  int32_t y0, x0;   // tile origin (in the map the kind works on)
  int32_t th, tw;   // tile size
  int32_t tid;      // index of this tile among the tiles of its map (partials slot)
  int32_t kind;     // JobKind (kernels that serve several kinds switch on it)
};

// Static description of one stream: geometry, scratch pointers, parameters.
struct StreamDesc {
  int32_t H, W, top, c_min, c_max, n_pairs, border, n_rgb;
  int32_t pc[SP_MAXP], ps[SP_MAXP];
  int32_t Hl[SP_MAXL], Wl[SP_MAXL];
  int32_t ntiles_lvl[SP_MAXL];   // number of CS tiles of a map at level l
  int32_t cs_off[SP_MAXP];       // offset (in partial triples) of pair p: [8][cs_nt[p]]
  int32_t cs_nt[SP_MAXP];        // partial triples per map of pair p
  int32_t gpath;                 // 1: every pair has c_max - c <= 1 (reduced-map path)
  int32_t rgb_tr;                // rows of a colour-statistics tile
  int32_t n_cmax_tiles;          // tiles of the c_max grid (fbar / consp / smax partials)
  int32_t gr;                    // Gabor radius
  uint32_t used;                 // bit l: level l is a centre or a surround level
  float* base[SP_MAXL];          // [4][H_l][W_l] per level (levels 1..top)
  float* gab[SP_MAXL];           // [4][H_l][W_l] per used level
  uint32_t* rgb_max_part;        // [n_rgb]
  unsigned long long* rgb_d2_part;  // [n_rgb]
  float* cs_part;                // triples (min, max, sum of block maxima)
  float* fbar;                   // [8][Hc][Wc]
  float* fbar_part;              // [8][n_cmax_tiles] triples
  float* s_part;                 // [n_cmax_tiles] pairs (max, index as float bits)
  float* cs_np;                  // [n_pairs][8][4] N(.) parameters of the centre-surround maps
  float* gmap;                   // [n_pairs][8][Hc][Wc] maps reduced to c_max (reduced-map path)
  float w[SP_NCH];
  float eps, flat_tol, lam, potts;
  float c45;                     // DC weight of the diagonal Gabor kernels
  int32_t dt_r;                  // distance-transform prediction: search radius (pixels)
  float dt_k;                    // its exponent factor, -log2(e) / (2 sigma^2)
  float gf[4][2 * SP_MAXR + 1];  // 1-D Gabor factors: g, g*(cos - c0), g*cos(a u), g*sin(a u)
};

// Per-step, per-stream inputs and outputs.
struct StepIO {
  const uint8_t* rgb;        // [H][W][3] frame t
  const uint8_t* rgb_prev;   // frame t-1 (null: t = 0, motion is zero)
  float* S_out;              // [Hc][Wc]
  float* C_out;              // [8][Hc][Wc] or null
  float* ckpt;               // base channels of level c_min: overrides base[c_min] when set
  float* S_tape;             // copy of S for the adjoint (or null)
  const float* S_in;         // saliency map read by the prior update
  const uint8_t* seg_prev;   // previous segmentation (null: use the previous prior)
  const float* pi_prev;      // [H][W] prior of step t-1 (unused at t = 0)
  float* pi_next;            // [H][W] prior of step t (Kalman state)
  float* prior_out;          // [H][W] extra copy for the caller (or null)
  float* f_tape;             // [H][W] prediction f_t (or null)
  float* ms_tape;            // [2]: max S and its first argmax (or null)
  float* unary;              // [2][H][W]
  float* pairwise;           // [4][H][W]
  float* beta_out;           // [1] or null
  // conspicuity recomputed for the adjoint (one recorded frame per stream of the launch)
  const float* gs;           // [Hc][Wc] adjoint of S of the frame
  float* dot;                // [n_cmax_tiles][8] partial sums of gs * C_k
  float* cx;                 // [8] C_k at the frame's argmax of S (ms_tape: its max and argmax)
  // variants of the prior
  float* f_map;              // [H][W] prediction f from the distance transform (null: blur)
  const float* ssm_prev;     // [Hc][Wc] stochastic saliency means of step t-1 (null: first step)
  float* ssm_next;           // [Hc][Wc] means of this step (null: no stochastic map)
  float Ks;                  // gain of the stochastic map at this step
  float K;                   // Kalman gain of this step
  int32_t t;                 // step index
};

// Arguments of the adjoint sweep (one frame at a time).
struct BwdIO {
  const float* grad;         // [H][W] dL/dpi_t
  const float* nu_next;      // [H][W] masked adjoint of step t+1 (null: none)
  float* nu_out;             // [H][W]
  float* gu;                 // [H][W] adjoint of the unclamped observation
  float* gs;                 // [Hc][Wc] adjoint of S_t (before the 1/m and argmax terms)
  float* gk_part;            // per level-0 tile partial of sum nu (q - f)
  const float* f;            // [H][W] f_t (null at t = 0)
  const float* S;            // [Hc][Wc] S_t
  const float* ms;           // [2] m_t, argmax
  float K;                   // K_t (1 at t = 0)
  float carry;               // 1 - K_{t+1} (0 when no step reads pi_t)
  int32_t t, pad;
};

// Device-resident per-stream state of the batched step.
struct BatchState {
  long long t;               // steps done since the reset
  double P;                  // Kalman variance after the last step
  float* pi[2];              // prior ping-pong
  float* S;                  // saliency map scratch [Hc][Wc]
  float* unary;              // [2][H][W] or null
  float* pairwise;           // [4][H][W] or null
  float* beta;               // [1] or null
  float* C;                  // [8][Hc][Wc] conspicuity maps or null
  const uint8_t* last_rgb;   // frame of the last step (next step's previous frame)
  int32_t cur;
  int32_t tape_cap;          // frames the tape holds (0: no tape); steps >= tape_cap record nothing
  float* tape_ckpt;          // [tape_cap][4][H_cmin][W_cmin] base channels of level c_min
  float* tape_S;             // [tape_cap][Hc][Wc]
  float* tape_f;             // [tape_cap][H][W] prediction f_t
  float* tape_ms;            // [tape_cap][2] max S and its first argmax
  float* tape_pi;            // [tape_cap][H][W] prior of every step
};

// Adjoint reduction of one stream: per-frame partials -> gradients of (w, Q, R).
struct BwdFin {
  const float* gk_part;      // [T][n_lvl0_tiles] partials of sum nu (q - f)
  const float* dot_part;     // [T][n_cmax_tiles][8] partials of sum gs * C_k
  const float* cx;           // [T][8] C_k at the argmax
  const float* ms;           // [T][2] max S and argmax
  const float* w;            // [8] channel weights
  double* gK;                // scratch: [T] dL/dK_t, then [T][8] each step's share of dL/dw
  float* grad_w;             // [8]
  float* grad_q;             // [1]
  float* grad_r;             // [1]
  int32_t n_lvl0_tiles, n_cmax_tiles;
};

// Masked-MSE loss of one stream's clip of priors.
struct LossIO {
  const float* prior;        // [T][H][W]
  const uint8_t* mask;       // [T][H][W] in {0, 1}
  float* grad;               // [T][H][W] dL/dprior (or null)
  float* part;               // [nblk] partial sums
  float* loss;               // [1]
  unsigned long long n;      // T * H * W
};

// Arguments that make the colour-statistics launch also start a batched step: its
// workgroup 0 does every stream's step bookkeeping, and every workgroup reads its frame
// from in_ptrs (in_ptrs null: an ordinary launch).
struct BatchBegin {
  const uint8_t* const* in_ptrs;   // [n] device pointers to this step's frames
  BatchState* st;
  StepIO* ios;
  int32_t n, pad;
  double Q, R;
};

// LDS layout (in floats) of the across-scale-sum job: centre values of the c_max tile
// and of the regions one and two levels finer, the reduction temporary, and one
// surround footprint per pair.  Shared by the kernel and the host (which sizes the
// dynamic LDS of the launch with it).
#define SP_CA_T 16
struct CaLayout {
  int x0, x1, x2, tm, foot0, total;   // foot0: first footprint; pair p follows pairs < p
};

// Footprint capacity (floats) of pair (c, s) for the region of centre level c.
__host__ __device__ inline int csapply_foot_cap(int r, int d) {
  const int n1 = 2 * SP_CA_T + 3, n2 = 2 * n1 + 3;
  const int n = (r == 0) ? SP_CA_T : ((r == 1) ? n1 : n2);
  const int e = ((n - 1) >> d) + 3;
  return e * e;
}

__host__ __device__ inline CaLayout csapply_layout(const int32_t* pc, const int32_t* ps, int n_pairs, int c_max) {
  bool has[3] = {false, false, false};
  for (int p = 0; p < n_pairs; ++p) has[c_max - pc[p]] = true;
  const int n1 = 2 * SP_CA_T + 3, n2 = 2 * n1 + 3;
  CaLayout L;
  int o = 0;
  L.x0 = o;
  if (has[0]) o += SP_CA_T * SP_CA_T;
  L.x1 = o;
  if (has[1] || has[2]) o += n1 * n1;
  L.x2 = o;
  if (has[2]) o += n2 * n2;
  L.tm = o;
  o += has[2] ? n2 * n1 : ((has[1]) ? n1 * SP_CA_T : 0);
  L.foot0 = o;
  for (int p = 0; p < n_pairs; ++p) o += csapply_foot_cap(c_max - pc[p], ps[p] - pc[p]);
  L.total = o;
  return L;
}

// LDS of the reduced-map job for a group of NC channels, in floats per channel:
// x1n, the centre region of the level below c_max in whole 16-byte quads per row
// (CG_X1N each, at a compile-time stride so per-channel offsets fold into the LDS
// instructions); x0n, the c_max tile (its tiles start at multiples of 16 columns, so
// SP_CA_T quads per row); footn, one surround footprint per pair (pair p's block holds
// the NC channels at a stride of its cap); then, channel-interleaved (element e of
// channel j at e * NC + j), fqn for one pair's centre-surround map on the region and
// ttn for a table holding first that pair's footprint rows interpolated at the
// region's columns, then the row pass of the reduction.  The blocks follow each other
// in this order, each NC * size floats long.
#define CG_N1 (2 * SP_CA_T + 3)
#define CG_PW1 ((CG_N1 + 6) & ~3)   // widest row of whole 16-byte quads covering CG_N1 columns
#define CG_X1N (CG_N1 * CG_PW1)
struct CgLayout {
  int x1n, x0n, footn, fqn, ttn, total;
};

// From each pair's level offsets r = c_max - c and d = s - c.
__host__ __device__ inline CgLayout csg_layout_rd(const int* rs, const int* ds, int n_pairs) {
  bool has0 = false, has1 = false;
  for (int p = 0; p < n_pairs; ++p) {
    has0 |= rs[p] == 0;
    has1 |= rs[p] == 1;
  }
  const int n1 = CG_N1;
  CgLayout L;
  L.x1n = has1 ? CG_X1N : 0;
  L.x0n = has0 ? SP_CA_T * SP_CA_T : 0;
  int f = 0, tt = has1 ? n1 * SP_CA_T : 0;
  for (int p = 0; p < n_pairs; ++p) {
    const int r = rs[p], d = ds[p];
    f += csapply_foot_cap(r, d);
    if (r == 1) tt = tt > (((n1 - 1) >> d) + 3) * n1 ? tt : (((n1 - 1) >> d) + 3) * n1;
  }
  L.footn = (f + 3) & ~3;
  L.fqn = has1 ? (n1 * n1 + 3) & ~3 : 0;
  L.ttn = (tt + 3) & ~3;
  L.total = L.x1n + L.x0n + L.footn + L.fqn + L.ttn;
  return L;
}

__host__ __device__ inline CgLayout csg_layout(const int32_t* pc, const int32_t* ps, int n_pairs, int c_max) {
  int rs[SP_MAXP], ds[SP_MAXP];
  for (int p = 0; p < n_pairs; ++p) {
    rs[p] = c_max - pc[p];
    ds[p] = ps[p] - pc[p];
  }
  return csg_layout_rd(rs, ds, n_pairs);
}

// Pair sets the reduced-map kernel is compiled for, as (r, d) = (c_max - c, s - c) per
// pair in the stream's pair order; set 0 reads the pairs from the stream description.
// Set 1: centres c_max - 1 and c_max, each with surround offsets 2 and 3 (the default
// parameters' centres 1, 2 and deltas 2, 3).
#define CG_SET1_N 4
__host__ __device__ constexpr int cg_set1_r(int p) { return p < 2 ? 1 : 0; }
__host__ __device__ constexpr int cg_set1_d(int p) { return 2 + (p & 1); }

// Colour likelihood of the t-links: per label (0 background, 1 object) a mixture of up to
// SP_GMM_MAXM Gaussians over RGB in [0, 1].
#define SP_GMM_MAXM 4
#define SP_GMM_TILE 1024   // pixels of an accumulation workgroup (4 per thread)
struct GmmComp {           // E-step form of one component (FP32)
  float mu[3];             // mean, also the centre of the moments accumulated for it
  float P[6];              // precision: xx, xy, xz, yy, yz, zz
  float lnorm;             // log(alpha) - log det(Sigma) / 2 - 3 log(2 pi) / 2
  int32_t on;              // weight > 0
  int32_t pad;
};
struct GmmState {
  double alpha[2][SP_GMM_MAXM];
  double mu[2][SP_GMM_MAXM][3];
  double cov[2][SP_GMM_MAXM][6];
  GmmComp comp[2][SP_GMM_MAXM];
  int32_t label_on[2];     // the label's total weight is positive
};
struct GmmIO {
  const uint8_t* rgb;      // [n][3]
  const float* prior;      // [n] p(A = 1): the object's sample weights (1 - p: the background's)
  const GmmState* st_prev; // mixtures the launch reads (the E-step's; the M-step's centres)
  GmmState* st_next;       // mixtures a fit stores (may be st_prev: read before written)
  const double* part_in;   // [values][ntiles] FP64 moments per tile, read by a fit
  double* part_out;        // [values][ntiles] written by the moment passes
  float* unary;            // [2][n], psi added in place
  float* out;              // [2][M][10] alpha, mu, cov (xx, xy, xz, yy, yz, zz) or null
  int32_t n, ntiles;
  float reg;               // added to the covariance diagonals
  int32_t pad;
};

// Minimum cut of the MRF on the pixel grid: integer residual capacities of the 8 n-links
// of every pixel, in the direction order E, W, S, N, SE, NW, SW, NE (d ^ 1 is the reverse
// of d), the excess, the height (distance to the sink in the residual graph; SP_CUT_INF:
// the sink cannot be reached) and the residual capacity to the sink.
#define SP_CUT_INF (1 << 30)
#define SP_CUT_T 32        // tile edge of the relabel pass
#define SP_CUT_CAPMAX (1 << 24)
struct CutIO {
  const float* unary;      // [2][n] U0 (cost of the background), U1 (cost of the object)
  const float* pairwise;   // [4][n] E, S, SE, SW
  int32_t* r;              // [8][n]
  int32_t* e;              // [n]
  int32_t* h;              // [n]
  int32_t* rt;             // [n]
  uint8_t* labels;         // [n] 1 = object (source side)
  unsigned long long* flow;   // [2] flow through the t-links at the start, flow pushed into the sink
  int32_t* flags;          // [2] heights lowered by a relabel pass, pixels with excess that reach the sink
  int64_t* flow_out;       // caller's, or null
  int32_t H, W;
  float scale;
  int32_t cycles;          // push / relabel cycles per thread and launch
  int32_t reset;           // relabel pass: start from the sink's neighbours (1) or from the heights (0)
  int32_t pad;
};

// Pixel-level adjoint (dL/d frame): one map of the N(.) adjoint.
struct PaStrip {           // partial sums of one 8-row strip of an N(.) adjoint map
  double sb, sgy, sg;      // block maxima of Y, g Y, g
  int32_t jn, jx;          // first positions within the tie tolerance of the minimum and maximum
};
#define SP_PA_MMT 4096     // pixels of a min / max partial of an N(.) adjoint map
struct PaMap {
  const float* X;          // [h][w] the map N was applied to
  const float* g;          // [h][w] dL/dN before the factor gs
  float* out;              // [h][w] dL/dX (may be the storage of X: the apply pass does not read X)
  int32_t* bpos;           // [nb] first position of each 8x8 block maximum
  float* sc;               // [8] A/range, gb/range, g(min), g(max), argmin, argmax (int bits), flat, nb
  float2* mm;              // [ceil(h w / SP_PA_MMT)] (min, max) partials
  PaStrip* strip;          // [ceil(h / 8)] strip partials
  int32_t h, w;
  float gs;
  int32_t pad;
};
// A plane pair of a gather pass (pyramid-step transpose, centre-surround, up-sample transpose).
struct PaPlane {
  const float* a;          // input plane(s)
  const float* b;
  float* out;
  uint32_t* amax;          // centre-surround: the pair's scale max |X(c)|, |X(s)| (float bits), as the
                           // maximum of SP_PA_AMAX slots (workgroup b takes slot b mod SP_PA_AMAX)
  int32_t ha, wa, hb, wb;  // sizes of a and b (b: the surround level of a centre-surround pair)
  int32_t d;               // level offset of the pair
  int32_t pad;
};

// The Gabor transposes of several levels in one launch: level blockIdx.y's plane table.
#define SP_PA_AMAX 16   // atomic-maximum slots of a pair's scale (fewer workgroups per address)

struct PaGabLevels {
  const PaPlane* tab[SP_MAXL];
  int32_t n;
};
#define SP_PA_R 8          // largest Gabor radius of the adjoint's 2-D taps
#define SP_PA_SC 8         // floats of the statistics of one N(.) adjoint map
