// Host side of the Cool-chic encode-step library: configuration checks,
// state-slab layout, launch planning over a batch of images and the C ABI
// declared in include/coolchic.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <queue>
#include <utility>
#include <vector>

#include "cc_internal.h"

// Static scratch of cc_rd_eval_noalloc (one copy per device, held until the
// process ends; host code reaches it only through hipGetSymbolAddress).
static __device__ __align__(256) char scratch[CC_NOALLOC_SCRATCH_BYTES];

int cc_arm_shape_supported(int S, int F, int H1, int H2);
int cc_syn_shape_supported(int nh, int w1, int w2);
int cc_launch_arm_plain(const Launch& l, const DevDesc& h, int bwd, hipStream_t st);
int cc_launch_arm_fused(const Launch& l, const DevDesc& h, int bwd, hipStream_t st);
int cc_arm_fused_supported(const DevDesc& h);
int cc_launch_syn_fwd_plain(const Launch& l, const DevDesc& h, int final_mse, hipStream_t st);
int cc_launch_syn_bwd_plain(const Launch& l, const DevDesc& h, int src_b, hipStream_t st);
int cc_launch_res_bwd2(const Launch& l, int r, int src_b, hipStream_t st);

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail(CC_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// Causal neighbours in decoding order: the half-plane {dy < 0, or dy = 0 and
// dx < 0} sorted by (dy^2 + dx^2, dy, dx).
void causal_offsets(int s, int* dy, int* dx) {
  struct O { int y, x; };
  std::vector<O> c;
  for (int y = -8; y <= 0; ++y)
    for (int x = -8; x <= 8; ++x)
      if (y < 0 || x < 0) c.push_back({y, x});
  std::stable_sort(c.begin(), c.end(), [](const O& a, const O& b) {
    const int da = a.y * a.y + a.x * a.x, db = b.y * b.y + b.x * b.x;
    if (da != db) return da < db;
    if (a.y != b.y) return a.y < b.y;
    return a.x < b.x;
  });
  for (int m = 0; m < s; ++m) {
    dy[m] = c[m].y;
    dx[m] = c[m].x;
  }
}

struct Layout {
  DevDesc h{};          // host copy (pointers filled relative to a base)
  size_t bytes = 0;
  size_t off_desc = 0, off_img, off_theta, off_m, off_v, off_grad, off_yhat, off_dq, off_dyd,
         off_dyq, off_dc, off_df, off_U, off_dU, off_V, off_dV, off_X, off_dXa, off_dXb, off_wp, off_wp2,
         off_agt, off_sgt, off_lpb, off_lpm, off_scal, off_aft, off_abl, off_awb;
  std::vector<unsigned> arm_gtab, syn_gtab, arm_ftab;
  std::vector<int> arm_blist, arm_wbeg;
  std::vector<int> soap_tab;
  std::vector<unsigned char> nnq_group;
  size_t off_ngrp = 0, off_nkeep = 0, off_nbits = 0;
  size_t off_stab = 0, off_sm = 0, off_sv = 0, off_sp = 0, off_sq = 0;
  int syn_o[7];
};

// Workgroups of the IFCE gradient pooling: one per (child grid c, channel,
// base block of side 2^(L-1-c)).
// Producer rows of the ARM for the current form: the plain kernel's rows
// cover the ARM and IFCE parameters; the fused kernel's rows end before the
// IFCE parameters, whose gradients come from the pooling kernel's rows.
void arm_form(DevDesc& h) {
  h.arm_nwg = h.arm_fused ? h.arm_nwg_fused : h.arm_nwg_plain;
  h.prod[h.prod_arm].nrows = h.arm_nwg;
  h.prod[h.prod_arm].pcnt = (h.arm_fused && h.F > 0 && h.G > 0) ? h.p_iw[0] : h.n_arm_par;
}

int pool_blocks(const DevDesc& h) {
  int tot = 0;
  for (int c = 0; c < h.G; ++c) {
    const int B = 1 << (h.L - 1 - c);
    tot += h.F * (h.gh[c] / B) * (h.gw[c] / B);
  }
  return tot;
}

// First upsampling level run by the per-source chain kernels: the levels
// whose output grid (j - 1) has at most CC_UPS_COARSE positions (sizes fall
// with j, so these are the levels jc .. L - 1); L when there is none.
int ups_chain_first(const DevDesc& h) {
  int jc = h.L;
  while (jc > 1 && h.gh[jc - 2] * h.gw[jc - 2] <= CC_UPS_COARSE) --jc;
  return jc;
}

// Bands of the fused ARM kernel (CC_FUSED_BAND rows of one grid, grid 0's
// first) packed onto nw workgroups, longest first, each onto the least
// loaded workgroup (LPT).  A band's load is its positions plus a fixed
// per-band cost (staging, merges).  blist: bands grouped by workgroup, in
// ascending order within a workgroup; wbeg: nw + 1 offsets.  Returns the
// largest load.
constexpr long long ARM_BAND_COST = 256;
long long arm_pack(const DevDesc& h, int nw, std::vector<int>& blist, std::vector<int>& wbeg) {
  std::vector<std::pair<long long, int>> bands;   // (-load, band)
  for (int k = 0, b = 0; k < h.NG; ++k)
    for (int y = 0; y < h.gh[k]; y += CC_FUSED_BAND, ++b)
      bands.push_back({-((long long)std::min(CC_FUSED_BAND, h.gh[k] - y) * h.gw[k] + ARM_BAND_COST), b});
  std::sort(bands.begin(), bands.end());
  std::priority_queue<std::pair<long long, int>, std::vector<std::pair<long long, int>>,
                      std::greater<std::pair<long long, int>>> heap;
  for (int w = 0; w < nw; ++w) heap.push({0, w});
  std::vector<std::vector<int>> per(nw);
  long long mx = 0;
  for (const auto& b : bands) {
    auto top = heap.top();
    heap.pop();
    top.first -= b.first;
    per[top.second].push_back(b.second);
    mx = std::max(mx, top.first);
    heap.push(top);
  }
  blist.clear();
  wbeg.assign(1, 0);
  for (auto& v : per) {
    std::sort(v.begin(), v.end());
    blist.insert(blist.end(), v.begin(), v.end());
    wbeg.push_back((int)blist.size());
  }
  return mx;
}

// Default fused-ARM workgroups per image: one per band, at most
// CC_FUSED_MAXWG (larger images pack several bands per workgroup).  Fewer
// workgroups (each grid-0 band alone, the coarser bands grouped) leave
// compute units to the distortion branch while the ARM runs; they are a
// tuning choice: they lengthen the kernel, and the overlapped step gained
// from them only while the distortion branch was the longer one.
int arm_default_wgs(const DevDesc& h) { return std::min(h.arm_nwg_fused, CC_FUSED_MAXWG); }

// Tiles of the residual-layer adjoint.
int res_tiles(const DevDesc& h) { return cdiv(h.H, CC_RES_TH) * cdiv(h.W, CC_RES_TW); }

// Workgroups of the tiled upsampling adjoint at level j: one per (channel of
// T_j, 16x16 tile of grid j); none for the chain levels.
int ups_tile_wgs(const DevDesc& h, int j) {
  return j < h.ups_jc ? cdiv(h.gh[j], CC_UPS_TILE) * cdiv(h.gw[j], CC_UPS_TILE) * (h.L - j) : 0;
}

// Weight-gradient partial rows of level j: one per tiled workgroup, or one
// per source grid on the chain levels.
int ups_bwd_rows(const DevDesc& h, int j) { return j < h.ups_jc ? ups_tile_wgs(h, j) : h.L - j; }

// Workgroups of the Conv refinement at level j (forward and adjoint): one
// per (channel of T_j, CC_UPC_TH x CC_UPC_TW tile of grid j); none without
// the refinement or on the chain levels (the chain kernels include it).
int upc_wgs(const DevDesc& h, int j) {
  return h.ups_conv && j < h.ups_jc ? cdiv(h.gh[j], CC_UPC_TH) * cdiv(h.gw[j], CC_UPC_TW) * (h.L - j) : 0;
}

int check_config(const cc_config* c, int H, int W) {
  if (!c) return fail(CC_EINVAL, "config is NULL");
  if (c->L < 2 || c->L > CC_MAX_L) return fail(CC_EINVAL, "L=%d outside [2, %d]", c->L, CC_MAX_L);
  const int m = 1 << (c->L - 1);
  if (H <= 0 || W <= 0 || H % m || W % m)
    return fail(CC_EINVAL, "image %dx%d: sides must be positive multiples of 2^(L-1)=%d", H, W, m);
  if ((long long)H * W > (1ll << 26)) return fail(CC_EINVAL, "image %dx%d too large", H, W);
  if (c->n_spatial < 1 || c->n_spatial > CC_MAX_S) return fail(CC_EINVAL, "n_spatial=%d", c->n_spatial);
  if (c->n_ifce_feat < 0 || c->n_ifce_grids < 0 || c->n_ifce_grids > 3 ||
      c->n_ifce_grids > c->L - 1 || (c->n_ifce_feat == 0) != (c->n_ifce_grids == 0))
    return fail(CC_EINVAL, "IFCE F=%d grids=%d", c->n_ifce_feat, c->n_ifce_grids);
  if (!cc_arm_shape_supported(c->n_spatial, c->n_ifce_feat, c->arm_hidden[0], c->arm_hidden[1]))
    return fail(CC_EINVAL, "ARM shape s=%d F=%d hidden=%d,%d not compiled in", c->n_spatial,
                c->n_ifce_feat, c->arm_hidden[0], c->arm_hidden[1]);
  if (c->n_syn_hidden < 1 || c->n_syn_hidden > 2 ||
      !cc_syn_shape_supported(c->n_syn_hidden, c->syn_hidden[0], c->syn_hidden[1]))
    return fail(CC_EINVAL, "synthesis shape not compiled in");
  if (c->n_res < 0 || c->n_res > 4) return fail(CC_EINVAL, "n_res=%d outside [0, 4]", c->n_res);
  if (c->n_ifce_feat > 0 && (1 << (c->L - 1)) > CC_POOL_BLOCK)
    return fail(CC_EINVAL, "IFCE needs L <= 7 (L=%d)", c->L);
  if (c->n_hyper < 0 || c->n_hyper > 4) return fail(CC_EINVAL, "n_hyper=%d outside [0, 4]", c->n_hyper);
  if (c->n_hyper > 0 && (c->hyper_first < 1 || c->hyper_first < c->n_ifce_grids ||
                         c->hyper_first + c->n_hyper > c->L))
    return fail(CC_EINVAL, "hyperlatent grids from 1/2^%d (%d of them) need n_ifce_grids <= first and first + n <= L",
                c->hyper_first, c->n_hyper);
  if (c->L + c->n_hyper > CC_MAX_G) return fail(CC_EINVAL, "too many grids");
  if (c->ups_conv != 0 && c->ups_conv != 1) return fail(CC_EINVAL, "ups_conv=%d is not 0 or 1", c->ups_conv);
  if (c->n_ifce_grids > 0 && c->L - 1 + c->n_hyper > CC_MAX_NIN)
    return fail(CC_EINVAL, "an IFCE would have more than %d inputs", CC_MAX_NIN);
  if (!(c->logscale_min < c->logscale_max)) return fail(CC_EINVAL, "log-scale clamp");
  if (!(c->p_min > 0.0f && c->p_min < 1.0f)) return fail(CC_EINVAL, "p_min must be in (0, 1)");
  if (c->precision != CC_FP32_PLAIN && c->precision != CC_BF16_FUSED)
    return fail(CC_EINVAL, "precision=%d", c->precision);
  return CC_OK;
}

void build_layout(const cc_config* c, int H, int W, Layout& Lo) {
  DevDesc& h = Lo.h;
  memset(&h, 0, sizeof h);
  h.H = H;
  h.W = W;
  h.L = c->L;
  h.S = c->n_spatial;
  h.F = c->n_ifce_feat;
  h.G = c->n_ifce_grids;
  h.H1 = c->arm_hidden[0];
  h.H2 = c->arm_hidden[1];
  h.ctx = h.S + h.F;
  h.arm_stab = c->arm_stab ? 1 : 0;
  h.syn_stab = c->syn_stab ? 1 : 0;
  h.n_syn_hidden = c->n_syn_hidden;
  h.n_res = c->n_res;
  h.syn_w[0] = c->L;
  for (int i = 0; i < c->n_syn_hidden; ++i) h.syn_w[1 + i] = c->syn_hidden[i];
  h.syn_w[1 + c->n_syn_hidden] = 3;
  // flat latent pyramid: latent grids 0 .. L-1, then the hyperlatent grids
  h.n_hyper = c->n_hyper;
  h.hyper_first = c->n_hyper > 0 ? c->hyper_first : 0;
  h.NG = c->L + c->n_hyper;
  int off = 0;
  for (int k = 0; k < h.NG; ++k) {
    const int lev = k < c->L ? k : c->hyper_first + (k - c->L);
    h.glev[k] = lev;
    h.gh[k] = H >> lev;
    h.gw[k] = W >> lev;
    h.goff[k] = off;
    off += h.gh[k] * h.gw[k];
  }
  h.n_lat = off;
  // IFCE inputs of grid k: the coarser latent grids, then the hyperlatent
  // grids, each at its resolution shift from grid k
  for (int k = 0; k < h.G; ++k) {
    int q = 0;
    for (int j = k + 1; j < h.NG; ++j) {
      h.isrc[k][q] = j;
      h.ish[k][q] = h.glev[j] - k;
      ++q;
    }
    h.nin[k] = q;
  }
  causal_offsets(h.S, h.dy, h.dx);

  // decoder parameter offsets in the documented order
  int p = 0;
  const int aw[4] = {h.ctx, h.H1, h.H2, 2};
  for (int i = 0; i < 3; ++i) {
    h.p_aw[i] = p;
    p += aw[i + 1] * aw[i];
    h.p_ab[i] = p;
    p += aw[i + 1];
  }
  h.p_asw = h.p_asb = -1;
  if (h.arm_stab) {
    h.p_asw = p;
    p += 2 * h.ctx;
    h.p_asb = p;
    p += 2;
  }
  for (int k = 0; k < h.G; ++k) {
    h.p_iw[k] = p;
    p += h.F * h.nin[k];
    h.p_ib[k] = p;
    p += h.F;
  }
  h.n_arm_par = p;
  for (int j = 1; j < h.L; ++j) {
    h.p_ups[j] = p;
    p += 4;
  }
  h.ups_conv = c->ups_conv;
  for (int j = 1; j < h.L; ++j) {
    h.p_upc[j] = h.ups_conv ? p : -1;
    if (h.ups_conv) p += 4;
  }
  const int nsl = h.n_syn_hidden + 1;
  for (int i = 0; i < nsl; ++i) {
    h.p_sw[i] = p;
    p += h.syn_w[i + 1] * h.syn_w[i];
    h.p_sb[i] = p;
    p += h.syn_w[i + 1];
  }
  h.p_ssw = h.p_ssb = -1;
  if (h.syn_stab) {
    h.p_ssw = p;
    p += 3 * h.L;
    h.p_ssb = p;
    p += 3;
  }
  const int syn_end = p;
  for (int r = 0; r < h.n_res; ++r) {
    h.p_rw[r] = p;
    p += 81;
    h.p_rb[r] = p;
    p += 3;
  }
  h.n_par = p;
  h.n_theta = h.n_lat + h.n_par;

  h.lmin = c->logscale_min;
  h.lmax = c->logscale_max;
  h.pmin = c->p_min;
  h.bits_max = (float)(-log2((double)c->p_min));

  // producer geometry
  for (int k = 0; k < h.NG; ++k) h.arm_nchunk += cdiv(h.gh[k] * h.gw[k], CC_ARM_CHUNK);
  h.arm_nwg_plain = cdiv(h.arm_nchunk, CC_ARM_CPW);
  h.arm_nwg_fused = 0;
  for (int k = 0; k < h.NG; ++k) h.arm_nwg_fused += cdiv(h.gh[k], CC_FUSED_BAND);
  h.arm_fused = (c->precision == CC_BF16_FUSED && cc_arm_fused_supported(h)) ? 1 : 0;
  // partial rows are sized for either form; the current one is selected below
  h.arm_nwg = std::max(h.arm_nwg_plain, h.arm_nwg_fused);
  const int npix = H * W;
  h.syn_nchunk = cdiv(npix, CC_SYN_CHUNK);
  h.syn_cpw = CC_SYN_CPW;
  h.syn_nwg = cdiv(h.syn_nchunk, h.syn_cpw);
  h.pix_ntile = cdiv(npix, CC_PIX_TILE);
  h.pix_nwg = h.pix_ntile;
  h.lat_ntile = cdiv(h.n_lat, CC_ELT_TILE);
  long long wpo = 0;
  int q = 0;
  h.prod_arm = q;
  h.prod[q++] = {0, h.n_arm_par, h.arm_nwg, 0, wpo};
  wpo += (long long)std::max(h.arm_nwg_plain, h.arm_nwg_fused) * h.n_arm_par;
  // the fused form takes the IFCE weight gradients of grid c from the pooling
  // kernel: one partial row per pooling block (F (nin + 1) entries, the
  // grid's IFCE weights then biases); its ARM rows stop before them
  h.prod_ifce0 = q;
  for (int c = 0; h.F > 0 && c < h.G; ++c) {
    const int B = 1 << (h.L - 1 - c);
    const int rows = (h.gh[c] / B) * (h.gw[c] / B), cnt = h.F * (h.nin[c] + 1);
    h.prod[q++] = {h.p_iw[c], cnt, rows, 0, wpo};
    wpo += (long long)rows * cnt;
  }
  h.ups_jc = ups_chain_first(h);
  h.prod_ups1 = q;
  for (int j = 1; j < h.L; ++j) {
    const int rows = ups_bwd_rows(h, j);
    h.prod[q++] = {h.p_ups[j], 4, rows, 0, wpo};
    wpo += (long long)rows * 4;
  }
  h.prod_upc1 = q;
  for (int j = 1; h.ups_conv && j < h.L; ++j) {
    const int rows = j < h.ups_jc ? upc_wgs(h, j) : h.L - j;   // tiles, or one per source
    h.prod[q++] = {h.p_upc[j], 4, rows, 0, wpo};
    wpo += (long long)rows * 4;
  }
  h.prod_syn = q;
  // partial rows sized for the smallest tunable chunks per workgroup
  h.prod[q++] = {h.p_sw[0], syn_end - h.p_sw[0], h.syn_nwg, 0, wpo};
  wpo += (long long)cdiv(h.syn_nchunk, CC_SYN_CPW_MIN) * (syn_end - h.p_sw[0]);
  h.prod_res0 = q;
  h.res_tpw = CC_RES_TPW;
  h.res_nwg = cdiv(res_tiles(h), h.res_tpw);
  for (int r = 0; r < h.n_res; ++r) {
    // partial rows sized for one tile per workgroup
    h.prod[q++] = {h.p_rw[r], 84, h.res_nwg, 0, wpo};
    wpo += (long long)res_tiles(h) * 84;
  }
  h.nprod = q;
  arm_form(h);
  h.arm_wgs = arm_default_wgs(h);
  arm_pack(h, h.arm_wgs, Lo.arm_blist, Lo.arm_wbeg);

  // weight-gradient tables: (index into gradient vector, index into
  // activation vector, grid requirement) per parameter, matching the LDS row
  // layouts of the ARM and synthesis backward kernels.
  {
    const int CTX = h.ctx, RM = CC_MAX_NIN;
    const int O_H1 = CTX, O_H2 = O_H1 + h.H1, O_R = O_H2 + h.H2, O_DH1 = O_R + RM,
              O_DH2 = O_DH1 + h.H1, O_DO = O_DH2 + h.H2, O_DF = O_DO + 2, O_ONE = O_DF + h.F;
    auto ent = [](int a, int b, int k) {
      return (unsigned)a | ((unsigned)b << 8) | ((unsigned)(k & 0xFF) << 16);
    };
    std::vector<unsigned>& t = Lo.arm_gtab;
    t.assign(h.n_arm_par, 0xFFFFFFFFu);
    for (int a = 0; a < h.H1; ++a)
      for (int b = 0; b < CTX; ++b) t[h.p_aw[0] + a * CTX + b] = ent(O_DH1 + a, b, 0xFF);
    for (int a = 0; a < h.H1; ++a) t[h.p_ab[0] + a] = ent(O_DH1 + a, O_ONE, 0xFF);
    for (int a = 0; a < h.H2; ++a)
      for (int b = 0; b < h.H1; ++b) t[h.p_aw[1] + a * h.H1 + b] = ent(O_DH2 + a, O_H1 + b, 0xFF);
    for (int a = 0; a < h.H2; ++a) t[h.p_ab[1] + a] = ent(O_DH2 + a, O_ONE, 0xFF);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < h.H2; ++b) t[h.p_aw[2] + a * h.H2 + b] = ent(O_DO + a, O_H2 + b, 0xFF);
    for (int a = 0; a < 2; ++a) t[h.p_ab[2] + a] = ent(O_DO + a, O_ONE, 0xFF);
    if (h.arm_stab) {
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < CTX; ++b) t[h.p_asw + a * CTX + b] = ent(O_DO + a, b, 0xFF);
      for (int a = 0; a < 2; ++a) t[h.p_asb + a] = ent(O_DO + a, O_ONE, 0xFF);
    }
    for (int k = 0; k < h.G; ++k) {
      const int nin = h.nin[k];
      for (int f = 0; f < h.F; ++f)
        for (int qq = 0; qq < nin; ++qq) t[h.p_iw[k] + f * nin + qq] = ent(O_DF + f, O_R + qq, k);
      for (int f = 0; f < h.F; ++f) t[h.p_ib[k] + f] = ent(O_DF + f, O_ONE, k);
    }
  }
  {
    // fused ARM: parameter -> (grid requirement, accumulator, row, column) of
    // its weight-gradient accumulators: 0 = dH1 C^T (stabilizer rows H1,
    // H1 + 1; bias column CTX), 1 = dH2 H1^T (bias column H1), 2 = rows H1,
    // H1 + 1 (d mu, d l) against H2^T (bias column H2), 3 = the IFCE rows
    // S + f of the context gradient against the IFCE inputs (bias column
    // CC_MAX_NIN), taken only from the bands of the IFCE's own grid
    auto ent = [](int k, int a, int row, int col) {
      return ((unsigned)(k & 0xFF) << 16) | ((unsigned)a << 10) | ((unsigned)row << 5) | (unsigned)col;
    };
    const int CTX = h.ctx;
    std::vector<unsigned>& t = Lo.arm_ftab;
    t.assign(h.n_arm_par, 0xFFFFFFFFu);
    for (int u = 0; u < h.H1; ++u) {
      for (int q2 = 0; q2 < CTX; ++q2) t[h.p_aw[0] + u * CTX + q2] = ent(0xFF, 0, u, q2);
      t[h.p_ab[0] + u] = ent(0xFF, 0, u, CTX);
    }
    for (int u = 0; u < h.H2; ++u) {
      for (int q2 = 0; q2 < h.H1; ++q2) t[h.p_aw[1] + u * h.H1 + q2] = ent(0xFF, 1, u, q2);
      t[h.p_ab[1] + u] = ent(0xFF, 1, u, h.H1);
    }
    for (int a = 0; a < 2; ++a) {
      for (int q2 = 0; q2 < h.H2; ++q2) t[h.p_aw[2] + a * h.H2 + q2] = ent(0xFF, 2, h.H1 + a, q2);
      t[h.p_ab[2] + a] = ent(0xFF, 2, h.H1 + a, h.H2);
      if (h.arm_stab) {
        for (int q2 = 0; q2 < CTX; ++q2) t[h.p_asw + a * CTX + q2] = ent(0xFF, 0, h.H1 + a, q2);
        t[h.p_asb + a] = ent(0xFF, 0, h.H1 + a, CTX);
      }
    }
    for (int k = 0; k < h.G; ++k) {
      const int nin = h.nin[k];
      for (int f = 0; f < h.F; ++f) {
        for (int q2 = 0; q2 < nin; ++q2) t[h.p_iw[k] + f * nin + q2] = ent(k, 3, h.S + f, q2);
        t[h.p_ib[k] + f] = ent(k, 3, h.S + f, CC_MAX_NIN);
      }
    }
  }
  {
    const int W1 = h.syn_w[1], NH = h.n_syn_hidden, HW2 = NH == 2 ? h.syn_w[2] : 0;
    const int WL = NH == 2 ? h.syn_w[2] : W1;
    const int O_Z = 0, O_H1 = CC_MAX_L, O_H2 = O_H1 + W1, O_DH1 = O_H2 + HW2,
              O_DH2 = O_DH1 + W1, O_DO = O_DH2 + HW2, O_ONE = O_DO + 3;
    auto ent = [](int a, int b) { return (unsigned)a | ((unsigned)b << 8) | (0xFFu << 16); };
    const int base = h.p_sw[0];
    std::vector<unsigned>& t = Lo.syn_gtab;
    t.assign(syn_end - base, 0xFFFFFFFFu);
    for (int a = 0; a < W1; ++a)
      for (int b = 0; b < h.L; ++b) t[h.p_sw[0] - base + a * h.L + b] = ent(O_DH1 + a, O_Z + b);
    for (int a = 0; a < W1; ++a) t[h.p_sb[0] - base + a] = ent(O_DH1 + a, O_ONE);
    if (NH == 2) {
      for (int a = 0; a < HW2; ++a)
        for (int b = 0; b < W1; ++b) t[h.p_sw[1] - base + a * W1 + b] = ent(O_DH2 + a, O_H1 + b);
      for (int a = 0; a < HW2; ++a) t[h.p_sb[1] - base + a] = ent(O_DH2 + a, O_ONE);
    }
    const int O_HL = NH == 2 ? O_H2 : O_H1;
    for (int c3 = 0; c3 < 3; ++c3)
      for (int b = 0; b < WL; ++b) t[h.p_sw[NH] - base + c3 * WL + b] = ent(O_DO + c3, O_HL + b);
    for (int c3 = 0; c3 < 3; ++c3) t[h.p_sb[NH] - base + c3] = ent(O_DO + c3, O_ONE);
    if (h.syn_stab) {
      for (int c3 = 0; c3 < 3; ++c3)
        for (int b = 0; b < h.L; ++b) t[h.p_ssw - base + c3 * h.L + b] = ent(O_DO + c3, O_Z + b);
      for (int c3 = 0; c3 < 3; ++c3) t[h.p_ssb - base + c3] = ent(O_DO + c3, O_ONE);
    }
  }

  // SOAP table: every decoder-parameter tensor in layout order
  {
    struct TT { int poff, nd, dims[4]; };
    std::vector<TT> ts;
    const int widths[4] = {h.ctx, h.H1, h.H2, 2};
    for (int i = 0; i < 3; ++i) {
      ts.push_back({h.p_aw[i], 2, {widths[i + 1], widths[i], 1, 1}});
      ts.push_back({h.p_ab[i], 1, {widths[i + 1], 1, 1, 1}});
    }
    if (h.arm_stab) {
      ts.push_back({h.p_asw, 2, {2, h.ctx, 1, 1}});
      ts.push_back({h.p_asb, 1, {2, 1, 1, 1}});
    }
    for (int k = 0; k < h.G; ++k) {
      ts.push_back({h.p_iw[k], 2, {h.F, h.nin[k], 1, 1}});
      ts.push_back({h.p_ib[k], 1, {h.F, 1, 1, 1}});
    }
    for (int j = 1; j < h.L; ++j) ts.push_back({h.p_ups[j], 1, {4, 1, 1, 1}});
    for (int j = 1; h.ups_conv && j < h.L; ++j) ts.push_back({h.p_upc[j], 1, {4, 1, 1, 1}});
    for (int i = 0; i <= h.n_syn_hidden; ++i) {
      ts.push_back({h.p_sw[i], 2, {h.syn_w[i + 1], h.syn_w[i], 1, 1}});
      ts.push_back({h.p_sb[i], 1, {h.syn_w[i + 1], 1, 1, 1}});
    }
    if (h.syn_stab) {
      ts.push_back({h.p_ssw, 2, {3, h.L, 1, 1}});
      ts.push_back({h.p_ssb, 1, {3, 1, 1, 1}});
    }
    for (int r = 0; r < h.n_res; ++r) {
      ts.push_back({h.p_rw[r], 4, {3, 3, 3, 3}});
      ts.push_back({h.p_rb[r], 1, {3, 1, 1, 1}});
    }
    std::vector<int>& tab = Lo.soap_tab;
    tab.assign(ts.size() * CC_SOAP_TAB, 0);
    int fac = 0;
    for (size_t t = 0; t < ts.size(); ++t) {
      int* r = &tab[t * CC_SOAP_TAB];
      int numel = 1;
      for (int e = 0; e < ts[t].nd; ++e) numel *= ts[t].dims[e];
      r[0] = ts[t].poff;
      r[1] = numel;
      r[2] = ts[t].nd;
      for (int e = 0; e < 4; ++e) {
        r[3 + e] = e < ts[t].nd ? ts[t].dims[e] : 1;
        r[7 + e] = -1;
        if (ts[t].nd >= 2 && e < ts[t].nd && ts[t].dims[e] <= CC_SOAP_MAXDIM) {
          r[7 + e] = fac;
          fac += ts[t].dims[e] * ts[t].dims[e];
        }
      }
    }
    h.soap_ntens = (int)ts.size();
    h.soap_nfac = fac;
  }

  // quantisation groups of the decoder parameters: 2 * submodule + is_bias,
  // submodules 0 ARM, 1 synthesis (with the residual layers), 2 upsampling,
  // 3 IFCE
  {
    std::vector<unsigned char>& g = Lo.nnq_group;
    g.assign(h.n_par, 0);
    auto mark = [&](int beg, int cnt, int grp) {
      for (int i = 0; i < cnt; ++i) g[beg + i] = (unsigned char)grp;
    };
    const int widths[4] = {h.ctx, h.H1, h.H2, 2};
    for (int i = 0; i < 3; ++i) {
      mark(h.p_aw[i], widths[i + 1] * widths[i], 0);
      mark(h.p_ab[i], widths[i + 1], 1);
    }
    if (h.arm_stab) {
      mark(h.p_asw, 2 * h.ctx, 0);
      mark(h.p_asb, 2, 1);
    }
    for (int k = 0; k < h.G; ++k) {
      mark(h.p_iw[k], h.F * h.nin[k], 6);
      mark(h.p_ib[k], h.F, 7);
    }
    for (int j = 1; j < h.L; ++j) mark(h.p_ups[j], 4, 4);
    for (int j = 1; h.ups_conv && j < h.L; ++j) mark(h.p_upc[j], 4, 4);
    for (int i = 0; i <= h.n_syn_hidden; ++i) {
      mark(h.p_sw[i], h.syn_w[i + 1] * h.syn_w[i], 2);
      mark(h.p_sb[i], h.syn_w[i + 1], 3);
    }
    if (h.syn_stab) {
      mark(h.p_ssw, 3 * h.L, 2);
      mark(h.p_ssb, 3, 3);
    }
    for (int r = 0; r < h.n_res; ++r) {
      mark(h.p_rw[r], 81, 2);
      mark(h.p_rb[r], 3, 3);
    }
  }

  // slab layout
  size_t o = 0;
  auto take = [&](size_t n) {
    const size_t r = o;
    o = al256(o + n);
    return r;
  };
  Lo.off_desc = take(sizeof(DevDesc));
  Lo.off_img = take(sizeof(float) * 3 * (size_t)npix);
  Lo.off_theta = take(sizeof(float) * (size_t)h.n_theta);
  Lo.off_m = take(sizeof(float) * (size_t)h.n_theta);
  Lo.off_v = take(sizeof(float) * (size_t)h.n_theta);
  Lo.off_grad = take(sizeof(float) * (size_t)h.n_theta);
  Lo.off_yhat = take(sizeof(float) * (size_t)h.n_lat);
  Lo.off_dq = take(sizeof(float) * (size_t)h.n_lat);
  Lo.off_dyd = take(sizeof(float) * (size_t)h.n_lat);
  Lo.off_dyq = take(sizeof(float) * (size_t)h.n_lat);
  Lo.off_dc = take(sizeof(float) * (size_t)h.S * h.n_lat);
  size_t dfn = 0;
  for (int cg = 0; cg < h.G; ++cg)
    for (int f = 0; cg + f < h.L; ++f) {
      h.dfoff[cg][f] = (int)dfn;
      dfn += (size_t)h.F * h.gh[cg + f] * h.gw[cg + f];
    }
  Lo.off_df = take(sizeof(float) * std::max<size_t>(dfn, 1));
  size_t un = 0;
  for (int j = 1; j < h.L; ++j) {
    h.uoff[j] = (int)un;
    un += (size_t)(h.L - j) * h.gh[j - 1] * h.gw[j - 1];
  }
  Lo.off_U = take(sizeof(float) * un);
  Lo.off_dU = take(sizeof(float) * un);
  size_t vn = 0;
  for (int j = 1; j < h.L; ++j) {
    h.voff[j] = (int)vn;
    if (h.ups_conv) vn += (size_t)(h.L - j) * h.gh[j] * h.gw[j];
  }
  Lo.off_V = take(sizeof(float) * std::max<size_t>(vn, 1));
  Lo.off_dV = take(sizeof(float) * std::max<size_t>(vn, 1));
  Lo.off_X = take(sizeof(float) * (size_t)(h.n_res + 1) * 3 * npix);
  Lo.off_dXa = take(sizeof(float) * 3 * (size_t)npix);
  Lo.off_dXb = take(sizeof(float) * 3 * (size_t)npix);
  Lo.off_wp = take(sizeof(float) * (size_t)wpo);
  Lo.off_wp2 = take(sizeof(double) * (size_t)CC_WRED_SPLIT * h.n_par);
  Lo.off_agt = take(sizeof(unsigned) * (size_t)h.n_arm_par);
  Lo.off_sgt = take(sizeof(unsigned) * Lo.syn_gtab.size());
  Lo.off_lpb = take(sizeof(double) * (size_t)std::max(h.arm_nwg_plain, h.arm_nwg_fused));
  Lo.off_aft = take(sizeof(unsigned) * (size_t)h.n_arm_par);
  Lo.off_abl = take(sizeof(int) * (size_t)h.arm_nwg_fused);
  Lo.off_awb = take(sizeof(int) * (size_t)(h.arm_nwg_fused + 1));
  Lo.off_lpm = take(sizeof(double) * (size_t)h.pix_ntile);
  Lo.off_scal = take(sizeof(double) * 8);
  Lo.off_stab = take(sizeof(int) * Lo.soap_tab.size());
  Lo.off_sm = take(sizeof(float) * (size_t)h.n_par);
  Lo.off_sv = take(sizeof(float) * (size_t)h.n_par);
  Lo.off_sp = take(sizeof(float) * (size_t)h.soap_nfac);
  Lo.off_sq = take(sizeof(float) * (size_t)h.soap_nfac);
  Lo.off_ngrp = take((size_t)h.n_par);
  Lo.off_nkeep = take(sizeof(float) * (size_t)h.n_par);
  Lo.off_nbits = take(sizeof(long long) * CC_NNQ_NG * CC_NNQ_NK);
  Lo.bytes = o;
}

void set_pointers(Layout& Lo, char* base) {
  DevDesc& h = Lo.h;
  h.img = (float*)(base + Lo.off_img);
  h.theta = (float*)(base + Lo.off_theta);
  h.m = (float*)(base + Lo.off_m);
  h.v = (float*)(base + Lo.off_v);
  h.grad = (float*)(base + Lo.off_grad);
  h.yhat = (float*)(base + Lo.off_yhat);
  h.dq = (float*)(base + Lo.off_dq);
  h.dyd = (float*)(base + Lo.off_dyd);
  h.dyq = (float*)(base + Lo.off_dyq);
  h.dc = (float*)(base + Lo.off_dc);
  h.df = (float*)(base + Lo.off_df);
  h.U = (float*)(base + Lo.off_U);
  h.dU = (float*)(base + Lo.off_dU);
  h.V = (float*)(base + Lo.off_V);
  h.dV = (float*)(base + Lo.off_dV);
  h.X = (float*)(base + Lo.off_X);
  h.dXa = (float*)(base + Lo.off_dXa);
  h.dXb = (float*)(base + Lo.off_dXb);
  h.wp = (float*)(base + Lo.off_wp);
  h.wp2 = (double*)(base + Lo.off_wp2);
  h.arm_gtab = (unsigned*)(base + Lo.off_agt);
  h.arm_ftab = (unsigned*)(base + Lo.off_aft);
  h.arm_blist = (int*)(base + Lo.off_abl);
  h.arm_wbeg = (int*)(base + Lo.off_awb);
  h.syn_gtab = (unsigned*)(base + Lo.off_sgt);
  h.lp_bits = (double*)(base + Lo.off_lpb);
  h.lp_mse = (double*)(base + Lo.off_lpm);
  h.scal = (double*)(base + Lo.off_scal);
  h.soap_tab = (int*)(base + Lo.off_stab);
  h.soap_m = (float*)(base + Lo.off_sm);
  h.soap_v = (float*)(base + Lo.off_sv);
  h.soap_p = (float*)(base + Lo.off_sp);
  h.soap_q = (float*)(base + Lo.off_sq);
  h.nnq_group = (unsigned char*)(base + Lo.off_ngrp);
  h.nnq_keep = (float*)(base + Lo.off_nkeep);
  h.nnq_bits = (long long*)(base + Lo.off_nbits);
}

// Seeded default decoder parameters (splitmix64 uniforms).
struct SplitMix {
  uint64_t s;
  double next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  }
};

void default_params(const DevDesc& h, uint64_t seed, std::vector<float>& P) {
  P.assign(h.n_par, 0.0f);
  SplitMix g{seed ^ 0x5EEDC0DEull};
  auto fill = [&](int off, int n, int fan_in) {
    const double b = 1.0 / sqrt((double)fan_in);
    for (int i = 0; i < n; ++i) P[off + i] = (float)((2.0 * g.next() - 1.0) * b);
  };
  fill(h.p_aw[0], h.H1 * h.ctx + h.H1, h.ctx);
  fill(h.p_aw[1], h.H2 * h.H1 + h.H2, h.H1);
  for (int k = 0; k < h.G; ++k) fill(h.p_iw[k], h.F * h.nin[k] + h.F, h.nin[k]);
  const float bic[4] = {-0.03515625f, -0.10546875f, 0.26171875f, 0.87890625f};
  for (int j = 1; j < h.L; ++j)
    for (int t = 0; t < 4; ++t) P[h.p_ups[j] + t] = bic[t];
  for (int j = 1; h.ups_conv && j < h.L; ++j) P[h.p_upc[j]] = 1.0f;   // identity Conv
  for (int i = 0; i <= h.n_syn_hidden; ++i)
    fill(h.p_sw[i], h.syn_w[i + 1] * h.syn_w[i] + h.syn_w[i + 1], h.syn_w[i]);
  if (h.syn_stab) fill(h.p_ssw, 3 * h.L + 3, h.L);
  for (int r = 0; r < h.n_res; ++r) fill(h.p_rw[r], 84, 27);
}

}  // namespace

struct cc_state {
  cc_config cfg;
  Layout lo;
  DevDesc* ddev;   // device copy
  char* base;
  int precision;
  int nonfinite;
  int64_t t;
  int device;
  int optimizer = CC_OPT_ADAM;   // for the decoder parameters
  int soap_calls = 0;            // SOAP calls made (0: the next one initialises)
};

namespace {

// ------------------------------------------------------- launch planning --
template <class F>
Launch plan(cc_state* const* s, int n, F count) {
  Launch l;
  memset(&l, 0, sizeof l);
  l.n = n;
  int acc = 0;
  for (int i = 0; i < n; ++i) {
    l.tile0[i] = acc;
    l.d[i] = s[i]->ddev;
    acc += count(s[i]->lo.h);
  }
  l.tile0[n] = acc;
  return l;
}

bool same_shape(const cc_state* a, const cc_state* b) {
  const DevDesc &x = a->lo.h, &y = b->lo.h;
  return x.L == y.L && x.NG == y.NG && x.hyper_first == y.hyper_first && x.ups_conv == y.ups_conv && x.S == y.S && x.F == y.F && x.G == y.G && x.H1 == y.H1 && x.H2 == y.H2 &&
         x.n_syn_hidden == y.n_syn_hidden && x.syn_w[1] == y.syn_w[1] &&
         x.syn_w[2] == y.syn_w[2] && x.n_res == y.n_res && a->precision == b->precision;
}

StepArgs step_args(const cc_step_params& p) {
  StepArgs a{};
  const double T = p.temperature > 0.0f ? (double)p.temperature : 1.0;
  a.T = (float)T;
  a.sr_c = (float)(1.0 / (2.0 * tanh(1.0 / (2.0 * T))));
  a.sr_invT = (float)(1.0 / T);
  a.sigma = p.sigma;
  a.lr = p.lr;
  const double tt = (double)(p.t < 1 ? 1 : p.t);
  a.bc1 = (float)(1.0 - pow(0.9, tt));
  a.bc2 = (float)(1.0 - pow(0.999, tt));
  a.t_lo = (unsigned)(p.t & 0xFFFFFFFFll);
  a.mode = p.quant_mode;
  a.upd = p.update_latents;
  return a;
}

int check_params(const cc_step_params* p) {
  if (!p) return fail(CC_EINVAL, "step params are NULL");
  if (p->quant_mode != CC_SOFT && p->quant_mode != CC_HARD) return fail(CC_EINVAL, "quant_mode");
  if (p->quant_mode == CC_SOFT && !(p->temperature > 0.0f))
    return fail(CC_EINVAL, "temperature must be > 0");
  if (!(p->sigma >= 0.0f) || !(p->lr >= 0.0f) || p->t < 1)
    return fail(CC_EINVAL, "sigma, lr must be >= 0 and t >= 1");
  return CC_OK;
}

#define RET(x)                    \
  do {                            \
    int r_ = (x);                 \
    if (r_ != CC_OK) return r_ == CC_EDEVICE ? fail(CC_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError())) : r_; \
  } while (0)

// Quantisation proxy (a1) for a set of states; the kernel also stores the
// step's schedule values in each descriptor for the rest of the step.
int quantise(cc_state* const* s, int n, const cc_step_params* p, hipStream_t st) {
  StepPack a;
  memset(&a, 0, sizeof a);
  for (int i = 0; i < n; ++i) a.a[i] = step_args(p[i]);
  return cc_launch_qtrain(plan(s, n, [](const DevDesc& h) { return h.lat_ntile; }), a, st);
}

// Optional live timing of one kernel class with HIP events recorded on the
// launch stream around each of its launches (see cc_timing_enable).
enum { TK_NONE = 0, TK_ARM = 1, TK_SYN_BWD = 2, TK_RES_BWD = 3, TK_UPS_BWD = 4, TK_JOIN = 5, TK_UPS_FWD = 6, TK_POOL = 7, TK_DIST_FWD = 8 };
struct Timing {
  int kind = TK_NONE;
  int every = 1;                // time one launch in `every`
  long long seen = 0;           // launches of the kind since enabling
  std::vector<hipEvent_t> ev;   // pairs (start, stop)
  size_t used = 0;
};
Timing g_timing;

struct TimeScope {
  hipStream_t st;
  bool on;
  hipEvent_t e1 = nullptr;
  TimeScope(int kind, hipStream_t s) : st(s), on(g_timing.kind == kind) {
    if (!on) return;
    on = g_timing.seen++ % g_timing.every == 0;
    if (!on) return;
    if (g_timing.used + 2 > g_timing.ev.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
          on = false;
          return;
        }
        g_timing.ev.push_back(e);
      }
    }
    (void)hipEventRecord(g_timing.ev[g_timing.used], st);
    e1 = g_timing.ev[g_timing.used + 1];
    g_timing.used += 2;
  }
  ~TimeScope() {
    if (on) (void)hipEventRecord(e1, st);
  }
};

// Second stream per device for the rate branch of a step (ARM and IFCE
// gradient pooling), which depends on the distortion branch (upsampling,
// synthesis, residual layers, their backward) only through the latent
// gradient join: the two branches run concurrently, the rate branch on this
// stream, forked from and joined back into the caller's stream with events.
// The stream is non-blocking so that the fork also overlaps when the caller
// uses the legacy default stream.  Calls on one device take the device's lock
// for their launches, so concurrent callers never interleave their event
// pairs.
struct Side {
  std::mutex mu;
  bool tried = false;
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMaxSideDev = 64;
Side g_side[kMaxSideDev];
std::atomic<bool> g_overlap{true};

// The device's side stream (created on first use with the device current),
// or nullptr to run both branches on the caller's stream.  Caller holds mu.
Side* side_stream(int dev) {
  Side& sd = g_side[dev];
  if (!sd.tried) {
    sd.tried = true;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != dev) {
      sd.tried = false;
      return nullptr;
    }
    if (hipStreamCreateWithFlags(&sd.st, hipStreamNonBlocking) != hipSuccess) sd.st = nullptr;
    if (sd.st && (hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming) != hipSuccess ||
                  hipEventCreateWithFlags(&sd.join, hipEventDisableTiming) != hipSuccess)) {
      (void)hipStreamDestroy(sd.st);
      sd.st = nullptr;
    }
    // a failed creation leaves HIP's last error set; clear it so that the
    // next launch check does not report it (the step then runs unforked)
    if (!sd.st) (void)hipGetLastError();
  }
  return sd.st ? &sd : nullptr;
}

// Fork of the rate branch; the destructor joins it back into the caller's
// stream if join() was not reached (an error return in between), so the
// caller's stream never runs ahead of work still queued on the side stream.
struct Fork {
  std::unique_lock<std::mutex> lk;
  Side* sd = nullptr;
  hipStream_t main;
  bool joined = false;
  Fork(int dev, hipStream_t st) : main(st) {
    if (!g_overlap || dev < 0 || dev >= kMaxSideDev) return;
    lk = std::unique_lock<std::mutex>(g_side[dev].mu);
    sd = side_stream(dev);
  }
  // stream for the rate branch, ordered after everything queued on main
  hipStream_t begin() {
    if (!sd) return main;
    if (hipEventRecord(sd->fork, main) != hipSuccess ||
        hipStreamWaitEvent(sd->st, sd->fork, 0) != hipSuccess) {
      sd = nullptr;
      return main;
    }
    return sd->st;
  }
  int join() {
    if (!sd || joined) return CC_OK;
    joined = true;
    HIPCHK(hipEventRecord(sd->join, sd->st));
    HIPCHK(hipStreamWaitEvent(main, sd->join, 0));
    return CC_OK;
  }
  ~Fork() { (void)join(); }
};

int arm(cc_state* const* s, int n, int bwd, hipStream_t st) {
  // the fused kernel's workgroups loop over the bands (at most one workgroup
  // per compute unit for one image, leaving room on each unit for the
  // distortion branch running beside it); the plain kernel has one per chunk
  const Launch l = plan(s, n, [](const DevDesc& h) {
    return h.arm_fused ? h.arm_wgs : h.arm_nwg;
  });
  TimeScope ts(bwd ? TK_ARM : TK_NONE, st);
  if (s[0]->lo.h.arm_fused) return cc_launch_arm_fused(l, s[0]->lo.h, bwd, st);
  return cc_launch_arm_plain(l, s[0]->lo.h, bwd, st);
}

// Forward of the distortion branch: upsampling, synthesis, residual layers
// (+ MSE when want_mse).
// Upsampling forward (a5): the chain levels first (coarsest), then the tiled
// levels from coarse to fine.
int ups_forward(cc_state* const* s, int n, hipStream_t st) {
  const Launch lc = plan(s, n, [](const DevDesc& h) { return h.L - h.ups_jc; });
  if (lc.tile0[n] > 0) RET(cc_launch_ups_fwd_chain(lc, st));
  for (int j = s[0]->lo.h.L - 1; j >= 1; --j) {
    // Conv refinement: V_j = Conv_j(T_j), the transposed convolution's input
    const Launch lv = plan(s, n, [j](const DevDesc& h) { return upc_wgs(h, j); });
    if (lv.tile0[n] > 0) RET(cc_launch_upc_fwd(lv, j, st));
    const Launch l = plan(s, n, [j](const DevDesc& h) {
      return j < h.ups_jc ? cdiv(h.gh[j - 1] * h.gw[j - 1], CC_PIX_TILE) : 0;
    });
    if (l.tile0[n] > 0) RET(cc_launch_ups_fwd(l, j, st));
  }
  return CC_OK;
}

// Upsampling backward (a9): the tiled levels from fine to coarse, then the
// chain levels.
int ups_backward(cc_state* const* s, int n, hipStream_t st) {
  for (int j = 1; j < s[0]->lo.h.L; ++j) {
    const Launch l = plan(s, n, [j](const DevDesc& h) { return ups_tile_wgs(h, j); });
    if (l.tile0[n] > 0) RET(cc_launch_ups_bwd(l, j, st));
    const Launch lv = plan(s, n, [j](const DevDesc& h) { return upc_wgs(h, j); });
    if (lv.tile0[n] > 0) RET(cc_launch_upc_bwd(lv, j, st));
  }
  const Launch lc = plan(s, n, [](const DevDesc& h) { return h.L - h.ups_jc; });
  if (lc.tile0[n] > 0) RET(cc_launch_ups_bwd_chain(lc, st));
  return CC_OK;
}

// Synthesis and residual layers of the distortion branch (+ MSE when
// want_mse), after the upsampling.
int forward_syn(cc_state* const* s, int n, int want_mse, hipStream_t st) {
  const DevDesc& h0 = s[0]->lo.h;
  const Launch lp = plan(s, n, [](const DevDesc& h) { return h.pix_ntile; });
  RET(cc_launch_syn_fwd_plain(lp, h0, (h0.n_res == 0 && want_mse) ? 1 : 0, st));
  for (int r = 0; r < h0.n_res; ++r) RET(cc_launch_res_fwd(lp, r, r == h0.n_res - 1, want_mse, st));
  return CC_OK;
}

int run_step(cc_state* const* s, int n, const cc_step_params* p, hipStream_t st, bool update,
             bool backward) {
  const DevDesc& h0 = s[0]->lo.h;
  RET(quantise(s, n, p, st));
  // the plain FP32 ARM kernel fills every compute unit with vector work for
  // longer than the whole distortion branch; sharing the units with it made
  // the step slower, so only the fused form forks
  Fork fk(h0.arm_fused ? s[0]->device : -1, st);
  {
    // rate branch (a2-a4, a10), forked before the distortion branch (later
    // fork points measured slower: the ARM is the longer branch)
    const hipStream_t sr = fk.begin();
    RET(arm(s, n, backward ? 1 : 0, sr));
    if (backward && h0.G > 0) {
      TimeScope ts(TK_POOL, sr);
      RET(cc_launch_pool(plan(s, n, pool_blocks), sr));
    }
  }
  {
    TimeScope ts(TK_UPS_FWD, st);
    RET(ups_forward(s, n, st));
  }
  {
    TimeScope ts(TK_DIST_FWD, st);
    RET(forward_syn(s, n, 1, st));
  }
  if (backward) {
    const Launch lp = plan(s, n, [](const DevDesc& h) { return h.res_nwg; });
    int src_b = 0;
    {
      TimeScope ts(TK_RES_BWD, st);
      for (int r = h0.n_res - 1; r >= 0; --r) {
        RET(cc_launch_res_bwd2(lp, r, src_b, st));
        src_b ^= 1;
      }
    }
    {
      TimeScope ts(TK_SYN_BWD, st);
      RET(cc_launch_syn_bwd_plain(plan(s, n, [](const DevDesc& h) { return h.syn_nwg; }), h0, src_b, st));
    }
    {
      TimeScope ts(TK_UPS_BWD, st);
      RET(ups_backward(s, n, st));
    }
    RET(fk.join());
    // latent gradients (with the latents' Adam update when updating) and the
    // first pass of the decoder-parameter gradients in one launch, then the
    // second pass (with their Adam update) and, in one extra block per image,
    // the loss totals
    const bool soap = s[0]->optimizer == CC_OPT_SOAP;
    const Launch lj = plan(s, n, [](const DevDesc& h) {
      return h.lat_ntile + cdiv(h.n_par, 64) * CC_WRED_SPLIT;
    });
    const Launch w2 = plan(s, n, [](const DevDesc& h) { return cdiv(h.n_par, CC_ELT_TILE) + 1; });
    {
      TimeScope ts(TK_JOIN, st);
      RET(cc_launch_join_wreduce1(lj, update ? 1 : 0, st));
    }
    RET(cc_launch_wreduce2(w2, (update && !soap) ? 1 : 0, st));
    if (update && soap) {
      // SOAP on the decoder parameters: one workgroup per parameter tensor
      SoapPack a;
      memset(&a, 0, sizeof a);
      for (int i = 0; i < n; ++i) a.calls[i] = s[i]->soap_calls;
      RET(cc_launch_soap(plan(s, n, [](const DevDesc& h) { return h.soap_ntens; }), a, st));
      for (int i = 0; i < n; ++i) ++s[i]->soap_calls;
    }
    return CC_OK;
  }
  RET(fk.join());
  Launch lr;
  memset(&lr, 0, sizeof lr);
  lr.n = n;
  for (int i = 0; i < n; ++i) lr.d[i] = s[i]->ddev;
  RET(cc_launch_lreduce(lr, st));
  return CC_OK;
}

int read_scal(cc_state* s, double* out3, hipStream_t st) {
  double sc[4];
  HIPCHK(hipMemcpyAsync(sc, s->lo.h.scal, sizeof sc, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (out3) {
    out3[0] = sc[0];
    out3[1] = sc[1];
    out3[2] = sc[2];
  }
  if (sc[3] != 1.0) {
    s->nonfinite = 1;
    return fail(CC_ENONFINITE, "non-finite loss (%g)", sc[0]);
  }
  return CC_OK;
}

int check_state(const cc_state* s) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  if (s->nonfinite) return fail(CC_ENONFINITE, "an earlier step produced a non-finite loss");
  return CC_OK;
}

// ------------------------------------------------ no-allocation evaluation --
// cc_rd_eval_noalloc keeps every buffer its kernels write (a relocated copy
// of the descriptor, quantised latents, upsampled planes, synthesis
// activations, FP64 partial sums and totals) in this array instead of the
// state slab.  Host code never uses the symbol's name as an address: each
// device's copy is looked up once with hipGetSymbolAddress (at the first
// cc_init_state on that device, with the device current) and only that
// pointer is passed to kernels and copies.
constexpr size_t kNoallocBytes = CC_NOALLOC_SCRATCH_BYTES;

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxSideDev] = {};

// The calling thread's current device's copy of `scratch` (looked up on the
// first call per device).
int scratch_for_device(int dev, char** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxSideDev) return fail(CC_EDEVICE, "device %d outside the supported range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != dev)
      return fail(CC_EDEVICE, "the state's device %d is not current", dev);
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();   // not left for the next launch check to report
      return fail(CC_EDEVICE, "scratch symbol lookup failed: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return CC_OK;
}

// Descriptor of state h with every buffer an evaluation writes relocated into
// the scratch array at base; returns the bytes used (0 if they do not fit).
size_t relocate_eval(DevDesc& h, char* base) {
  size_t o = 0;
  auto take = [&](size_t n) {
    const size_t r = o;
    o = al256(o + n);
    return base + r;
  };
  const size_t npix = (size_t)h.H * h.W;
  size_t un = 0, vn = 0;
  for (int j = 1; j < h.L; ++j) {
    un += (size_t)(h.L - j) * h.gh[j - 1] * h.gw[j - 1];
    if (h.ups_conv) vn += (size_t)(h.L - j) * h.gh[j] * h.gw[j];
  }
  take(sizeof(DevDesc));
  h.yhat = (float*)take(sizeof(float) * (size_t)h.n_lat);
  h.dq = (float*)take(sizeof(float) * (size_t)h.n_lat);
  h.U = (float*)take(sizeof(float) * std::max<size_t>(un, 1));
  h.V = (float*)take(sizeof(float) * std::max<size_t>(vn, 1));
  h.X = (float*)take(sizeof(float) * (size_t)(h.n_res + 1) * 3 * npix);
  h.dXa = (float*)take(sizeof(float) * 3 * npix);   // the MSE epilogue's gradient
  h.lp_bits = (double*)take(sizeof(double) * (size_t)std::max(std::max(h.arm_nwg_plain, h.arm_nwg_fused), 1));
  h.lp_mse = (double*)take(sizeof(double) * (size_t)std::max(h.pix_ntile, 1));
  h.scal = (double*)take(sizeof(double) * 8);
  return o <= kNoallocBytes ? o : 0;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

const char* cc_last_error(void) { return g_err; }

int cc_config_supported(const cc_config* cfg, int H, int W) { return check_config(cfg, H, W) == CC_OK; }

int64_t cc_n_latents(const cc_config* cfg, int H, int W) {
  if (!cfg || cfg->L < 1 || cfg->L > CC_MAX_L) return -1;
  if (cfg->n_hyper < 0 || cfg->L + cfg->n_hyper > CC_MAX_G) return -1;
  int64_t n = 0;
  for (int k = 0; k < cfg->L; ++k) n += (int64_t)(H >> k) * (W >> k);
  for (int k = 0; k < cfg->n_hyper; ++k) n += (int64_t)(H >> (cfg->hyper_first + k)) * (W >> (cfg->hyper_first + k));
  return n;
}

int cc_arm_fused_available(const cc_config* cfg) {
  if (!cfg || check_config(cfg, 1 << (cfg->L - 1), 1 << (cfg->L - 1)) != CC_OK) return -1;
  Layout lo;
  build_layout(cfg, 1 << (cfg->L - 1), 1 << (cfg->L - 1), lo);
  return cc_arm_fused_supported(lo.h) ? 1 : 0;
}

int cc_n_params(const cc_config* cfg) {
  if (check_config(cfg, 1 << (cfg ? cfg->L - 1 : 0), 1 << (cfg ? cfg->L - 1 : 0)) != CC_OK) return -1;
  Layout lo;
  build_layout(cfg, 1 << (cfg->L - 1), 1 << (cfg->L - 1), lo);
  return lo.h.n_par;
}

size_t cc_state_bytes(const cc_config* cfg, int H, int W) {
  if (check_config(cfg, H, W) != CC_OK) return 0;
  Layout lo;
  build_layout(cfg, H, W, lo);
  return lo.bytes;
}

int cc_arm_band_plan(const cc_config* cfg, int H, int W, int nw, int* nbands, int* default_nw,
                     int* wbeg, int* blist) {
  int rc = check_config(cfg, H, W);
  if (rc != CC_OK) return rc;
  Layout lo;
  build_layout(cfg, H, W, lo);
  const DevDesc& h = lo.h;
  if (nbands) *nbands = h.arm_nwg_fused;
  if (default_nw) *default_nw = h.arm_wgs;
  if (!wbeg && !blist) return CC_OK;
  if (nw < 1 || nw > h.arm_nwg_fused)
    return fail(CC_EINVAL, "nw=%d outside [1, %d]", nw, h.arm_nwg_fused);
  std::vector<int> bl, wb;
  arm_pack(h, nw, bl, wb);
  if (wbeg) memcpy(wbeg, wb.data(), sizeof(int) * wb.size());
  if (blist) memcpy(blist, bl.data(), sizeof(int) * bl.size());
  return CC_OK;
}

int cc_init_state(const cc_config* cfg, int H, int W, const float* img_dev, double lambda,
                  uint64_t seed, const float* init_latents_host, const float* init_params_host,
                  void* mem, size_t bytes, void* stream, cc_state** out) {
  if (!out) return fail(CC_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_config(cfg, H, W);
  if (rc != CC_OK) return rc;
  if (!img_dev || !mem) return fail(CC_EINVAL, "image or slab pointer is NULL");
  if (((uintptr_t)mem & 255) != 0) return fail(CC_EINVAL, "slab must be 256-byte aligned");
  if (!(lambda >= 0.0) || !isfinite(lambda)) return fail(CC_EINVAL, "lambda must be finite and >= 0");
  cc_state* s = new (std::nothrow) cc_state();
  if (!s) return fail(CC_EINVAL, "host allocation failed");
  s->cfg = *cfg;
  build_layout(cfg, H, W, s->lo);
  if (bytes < s->lo.bytes) {
    const size_t need = s->lo.bytes;
    delete s;
    return fail(CC_ENOMEM, "state slab has %zu bytes, needs %zu", bytes, need);
  }
  s->base = (char*)mem;
  s->precision = cfg->precision;
  s->ddev = (DevDesc*)(s->base + s->lo.off_desc);
  if (hipGetDevice(&s->device) != hipSuccess) s->device = -1;
  {
    // set-up of the no-allocation evaluation's array on this device (once)
    char* sp = nullptr;
    if (s->device >= 0) (void)scratch_for_device(s->device, &sp);
  }
  set_pointers(s->lo, s->base);
  DevDesc& h = s->lo.h;
  h.lambda = lambda;
  h.rate_scale = (float)(lambda / ((double)H * W));
  h.mse_scale = (float)(2.0 / (3.0 * (double)H * W));
  h.seed_lo = (unsigned)(seed & 0xFFFFFFFFull);
  h.seed_hi = (unsigned)(seed >> 32);
  hipStream_t st = (hipStream_t)stream;
  std::vector<float> theta(h.n_theta, 0.0f);
  if (init_latents_host) memcpy(theta.data(), init_latents_host, sizeof(float) * h.n_lat);
  if (init_params_host) {
    memcpy(theta.data() + h.n_lat, init_params_host, sizeof(float) * h.n_par);
  } else {
    std::vector<float> P;
    default_params(h, seed, P);
    memcpy(theta.data() + h.n_lat, P.data(), sizeof(float) * h.n_par);
  }
  std::vector<float> zeros(h.n_theta, 0.0f);
  auto cp = [&](void* dst, const void* src, size_t n) { return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st); };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = cp(s->ddev, &h, sizeof(DevDesc));
  if (e == hipSuccess) e = hipMemcpyAsync(h.img, img_dev, sizeof(float) * 3 * (size_t)H * W, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = cp(h.theta, theta.data(), sizeof(float) * h.n_theta);
  if (e == hipSuccess) e = cp(h.m, zeros.data(), sizeof(float) * h.n_theta);
  if (e == hipSuccess) e = cp(h.v, zeros.data(), sizeof(float) * h.n_theta);
  if (e == hipSuccess) e = cp(h.grad, zeros.data(), sizeof(float) * h.n_theta);
  if (e == hipSuccess) e = cp(h.scal, zeros.data(), sizeof(double) * 8);
  if (e == hipSuccess) e = cp(h.arm_gtab, s->lo.arm_gtab.data(), sizeof(unsigned) * s->lo.arm_gtab.size());
  if (e == hipSuccess) e = cp(h.syn_gtab, s->lo.syn_gtab.data(), sizeof(unsigned) * s->lo.syn_gtab.size());
  if (e == hipSuccess) e = cp(h.arm_ftab, s->lo.arm_ftab.data(), sizeof(unsigned) * s->lo.arm_ftab.size());
  if (e == hipSuccess) e = cp(h.arm_blist, s->lo.arm_blist.data(), sizeof(int) * s->lo.arm_blist.size());
  if (e == hipSuccess) e = cp(h.arm_wbeg, s->lo.arm_wbeg.data(), sizeof(int) * s->lo.arm_wbeg.size());
  if (e == hipSuccess) e = cp(h.soap_tab, s->lo.soap_tab.data(), sizeof(int) * s->lo.soap_tab.size());
  if (e == hipSuccess) e = cp(h.nnq_group, s->lo.nnq_group.data(), s->lo.nnq_group.size());
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete s;
    return fail(CC_EDEVICE, "init copies failed: %s", hipGetErrorString(e));
  }
  *out = s;
  return CC_OK;
}

int cc_encode_step_batch(cc_state* const* states, int n, const cc_step_params* p, double* out,
                         void* stream) {
  if (!states || n < 1 || n > CC_MAX_BATCH) return fail(CC_EINVAL, "batch size %d outside [1, %d]", n, CC_MAX_BATCH);
  for (int i = 0; i < n; ++i) {
    int rc = check_state(states[i]);
    if (rc != CC_OK) return rc;
    rc = check_params(&p[i]);
    if (rc != CC_OK) return rc;
    if (!same_shape(states[0], states[i])) return fail(CC_EINVAL, "batch mixes decoder shapes or precisions");
    if (states[i]->optimizer != states[0]->optimizer) return fail(CC_EINVAL, "batch mixes optimisers");
  }
  hipStream_t st = (hipStream_t)stream;
  RET(run_step(states, n, p, st, true, true));
  for (int i = 0; i < n; ++i) states[i]->t = p[i].t;
  if (out) {
    int worst = CC_OK;
    for (int i = 0; i < n; ++i) {
      const int rc = read_scal(states[i], out + 3 * i, st);
      if (rc != CC_OK && worst == CC_OK) worst = rc;
    }
    return worst;
  }
  return CC_OK;
}

int cc_encode_step(cc_state* s, const cc_step_params* p, double* out3, void* stream) {
  return cc_encode_step_batch(&s, 1, p, out3, stream);
}

int cc_eval_loss(cc_state* s, const cc_step_params* p, double* out3, void* stream) {
  int rc = check_state(s);
  if (rc != CC_OK) return rc;
  rc = check_params(p);
  if (rc != CC_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  RET(run_step(&s, 1, p, st, false, false));
  double sc[4];
  HIPCHK(hipMemcpyAsync(sc, s->lo.h.scal, sizeof sc, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (out3) memcpy(out3, sc, 3 * sizeof(double));
  return CC_OK;
}

int cc_rd_eval(cc_state* s, cc_rd_result* out, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  cc_step_params p{};
  p.t = 1;
  p.quant_mode = CC_HARD;
  p.temperature = 1.0f;
  hipStream_t st = (hipStream_t)stream;
  RET(run_step(&s, 1, &p, st, false, false));
  double sc[4];
  HIPCHK(hipMemcpyAsync(sc, s->lo.h.scal, sizeof sc, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (out) {
    const double hw = (double)s->lo.h.H * s->lo.h.W;
    out->loss = sc[0];
    out->bits = sc[1];
    out->mse = sc[2];
    out->bpp = sc[1] / hw;
    out->psnr = sc[2] > 0 ? 10.0 * log10(1.0 / sc[2]) : INFINITY;
  }
  return CC_OK;
}

int cc_rd_eval_noalloc(cc_state* s, cc_rd_result* out, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  char* base = nullptr;
  RET(scratch_for_device(s->device, &base));
  DevDesc h = s->lo.h;
  const size_t used = relocate_eval(h, base);
  if (used == 0)
    return fail(CC_ENOMEM, "evaluation of a %dx%d state needs more than the %zu bytes of static scratch",
                s->lo.h.H, s->lo.h.W, kNoallocBytes);
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(base, &h, sizeof(DevDesc), hipMemcpyHostToDevice, st));
  cc_step_params p{};
  p.t = 1;
  p.quant_mode = CC_HARD;
  p.temperature = 1.0f;
  // the same launches as cc_rd_eval, reading the relocated descriptor
  DevDesc* const own = s->ddev;
  s->ddev = (DevDesc*)base;
  const int rc = run_step(&s, 1, &p, st, false, false);
  s->ddev = own;
  RET(rc);
  double sc[4];
  HIPCHK(hipMemcpyAsync(sc, h.scal, sizeof sc, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));   // also keeps h alive until its copy is done
  if (out) {
    const double hw = (double)h.H * h.W;
    out->loss = sc[0];
    out->bits = sc[1];
    out->mse = sc[2];
    out->bpp = sc[1] / hw;
    out->psnr = sc[2] > 0 ? 10.0 * log10(1.0 / sc[2]) : INFINITY;
  }
  return CC_OK;
}

int cc_nn_quantize(cc_state* s, cc_nnq_result* out, void* stream) {
  RET(check_state(s));
  hipStream_t st = (hipStream_t)stream;
  const DevDesc& h = s->lo.h;
  // keep the unquantised parameters; every candidate is written from them
  HIPCHK(hipMemcpyAsync(h.nnq_keep, h.theta + h.n_lat, sizeof(float) * h.n_par,
                        hipMemcpyDeviceToDevice, st));
  int size[CC_NNQ_NG] = {0};
  for (int p = 0; p < h.n_par; ++p) ++size[s->lo.nnq_group[p]];
  Launch l;
  memset(&l, 0, sizeof l);
  l.n = 1;
  l.d[0] = s->ddev;
  NnqPack pack;
  long long cnt[CC_NNQ_NG * CC_NNQ_NK];
  int chosen[4][2];
  for (int a = 0; a < 4; ++a) chosen[a][0] = chosen[a][1] = -1;
  const double hw = (double)h.H * h.W;
  // evaluates the current pack: hard-quantised latents with the decoder of
  // the pack; returns the cost and fills mse, latent bits and R_NN
  auto evaluate = [&](double* mse, double* bits, double* nn_bits, int* kap) -> int {
    RET(cc_launch_nnq(l, pack, st));
    cc_rd_result r;
    RET(cc_rd_eval(s, &r, st));
    HIPCHK(hipMemcpyAsync(cnt, h.nnq_bits, sizeof cnt, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double nb = 0.0;
    for (int g = 0; g < CC_NNQ_NG; ++g) {
      if (kap) kap[g] = -1;
      if (!(pack.step[0][g] > 0.0f) || size[g] == 0) continue;
      int bk = 0;
      for (int k = 1; k < CC_NNQ_NK; ++k)
        if (cnt[g * CC_NNQ_NK + k] < cnt[g * CC_NNQ_NK + bk]) bk = k;
      nb += (double)cnt[g * CC_NNQ_NK + bk];
      if (kap) kap[g] = bk;
    }
    *mse = r.mse;
    *bits = r.bits;
    *nn_bits = nb;
    return CC_OK;
  };
  auto set_pack = [&](int cur, int iw, int ib) {
    memset(&pack, 0, sizeof pack);
    for (int a = 0; a < 4; ++a) {
      const int w = a == cur ? iw : chosen[a][0], b = a == cur ? ib : chosen[a][1];
      pack.step[0][2 * a] = w >= 0 ? ldexpf(1.0f, w - 8) : 0.0f;
      pack.step[0][2 * a + 1] = b >= 0 ? ldexpf(1.0f, b - 8) : 0.0f;
    }
  };
  for (int a = 0; a < 4; ++a) {   // ARM, synthesis, upsampling, IFCE
    if (size[2 * a] == 0 && size[2 * a + 1] == 0) continue;
    double best = INFINITY;
    int bw = 0, bb = -1;
    for (int iw = 0; iw < CC_NNQ_NSTEP; ++iw)
      for (int ib = size[2 * a + 1] ? 0 : -1; ib < (size[2 * a + 1] ? CC_NNQ_NSTEP : 0); ++ib) {
        set_pack(a, size[2 * a] ? iw : -1, ib);
        double mse, bits, nb;
        RET(evaluate(&mse, &bits, &nb, nullptr));
        const double cost = mse + h.lambda * (bits + nb) / hw;
        if (cost < best) {
          best = cost;
          bw = size[2 * a] ? iw : -1;
          bb = ib;
        }
      }
    chosen[a][0] = bw;
    chosen[a][1] = bb;
  }
  set_pack(-1, -1, -1);
  double mse, bits, nb;
  int kap[CC_NNQ_NG];
  RET(evaluate(&mse, &bits, &nb, kap));
  if (out) {
    for (int a = 0; a < 4; ++a)
      for (int w = 0; w < 2; ++w) {
        out->step_index[a][w] = chosen[a][w];
        out->step[a][w] = chosen[a][w] >= 0 ? ldexp(1.0, chosen[a][w] - 8) : 0.0;
        out->kappa[a][w] = kap[2 * a + w];
      }
    out->nn_bits = nb;
    out->bits = bits;
    out->mse = mse;
    out->psnr = mse > 0 ? 10.0 * log10(1.0 / mse) : INFINITY;
    out->loss = mse + h.lambda * (bits + nb) / hw;
  }
  return CC_OK;
}

int cc_decode(cc_state* s, float* out_img_dev, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  if (!out_img_dev) return fail(CC_EINVAL, "output pointer is NULL");
  cc_step_params p{};
  p.t = 1;
  p.quant_mode = CC_HARD;
  p.temperature = 1.0f;
  hipStream_t st = (hipStream_t)stream;
  RET(quantise(&s, 1, &p, st));
  RET(ups_forward(&s, 1, st));
  RET(forward_syn(&s, 1, 0, st));
  RET(cc_launch_copy_out(plan(&s, 1, [](const DevDesc& h) { return cdiv(3 * h.H * h.W, CC_ELT_TILE); }), out_img_dev, st));
  return CC_OK;
}

int cc_get_state(cc_state* s, float* latents, float* params, float* adam_m, float* adam_v,
                 int64_t* t, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  if (latents) HIPCHK(hipMemcpyAsync(latents, h.theta, sizeof(float) * h.n_lat, hipMemcpyDeviceToHost, st));
  if (params) HIPCHK(hipMemcpyAsync(params, h.theta + h.n_lat, sizeof(float) * h.n_par, hipMemcpyDeviceToHost, st));
  if (adam_m) HIPCHK(hipMemcpyAsync(adam_m, h.m, sizeof(float) * h.n_theta, hipMemcpyDeviceToHost, st));
  if (adam_v) HIPCHK(hipMemcpyAsync(adam_v, h.v, sizeof(float) * h.n_theta, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (t) *t = s->t;
  return CC_OK;
}

int cc_set_state(cc_state* s, const float* latents, const float* params, const float* adam_m,
                 const float* adam_v, int64_t t, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  if (latents) HIPCHK(hipMemcpyAsync(h.theta, latents, sizeof(float) * h.n_lat, hipMemcpyHostToDevice, st));
  if (params) HIPCHK(hipMemcpyAsync(h.theta + h.n_lat, params, sizeof(float) * h.n_par, hipMemcpyHostToDevice, st));
  if (adam_m) HIPCHK(hipMemcpyAsync(h.m, adam_m, sizeof(float) * h.n_theta, hipMemcpyHostToDevice, st));
  if (adam_v) HIPCHK(hipMemcpyAsync(h.v, adam_v, sizeof(float) * h.n_theta, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  s->t = t;
  s->nonfinite = 0;
  return CC_OK;
}

int cc_get_grad(cc_state* s, float* grad_host, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  if (!grad_host) return fail(CC_EINVAL, "grad pointer is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(grad_host, s->lo.h.grad, sizeof(float) * s->lo.h.n_theta, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return CC_OK;
}

// ------------------------------------------------- per-module entry points
namespace {

int module_check(cc_state* s) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  return CC_OK;
}

int copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!bytes) return CC_OK;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
  return CC_OK;
}

// Load the caller's decoder parameters, then run the weight-gradient
// reduction and copy parameter range [b, e) of the gradient out.
int params_grad_out(cc_state* s, float* out, int b, int e, hipStream_t st) {
  const DevDesc& h = s->lo.h;
  cc_state* one[1] = {s};
  const Launch w1 = plan(one, 1, [](const DevDesc& x) { return cdiv(x.n_par, 64) * CC_WRED_SPLIT; });
  const Launch w2 = plan(one, 1, [](const DevDesc& x) { return cdiv(x.n_par, CC_ELT_TILE) + 1; });
  RET(cc_launch_wreduce(w1, w2, 0, st));
  return copy_d2d(out + b, h.grad + h.n_lat + b, sizeof(float) * (e - b), st);
}

}  // namespace

int cc_arm_fwd_bwd(cc_state* s, const float* yhat, const float* params, double* bits_out,
                   float* grad_yhat, float* grad_params, void* stream) {
  int rc = module_check(s);
  if (rc != CC_OK) return rc;
  if (!yhat || !params) return fail(CC_EINVAL, "yhat and params are required");
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  cc_state* one[1] = {s};
  const bool bwd = grad_yhat || grad_params;
  RET(copy_d2d(h.yhat, yhat, sizeof(float) * h.n_lat, st));
  RET(copy_d2d(h.theta + h.n_lat, params, sizeof(float) * h.n_par, st));
  // gradients of the bits themselves: rate scale 1
  RET(cc_launch_poke(&s->ddev->rate_scale, 1.0f, st));
  rc = arm(one, 1, bwd ? 1 : 0, st);
  if (rc == CC_OK && bwd && h.G > 0) {
    rc = cc_launch_pool(plan(one, 1, pool_blocks), st);
  }
  if (rc == CC_OK && grad_yhat)
    rc = cc_launch_join(plan(one, 1, [](const DevDesc& x) { return x.lat_ntile; }), st, grad_yhat);
  const int rc2 = cc_launch_poke(&s->ddev->rate_scale, h.rate_scale, st);
  if (rc != CC_OK || rc2 != CC_OK) return fail(CC_EDEVICE, "ARM module launch failed");
  if (grad_params) RET(params_grad_out(s, grad_params, 0, h.n_arm_par, st));
  Launch lr;
  memset(&lr, 0, sizeof lr);
  lr.n = 1;
  lr.d[0] = s->ddev;
  RET(cc_launch_lreduce(lr, st));
  if (bits_out) {
    double sc[4];
    HIPCHK(hipMemcpyAsync(sc, h.scal, sizeof sc, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *bits_out = sc[1];
  }
  return CC_OK;
}

int cc_ups_fwd(cc_state* s, const float* yhat, const float* params, float* zhat, void* stream) {
  int rc = module_check(s);
  if (rc != CC_OK) return rc;
  if (!yhat || !params || !zhat) return fail(CC_EINVAL, "null pointer");
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  cc_state* one[1] = {s};
  const size_t npx = (size_t)h.H * h.W;
  RET(copy_d2d(h.yhat, yhat, sizeof(float) * h.n_lat, st));
  RET(copy_d2d(h.theta + h.n_lat, params, sizeof(float) * h.n_par, st));
  RET(ups_forward(one, 1, st));
  RET(copy_d2d(zhat, h.yhat, sizeof(float) * npx, st));
  return copy_d2d(zhat + npx, h.U + h.uoff[1], sizeof(float) * (h.L - 1) * npx, st);
}

int cc_ups_bwd(cc_state* s, const float* grad_zhat, float* grad_yhat, float* grad_params, void* stream) {
  int rc = module_check(s);
  if (rc != CC_OK) return rc;
  if (!grad_zhat) return fail(CC_EINVAL, "null pointer");
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  cc_state* one[1] = {s};
  const size_t npx = (size_t)h.H * h.W;
  RET(copy_d2d(h.dyq, grad_zhat, sizeof(float) * npx, st));
  RET(copy_d2d(h.dU + h.uoff[1], grad_zhat + npx, sizeof(float) * (h.L - 1) * npx, st));
  RET(ups_backward(one, 1, st));
  if (grad_yhat) RET(copy_d2d(grad_yhat, h.dyq, sizeof(float) * h.n_lat, st));
  if (grad_params)
    RET(params_grad_out(s, grad_params, h.p_ups[1], h.p_ups[1] + 4 * (h.L - 1) * (h.ups_conv ? 2 : 1), st));
  return CC_OK;
}

int cc_syn_fwd(cc_state* s, const float* zhat, const float* params, float* xhat, void* stream) {
  int rc = module_check(s);
  if (rc != CC_OK) return rc;
  if (!zhat || !params || !xhat) return fail(CC_EINVAL, "null pointer");
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  cc_state* one[1] = {s};
  const size_t npx = (size_t)h.H * h.W;
  RET(copy_d2d(h.yhat, zhat, sizeof(float) * npx, st));
  RET(copy_d2d(h.U + h.uoff[1], zhat + npx, sizeof(float) * (h.L - 1) * npx, st));
  RET(copy_d2d(h.theta + h.n_lat, params, sizeof(float) * h.n_par, st));
  const Launch lp = plan(one, 1, [](const DevDesc& x) { return x.pix_ntile; });
  RET(cc_launch_syn_fwd_plain(lp, h, 0, st));
  for (int r = 0; r < h.n_res; ++r) RET(cc_launch_res_fwd(lp, r, r == h.n_res - 1, 0, st));
  return copy_d2d(xhat, h.X + (size_t)h.n_res * 3 * npx, sizeof(float) * 3 * npx, st);
}

int cc_syn_bwd(cc_state* s, const float* grad_xhat, float* grad_zhat, float* grad_params, void* stream) {
  int rc = module_check(s);
  if (rc != CC_OK) return rc;
  if (!grad_xhat) return fail(CC_EINVAL, "null pointer");
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  cc_state* one[1] = {s};
  const size_t npx = (size_t)h.H * h.W;
  RET(copy_d2d(h.dXa, grad_xhat, sizeof(float) * 3 * npx, st));
  const Launch lr = plan(one, 1, [](const DevDesc& x) { return x.res_nwg; });
  int src_b = 0;
  for (int r = h.n_res - 1; r >= 0; --r) {
    RET(cc_launch_res_bwd2(lr, r, src_b, st));
    src_b ^= 1;
  }
  RET(cc_launch_syn_bwd_plain(plan(one, 1, [](const DevDesc& x) { return x.syn_nwg; }), h, src_b, st));
  if (grad_zhat) {
    RET(copy_d2d(grad_zhat, h.dyq, sizeof(float) * npx, st));
    RET(copy_d2d(grad_zhat + npx, h.dU + h.uoff[1], sizeof(float) * (h.L - 1) * npx, st));
  }
  if (grad_params) RET(params_grad_out(s, grad_params, h.p_sw[0], h.n_par, st));
  return CC_OK;
}

int cc_debug_read(cc_state* s, const char* buffer, float* host, int64_t count, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  if (!buffer || !host || count < 0) return fail(CC_EINVAL, "bad arguments");
  const DevDesc& h = s->lo.h;
  const float* src = nullptr;
  int64_t n = 0;
  if (!strcmp(buffer, "yhat")) { src = h.yhat; n = h.n_lat; }
  else if (!strcmp(buffer, "dq")) { src = h.dq; n = h.n_lat; }
  else if (!strcmp(buffer, "dyd")) { src = h.dyd; n = h.n_lat; }
  else if (!strcmp(buffer, "dyq")) { src = h.dyq; n = h.n_lat; }
  else if (!strcmp(buffer, "xhat")) { src = h.X + (size_t)h.n_res * 3 * h.H * h.W; n = 3ll * h.H * h.W; }
  else if (!strcmp(buffer, "dx0")) { src = (h.n_res % 2) ? h.dXb : h.dXa; n = 3ll * h.H * h.W; }
  else return fail(CC_EINVAL, "unknown buffer '%s'", buffer);
  if (count > n) return fail(CC_EINVAL, "buffer '%s' holds %lld values", buffer, (long long)n);
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(host, src, sizeof(float) * count, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return CC_OK;
}

int cc_set_precision(cc_state* s, int precision) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  if (precision != CC_FP32_PLAIN && precision != CC_BF16_FUSED) return fail(CC_EINVAL, "precision=%d", precision);
  DevDesc& h = s->lo.h;
  s->precision = precision;
  h.arm_fused = (precision == CC_BF16_FUSED && cc_arm_fused_supported(h)) ? 1 : 0;
  arm_form(h);
  HIPCHK(hipMemcpy(s->ddev, &h, sizeof(DevDesc), hipMemcpyHostToDevice));
  return CC_OK;
}

int cc_set_launch_shape(cc_state* s, int arm_wgs, int syn_chunks_per_wg, int res_tiles_per_wg,
                        void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  DevDesc& h = s->lo.h;
  if (arm_wgs < 0 || arm_wgs > h.arm_nwg_fused)
    return fail(CC_EINVAL, "arm_wgs=%d outside [1, %d] (0 keeps it)", arm_wgs, h.arm_nwg_fused);
  if (syn_chunks_per_wg != 0 && (syn_chunks_per_wg < CC_SYN_CPW_MIN || syn_chunks_per_wg > CC_SYN_CPW_MAX))
    return fail(CC_EINVAL, "synthesis chunks per workgroup %d outside [%d, %d]", syn_chunks_per_wg,
                CC_SYN_CPW_MIN, CC_SYN_CPW_MAX);
  if (res_tiles_per_wg < 0 || res_tiles_per_wg > CC_RES_TPW_MAX)
    return fail(CC_EINVAL, "residual tiles per workgroup %d outside [1, %d]", res_tiles_per_wg, CC_RES_TPW_MAX);
  // no step of this state may still read the descriptor (the side stream's
  // work joins back into the caller's stream, so this waits for it too)
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  if (arm_wgs > 0) {
    h.arm_wgs = arm_wgs;
    arm_pack(h, h.arm_wgs, s->lo.arm_blist, s->lo.arm_wbeg);
    HIPCHK(hipMemcpy(h.arm_blist, s->lo.arm_blist.data(), sizeof(int) * s->lo.arm_blist.size(),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h.arm_wbeg, s->lo.arm_wbeg.data(), sizeof(int) * s->lo.arm_wbeg.size(),
                     hipMemcpyHostToDevice));
  }
  if (syn_chunks_per_wg > 0) {
    h.syn_cpw = syn_chunks_per_wg;
    h.syn_nwg = cdiv(h.syn_nchunk, h.syn_cpw);
    h.prod[h.prod_syn].nrows = h.syn_nwg;
  }
  if (res_tiles_per_wg > 0) {
    h.res_tpw = res_tiles_per_wg;
    h.res_nwg = cdiv(res_tiles(h), h.res_tpw);
    for (int r = 0; r < h.n_res; ++r) h.prod[h.prod_res0 + r].nrows = h.res_nwg;
  }
  HIPCHK(hipMemcpy(s->ddev, &h, sizeof(DevDesc), hipMemcpyHostToDevice));
  return CC_OK;
}

int cc_get_launch_shape(const cc_state* s, int* arm_wgs, int* syn_chunks_per_wg, int* res_tiles_per_wg,
                        int* arm_bands) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  const DevDesc& h = s->lo.h;
  if (arm_wgs) *arm_wgs = h.arm_wgs;
  if (syn_chunks_per_wg) *syn_chunks_per_wg = h.syn_cpw;
  if (res_tiles_per_wg) *res_tiles_per_wg = h.res_tpw;
  if (arm_bands) *arm_bands = h.arm_nwg_fused;
  return CC_OK;
}

int cc_set_optimizer(cc_state* s, int optimizer, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  if (optimizer != CC_OPT_ADAM && optimizer != CC_OPT_SOAP) return fail(CC_EINVAL, "optimizer=%d", optimizer);
  const DevDesc& h = s->lo.h;
  if (optimizer == CC_OPT_SOAP) {
    for (int t = 0; t < h.soap_ntens; ++t)
      if (s->lo.soap_tab[(size_t)t * CC_SOAP_TAB + 1] > CC_SOAP_MAXNUMEL)
        return fail(CC_EINVAL, "parameter tensor %d has more than %d values", t, CC_SOAP_MAXNUMEL);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemsetAsync(h.soap_m, 0, sizeof(float) * h.n_par, st));
    HIPCHK(hipMemsetAsync(h.soap_v, 0, sizeof(float) * h.n_par, st));
    s->soap_calls = 0;
  }
  s->optimizer = optimizer;
  return CC_OK;
}

int64_t cc_soap_factor_size(const cc_config* cfg) {
  if (check_config(cfg, 1 << (cfg ? cfg->L - 1 : 0), 1 << (cfg ? cfg->L - 1 : 0)) != CC_OK) return -1;
  Layout lo;
  build_layout(cfg, 1 << (cfg->L - 1), 1 << (cfg->L - 1), lo);
  return lo.h.soap_nfac;
}

int cc_get_soap_state(cc_state* s, float* m, float* v, float* p, float* q, int* calls, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  if (m) HIPCHK(hipMemcpyAsync(m, h.soap_m, sizeof(float) * h.n_par, hipMemcpyDeviceToHost, st));
  if (v) HIPCHK(hipMemcpyAsync(v, h.soap_v, sizeof(float) * h.n_par, hipMemcpyDeviceToHost, st));
  if (p) HIPCHK(hipMemcpyAsync(p, h.soap_p, sizeof(float) * h.soap_nfac, hipMemcpyDeviceToHost, st));
  if (q) HIPCHK(hipMemcpyAsync(q, h.soap_q, sizeof(float) * h.soap_nfac, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (calls) *calls = s->soap_calls;
  return CC_OK;
}

int cc_set_soap_state(cc_state* s, const float* m, const float* v, const float* p, const float* q,
                      int calls, void* stream) {
  if (!s || !s->ddev) return fail(CC_ESTATE, "state not initialised");
  if (calls < 0) return fail(CC_EINVAL, "calls=%d", calls);
  const DevDesc& h = s->lo.h;
  hipStream_t st = (hipStream_t)stream;
  if (m) HIPCHK(hipMemcpyAsync(h.soap_m, m, sizeof(float) * h.n_par, hipMemcpyHostToDevice, st));
  if (v) HIPCHK(hipMemcpyAsync(h.soap_v, v, sizeof(float) * h.n_par, hipMemcpyHostToDevice, st));
  if (p) HIPCHK(hipMemcpyAsync(h.soap_p, p, sizeof(float) * h.soap_nfac, hipMemcpyHostToDevice, st));
  if (q) HIPCHK(hipMemcpyAsync(h.soap_q, q, sizeof(float) * h.soap_nfac, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  s->soap_calls = calls;
  return CC_OK;
}

int cc_set_branch_overlap(int enable) {
  return g_overlap.exchange(enable != 0) ? 1 : 0;
}

int cc_timing_enable(const char* kernel) {
  int k = TK_NONE;
  if (kernel && !strcmp(kernel, "arm")) k = TK_ARM;
  else if (kernel && !strcmp(kernel, "syn_bwd")) k = TK_SYN_BWD;
  else if (kernel && !strcmp(kernel, "res_bwd")) k = TK_RES_BWD;
  else if (kernel && !strcmp(kernel, "ups_bwd")) k = TK_UPS_BWD;
  else if (kernel && !strcmp(kernel, "join")) k = TK_JOIN;
  else if (kernel && !strcmp(kernel, "ups_fwd")) k = TK_UPS_FWD;
  else if (kernel && !strcmp(kernel, "pool")) k = TK_POOL;
  else if (kernel && !strcmp(kernel, "syn_fwd")) k = TK_DIST_FWD;
  else if (kernel && kernel[0]) return fail(CC_EINVAL, "unknown kernel class '%s'", kernel);
  g_timing.kind = k;
  g_timing.used = 0;
  g_timing.seen = 0;
  return CC_OK;
}
int cc_timing_every(int n) {
  if (n < 1) return fail(CC_EINVAL, "n=%d", n);
  g_timing.every = n;
  return CC_OK;
}

int cc_timing_read(double* total_ms, int* count) {
  double tot = 0.0;
  int n = 0;
  for (size_t i = 0; i + 1 < g_timing.used; i += 2) {
    HIPCHK(hipEventSynchronize(g_timing.ev[i + 1]));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, g_timing.ev[i], g_timing.ev[i + 1]));
    tot += ms;
    ++n;
  }
  if (total_ms) *total_ms = tot;
  if (count) *count = n;
  g_timing.used = 0;
  return CC_OK;
}

void cc_free_state(cc_state* s) { delete s; }

}  // extern "C"
