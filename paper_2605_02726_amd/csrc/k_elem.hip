// Elementwise and reduction kernels of the encode step: per-step scalars,
// training quantisation proxy with in-kernel Philox noise, IFCE gradient
// pyramid, the join of all latent gradients, deterministic reductions and
// Adam.
#include "cc_internal.h"

#include <math.h>

namespace {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies with the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const unsigned lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// Box-Muller on the top 24 bits of two words: u1 = (k + 1/2) 2^-24 with
// k = r0 >> 8 (never zero), u2 = (r1 >> 8) 2^-24.  k + 1/2 needs 25 bits when
// k >= 2^23, so there ln(u1) is taken as log1p(-(1 - u1)) with
// 1 - u1 = (2^24 - 1/2 - k) 2^-24, which is exact in FP32 on that half.
__device__ __forceinline__ float gauss(unsigned r0, unsigned r1) {
  const unsigned k = r0 >> 8;
  float lnu1;
  if (k >= (1u << 23))
    lnu1 = log1pf(-((float)(0xFFFFFFu - k) + 0.5f) * 5.9604644775390625e-8f);
  else
    lnu1 = logf(((float)k + 0.5f) * 5.9604644775390625e-8f);
  const float u2 = (float)(r1 >> 8) * 5.9604644775390625e-8f;
  return sqrtf(-2.0f * lnu1) * cospif(2.0f * u2);
}

// Softround s_T (Section IV-C, eq. softround) and its derivative;
// c = 1 / (2 tanh(1 / 2T)), invT = 1 / T.
// Written as s_T(x) = n + e with n the integer nearest to x: with f the
// distance from x to n and a = 1/(2T), |e| = c (tanh(a) - tanh(a - f/T)),
// and tanh(a) - tanh(b) = -2 exp(-2b) expm1(-2(a - b)) / ((1 + exp(-2a))
// (1 + exp(-2b))) has no cancellation.  The direct form fl + c tanh(..) + 1/2
// cancels where tanh saturates and leaves an absolute error of ~1e-7 on
// values near 0 at low temperature (relative error up to 100% there).
__device__ __forceinline__ float softround(float x, float c, float invT) {
  const float fl = floorf(x);
  const float fr = x - fl;                          // exact
  const bool lo = fr < 0.5f;
  const float n = lo ? fl : fl + 1.0f;
  const float f = lo ? fr : (fl + 1.0f) - x;        // exact (Sterbenz)
  const float B = expf(-2.0f * (0.5f - f) * invT);  // exp(-2b), b = (1/2 - f) / T
  const float A = expf(-invT);                      // exp(-2a)
  const float e = -2.0f * c * B * expm1f(-2.0f * f * invT) / ((1.0f + A) * (1.0f + B));
  return lo ? n + e : n - e;
}
// 1 - tanh^2(a) written as 4 e / (1 + e)^2 with e = exp(-2 |a|): no
// cancellation where tanh saturates near the half-integers.
__device__ __forceinline__ float dsoftround(float x, float c, float invT) {
  const float fl = floorf(x);
  const float a = fabsf((x - fl - 0.5f) * invT);
  const float e = expf(-2.0f * a);
  const float q = 1.0f + e;
  return invT * c * (4.0f * e / (q * q));
}

__device__ __forceinline__ int grid_of(const CDesc* d, int i) {
  int k = 0;
  while (k + 1 < d->NG && i >= d->goff[k + 1]) ++k;
  return k;
}

// Adam (Kingma and Ba) on element i of theta = [latents, parameters] with
// its gradient g; the step's learning rate and bias corrections come from
// the descriptor.
__device__ __forceinline__ void adam_update(const CDesc* d, int i, float g) {
  const float m = 0.9f * d->m[i] + 0.1f * g;
  const float v = 0.999f * d->v[i] + 0.001f * (g * g);
  d->m[i] = m;
  d->v[i] = v;
  const float mh = m / d->bc1, vh = v / d->bc2;
  d->theta[i] -= d->lr * mh / (sqrtf(vh) + 1e-8f);
}

// yhat = s_T(s_T(y) + sigma n) with n from Philox counter (t, k, i, 0), and
// d yhat / d y; or yhat = rint(y) with a straight-through derivative of 1.
// The step's schedule values arrive as kernel arguments; the first block of
// each image also stores them in the descriptor for the later kernels of the
// step.
__global__ __launch_bounds__(CC_ELT_TILE) void k_qtrain(Launch L, StepPack A) {
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const StepArgs a = A.a[im];
  const int b = blockIdx.x - L.tile0[im];
  if (b == 0 && threadIdx.x == 0) {
    DevDesc* dw = const_cast<DevDesc*>(L.d[im]);
    dw->T = a.T;
    dw->sr_c = a.sr_c;
    dw->sr_invT = a.sr_invT;
    dw->sigma = a.sigma;
    dw->lr = a.lr;
    dw->bc1 = a.bc1;
    dw->bc2 = a.bc2;
    dw->t_lo = a.t_lo;
    dw->mode = a.mode;
    dw->upd = a.upd;
  }
  if (b == 0) {
    // A non-finite decoder parameter need not reach the loss (a ReLU maps a
    // NaN pre-activation to 0), so the step checks them all here and the
    // loss totals report the state as non-finite (scal[4] = 1).
    int bad = 0;
    for (int p = threadIdx.x; p < d->n_par; p += CC_ELT_TILE) bad |= !isfinite(d->theta[d->n_lat + p]);
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) d->scal[4] = bad ? 1.0 : 0.0;
  }
  const int i = b * CC_ELT_TILE + threadIdx.x;
  if (i >= d->n_lat) return;
  const float y = d->theta[i];
  float yh, dq;
  if (a.mode == CC_HARD) {
    yh = rintf(y);
    dq = 1.0f;
  } else {
    const int k = grid_of(d, i);
    const uint4 r = philox10(make_uint4(a.t_lo, (unsigned)k, (unsigned)(i - d->goff[k]), 0u),
                             d->seed_lo, d->seed_hi);
    const float n = gauss(r.x, r.y);
    const float c = a.sr_c, iT = a.sr_invT;
    const float s0 = softround(y, c, iT);
    const float u = s0 + a.sigma * n;
    yh = softround(u, c, iT);
    dq = dsoftround(u, c, iT) * dsoftround(y, c, iT);
  }
  d->yhat[i] = yh;
  d->dq[i] = dq;
}

// The IFCE gradient pyramid in one launch: level f of child grid c (at grid
// c+f) holds the 2x2 sums of level f-1, level 0 being the IFCE feature
// gradient the ARM kernel wrote at grid c.  A workgroup takes one channel
// and one base block of side B = 2^(L-1-c) (the sides are multiples of it)
// and builds every level of that block in LDS, adding each 2x2 group as
// (top-left + top-right) + (bottom-left + bottom-right).
__global__ __launch_bounds__(CC_ELT_TILE) void k_pool(Launch L) {
  __shared__ float buf[2][CC_POOL_BLOCK * CC_POOL_BLOCK / 4];
  __shared__ float base[CC_POOL_BLOCK * CC_POOL_BLOCK];
  __shared__ float red[CC_MAX_NIN][CC_ELT_TILE / 64];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  int b = blockIdx.x - L.tile0[im];
  int c = 0;
  for (; c < d->G; ++c) {
    const int B = 1 << (d->L - 1 - c);
    const int nt = d->F * (d->gh[c] / B) * (d->gw[c] / B);
    if (b < nt) break;
    b -= nt;
  }
  if (c >= d->G) return;
  const int B = 1 << (d->L - 1 - c);
  const int tx = d->gw[c] / B, ty = d->gh[c] / B;
  const int ch = b / (tx * ty), t = b - ch * (tx * ty);
  const int by = t / tx, bx = t - by * tx;
  // the plain ARM kernel writes the per-position gradients (level 0); the
  // fused one writes them already summed over 2 x 2 blocks (level 1)
  const int l0 = d->arm_fused ? 1 : 0;
  const int Bb = B >> l0;
  {
    const int w0 = d->gw[c + l0], n0 = d->gh[c + l0] * w0;
    const float* src = d->df + d->dfoff[c][l0] + (size_t)ch * n0;
    // loads in groups of 8 per thread, each group issued before its LDS
    // stores, so their latencies overlap
    constexpr int NB = 8;
    for (int i0 = 0; i0 < Bb * Bb; i0 += NB * CC_ELT_TILE) {
      float v[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int i = i0 + u * CC_ELT_TILE + threadIdx.x;
        const int y = i / Bb, x = i - y * Bb;
        v[u] = i < Bb * Bb ? src[(by * Bb + y) * w0 + bx * Bb + x] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int i = i0 + u * CC_ELT_TILE + threadIdx.x;
        if (i < Bb * Bb) base[i] = v[u];
      }
    }
  }
  __syncthreads();
  // fused form: the IFCE weight gradient of feature ch,
  //   dW[ch][q] = sum over the grid's positions of df_ch * r_q,
  // where input q is grid isrc[c][q] read at (y >> s, x >> s), s = ish[c][q],
  // equals the sum over that input grid's positions of its value times the
  // df sum pooled to shift s, which this block forms below; the bias
  // gradient is the block's whole sum
  const bool wgrad = d->arm_fused != 0;
  const int nin = d->nin[c];
  float acc[CC_MAX_NIN];
#pragma unroll
  for (int q = 0; q < CC_MAX_NIN; ++q) acc[q] = 0.0f;
  auto wgrad_level = [&](int f, int so, int i, float v) {
    const int y = i / so, x = i - y * so;
#pragma unroll
    for (int q = 0; q < CC_MAX_NIN; ++q) {
      if (q < nin && d->ish[c][q] == f) {
        const int j = d->isrc[c][q];
        acc[q] += v * d->yhat[d->goff[j] + (by * so + y) * d->gw[j] + bx * so + x];
      }
    }
  };
  if (wgrad && l0 > 0)
    for (int i = threadIdx.x; i < Bb * Bb; i += CC_ELT_TILE) wgrad_level(l0, Bb, i, base[i]);
  const float* in = base;
  int side = Bb;
  for (int f = l0 + 1; f <= d->L - 1 - c; ++f) {
    const int so = side >> 1;
    float* out = buf[f & 1];
    const int w = d->gw[c + f], n = d->gh[c + f] * w;
    float* dst = d->df + d->dfoff[c][f] + (size_t)ch * n;
    for (int i = threadIdx.x; i < so * so; i += CC_ELT_TILE) {
      const int y = i / so, x = i - y * so;
      const float* r0 = in + (2 * y) * side + 2 * x;
      const float v = (r0[0] + r0[1]) + (r0[side] + r0[side + 1]);
      out[i] = v;
      dst[(by * so + y) * w + bx * so + x] = v;
      if (wgrad) wgrad_level(f, so, i, v);
    }
    __syncthreads();
    in = out;
    side = so;
  }
  if (!wgrad) return;
  // fixed-order block sums: lanes (xor tree), then the waves in order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < CC_MAX_NIN; ++q) {
    float v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[q][wv] = v;
  }
  __syncthreads();
  const int pi = d->prod_ifce0 + c;
  float* row = d->wp + d->prod[pi].off + (size_t)(by * tx + bx) * d->prod[pi].pcnt;
  if (threadIdx.x < nin) {
    float s = 0.0f;
    for (int u = 0; u < CC_ELT_TILE / 64; ++u) s += red[threadIdx.x][u];
    row[ch * nin + threadIdx.x] = s;
  } else if (threadIdx.x == CC_MAX_NIN) {
    // the last level holds one value: the block's sum of df_ch
    row[d->F * nin + ch] = in[0];
  }
}

// Gradient of the loss with respect to every latent y:
//   (d rate / d yhat + d distortion / d yhat) * d yhat / d y
// where d rate / d yhat gathers, in a fixed order, the direct term, the
// context gradients of the positions that use this latent as a causal
// neighbour (reversed offsets) and the IFCE gradients of finer grids; a
// hyperlatent (grid >= L) feeds every IFCE and has no distortion term.
__device__ __forceinline__ void join_tile(const CDesc* d, int tile, float* rate_only_out, int adam) {
  const int i = tile * CC_ELT_TILE + threadIdx.x;
  if (i >= d->n_lat) return;
  const int k = grid_of(d, i);
  const int h = d->gh[k], w = d->gw[k], li = i - d->goff[k];
  const int y = li / w, x = li - y * w;
  float g;
  if (d->arm_fused) {
    // planes of the band-tiled kernel: own band, then the halo rows written
    // by the bands q = 1 .. CC_FUSED_HPLANES below (the causal reach is 4 rows)
    g = d->dc[i];
    const int band = y / CC_FUSED_BAND, nb = (h + CC_FUSED_BAND - 1) / CC_FUSED_BAND;
#pragma unroll
    for (int q = 1; q <= CC_FUSED_HPLANES; ++q)
      if (band + q < nb) g += d->dc[(size_t)q * d->n_lat + i];
  } else {
    g = d->dyd[i];
    const float* dc = d->dc + d->goff[k];
    for (int m = 0; m < d->S; ++m) {
      const int sy = y - d->dy[m], sx = x - d->dx[m];
      if (sy >= 0 && sy < h && sx >= 0 && sx < w) g += dc[(size_t)m * d->n_lat + sy * w + sx];
    }
  }
  const CF* P = (const CF*)(d->theta + d->n_lat);
  const int nk = h * w, lev = d->glev[k];
  const bool hyper = k >= d->L;
  for (int c = 0; c < d->G && (hyper || c < k); ++c) {
    const CF* W = P + d->p_iw[c];             // [F, nin[c]]
    // input slot of this grid in the IFCE of grid c: the coarser latent
    // grids first, then the hyperlatent grids
    const int q = k - c - 1, nin = d->nin[c];
    const float* D = d->df + d->dfoff[c][lev - c];   // pooled to this resolution
    for (int f = 0; f < d->F; ++f) g += W[f * nin + q] * D[f * nk + li];
  }
  if (rate_only_out) {
    rate_only_out[i] = g;
    return;
  }
  if (!hyper) g += d->dyq[i];
  g *= d->dq[i];
  d->grad[i] = g;
  if (adam && d->upd) adam_update(d, i, g);
}

__global__ __launch_bounds__(CC_ELT_TILE) void k_join(Launch L, float* rate_only_out, int adam) {
  const int im = cc_find_img(L, blockIdx.x);
  join_tile((const CDesc*)L.d[im], blockIdx.x - L.tile0[im], rate_only_out, adam);
}

__global__ void k_poke(float* p, float v) { *p = v; }

__device__ __forceinline__ double block_sum_256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// FP64 totals of one image in a fixed order: scal = (loss, bits, mse, finite);
// finite also needs every decoder parameter finite (scal[4], set by the
// quantiser kernel of the same step).
__device__ void loss_totals(const CDesc* d, double* sh) {
  double b = 0.0, m = 0.0;
  for (int r = threadIdx.x; r < d->arm_nwg; r += 256) b += d->lp_bits[r];
  const double bits = block_sum_256(b, sh);
  __syncthreads();
  for (int r = threadIdx.x; r < d->pix_nwg; r += 256) m += d->lp_mse[r];
  const double sq = block_sum_256(m, sh);
  if (threadIdx.x == 0) {
    const double mse = sq / (3.0 * d->H * d->W);
    const double loss = mse + d->lambda * bits / ((double)d->H * d->W);
    d->scal[0] = loss;
    d->scal[1] = bits;
    d->scal[2] = mse;
    d->scal[3] = (isfinite(loss) && d->scal[4] == 0.0) ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_lreduce(Launch L) {
  __shared__ double sh[256];
  loss_totals((const CDesc*)L.d[blockIdx.x], sh);
}

// Weight-gradient reduction, pass 1: block (param block of 64, row split s)
// sums its share of every producer's partial rows in FP64, fixed order.
__device__ __forceinline__ void wreduce1_block(const CDesc* d, int b, double (*sh)[64]) {
  const int pb = b / CC_WRED_SPLIT, s = b - pb * CC_WRED_SPLIT;
  const int lane = threadIdx.x & 63, sub = threadIdx.x >> 6;
  const int p = pb * 64 + lane;
  double acc = 0.0;
  if (p < d->n_par) {
    int q = 0;
    while (q < d->nprod && !(p >= d->prod[q].pbeg && p < d->prod[q].pbeg + d->prod[q].pcnt)) ++q;
    if (q < d->nprod) {
      const int nrows = d->prod[q].nrows, pcnt = d->prod[q].pcnt;
      const int per = (nrows + CC_WRED_SPLIT - 1) / CC_WRED_SPLIT;
      const int r0 = s * per, r1 = min(nrows, r0 + per);
      const float* base = d->wp + d->prod[q].off + (p - d->prod[q].pbeg);
      for (int r = r0 + sub; r < r1; r += 4) acc += (double)base[(size_t)r * pcnt];
    }
  }
  sh[sub][lane] = acc;
  __syncthreads();
  if (sub == 0 && p < d->n_par)
    d->wp2[(size_t)s * d->n_par + p] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

__global__ __launch_bounds__(256) void k_wreduce1(Launch L) {
  __shared__ double sh[4][64];
  const int im = cc_find_img(L, blockIdx.x);
  wreduce1_block((const CDesc*)L.d[im], blockIdx.x - L.tile0[im], sh);
}

// The latent join (with the latents' Adam update) and the first pass of the
// weight-gradient reduction in one launch: per image, the join's tiles first,
// then the reduction's blocks (the two read disjoint data).
__global__ __launch_bounds__(256) void k_join_wreduce1(Launch L, int adam) {
  __shared__ double sh[4][64];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int b = blockIdx.x - L.tile0[im];
  if (b < d->lat_ntile)
    join_tile(d, b, nullptr, adam);
  else
    wreduce1_block(d, b - d->lat_ntile, sh);
}

// Pass 2: gradient of decoder parameter p = sum of the row splits.
// Weight-gradient reduction, pass 2: the CC_WRED_SPLIT partial sums of each
// parameter in a fixed order, then (adam) its Adam update.  The last block of
// each image computes the image's FP64 loss totals instead.
__global__ __launch_bounds__(CC_ELT_TILE) void k_wreduce2(Launch L, int adam) {
  __shared__ double sh[CC_ELT_TILE];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int b = blockIdx.x - L.tile0[im];
  if (b == L.tile0[im + 1] - L.tile0[im] - 1) {
    loss_totals(d, sh);
    return;
  }
  const int p = b * CC_ELT_TILE + threadIdx.x;
  if (p >= d->n_par) return;
  double acc = 0.0;
  for (int s = 0; s < CC_WRED_SPLIT; ++s) acc += d->wp2[(size_t)s * d->n_par + p];
  const float g = (float)acc;
  d->grad[d->n_lat + p] = g;
  if (adam) adam_update(d, d->n_lat + p, g);
}

__global__ __launch_bounds__(CC_ELT_TILE) void k_copy_out(Launch L, float* out) {
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int i = (blockIdx.x - L.tile0[im]) * CC_ELT_TILE + threadIdx.x;
  const int n = 3 * d->H * d->W;
  if (i >= n) return;
  out[i] = d->X[(size_t)d->n_res * n + i];
}

inline int check_launch() {
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EDEVICE;
}

}  // namespace

int cc_launch_qtrain(const Launch& l, const StepPack& a, hipStream_t st) {
  hipLaunchKernelGGL(k_qtrain, dim3(l.tile0[l.n]), dim3(CC_ELT_TILE), 0, st, l, a);
  return check_launch();
}
int cc_launch_pool(const Launch& l, hipStream_t st) {
  if (l.tile0[l.n] == 0) return CC_OK;
  hipLaunchKernelGGL(k_pool, dim3(l.tile0[l.n]), dim3(CC_ELT_TILE), 0, st, l);
  return check_launch();
}
int cc_launch_join(const Launch& l, hipStream_t st, float* rate_only_out, int adam) {
  hipLaunchKernelGGL(k_join, dim3(l.tile0[l.n]), dim3(CC_ELT_TILE), 0, st, l, rate_only_out, adam);
  return check_launch();
}
int cc_launch_poke(float* p, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_poke, dim3(1), dim3(1), 0, st, p, v);
  return check_launch();
}
int cc_launch_lreduce(const Launch& l, hipStream_t st) {
  hipLaunchKernelGGL(k_lreduce, dim3(l.n), dim3(256), 0, st, l);
  return check_launch();
}
int cc_launch_join_wreduce1(const Launch& lj, int adam_latents, hipStream_t st) {
  hipLaunchKernelGGL(k_join_wreduce1, dim3(lj.tile0[lj.n]), dim3(256), 0, st, lj, adam_latents);
  return check_launch();
}
int cc_launch_wreduce2(const Launch& l2, int adam_params, hipStream_t st) {
  hipLaunchKernelGGL(k_wreduce2, dim3(l2.tile0[l2.n]), dim3(CC_ELT_TILE), 0, st, l2, adam_params);
  return check_launch();
}
int cc_launch_wreduce(const Launch& l1, const Launch& l2, int adam, hipStream_t st) {
  hipLaunchKernelGGL(k_wreduce1, dim3(l1.tile0[l1.n]), dim3(256), 0, st, l1);
  if (check_launch() != CC_OK) return CC_EDEVICE;
  hipLaunchKernelGGL(k_wreduce2, dim3(l2.tile0[l2.n]), dim3(CC_ELT_TILE), 0, st, l2, adam);
  return check_launch();
}
int cc_launch_copy_out(const Launch& l, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_out, dim3(l.tile0[l.n]), dim3(CC_ELT_TILE), 0, st, l, out);
  return check_launch();
}
