// Distortion branch of the encode step, plain FP32 form: learned upsampling
// (Section III-B), synthesis trunk with stabilizer (Sections III-B, III-C),
// residual 3x3 post-filters, the MSE (Section IV-A) and the exact adjoints of
// all of them.
//
// Upsampling level j maps T_j (L-j channels at grid j) to U_j = Up_j(T_j)
// (L-j channels at grid j-1), where T_j = [yhat^(j); U_{j+1}] and
// Up_j is the symmetric 8-tap kernel (h0 h1 h2 h3 h3 h2 h1 h0) applied as a
// stride-2 transposed convolution (padding 3, replicate edge) on rows and on
// columns: output o reads the 4 inputs clamp((o + 3 - t) / 2) for the taps t
// with the parity of o + 3.  zhat = [yhat^(0); U_1].  With the Conv
// refinement, level j first filters T_j with the symmetric 7-tap kernel
// (c3 c2 c1 c0 c1 c2 c3) on rows and columns (replicate edge), V_j =
// Conv_j(T_j), and the transposed convolution reads V_j instead of T_j.
#include "cc_internal.h"

#include <math.h>

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Taps of output o: 4 (tap index, clamped input index) pairs.
__device__ __forceinline__ void out_taps(int o, int n, int* t, int* idx) {
  const int t0 = (o + 3) & 1;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    t[a] = t0 + 2 * a;
    idx[a] = clampi((o + 3 - t[a]) >> 1, 0, n - 1);
  }
}

__device__ __forceinline__ float tapv(const float* h, int t) { return h[t < 4 ? t : 7 - t]; }

// Input channel ch of T_j at position p (grid j).
__device__ __forceinline__ const float* tchan(const CDesc* d, int j, int ch) {
  return ch == 0 ? d->yhat + d->goff[j] : d->U + d->uoff[j + 1] + (size_t)(ch - 1) * d->gh[j] * d->gw[j];
}

// Input channel ch of the transposed convolution of level j: V_j with the
// Conv refinement, else T_j.
__device__ __forceinline__ const float* usrc(const CDesc* d, int j, int ch) {
  return d->ups_conv ? d->V + d->voff[j] + (size_t)ch * d->gh[j] * d->gw[j] : tchan(d, j, ch);
}

__device__ __forceinline__ float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// U_j = Up_j(T_j): one thread per output pixel of grid j-1, all channels.
__global__ __launch_bounds__(CC_PIX_TILE) void k_ups_fwd(Launch L, int j) {
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int ho = d->gh[j - 1], wo = d->gw[j - 1], hi = d->gh[j], wi = d->gw[j];
  const int p = cc_xcd_index(L, im) * CC_PIX_TILE + threadIdx.x;
  if (p >= ho * wo) return;
  const int oy = p / wo, ox = p - oy * wo;
  const CF* hc = (const CF*)(d->theta + d->n_lat + d->p_ups[j]);
  const float h[4] = {hc[0], hc[1], hc[2], hc[3]};
  int ty[4], iy[4], tx[4], ix[4];
  out_taps(oy, hi, ty, iy);
  out_taps(ox, wi, tx, ix);
  float wy[4], wx[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    wy[a] = tapv(h, ty[a]);
    wx[a] = tapv(h, tx[a]);
  }
  const int nch = d->L - j;
  float* out = d->U + d->uoff[j];
  for (int ch = 0; ch < nch; ++ch) {
    const float* in = usrc(d, j, ch);
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      float r = 0.0f;
#pragma unroll
      for (int b = 0; b < 4; ++b) r += wx[b] * in[iy[a] * wi + ix[b]];
      s += wy[a] * r;
    }
    out[(size_t)ch * ho * wo + p] = s;
  }
}

// Weight of input i in output o along one axis (sum over the taps of o whose
// clamped index is i).
__device__ __forceinline__ float axis_w(const float* h, int o, int i, int n) {
  int t[4], idx[4];
  out_taps(o, n, t, idx);
  float w = 0.0f;
#pragma unroll
  for (int a = 0; a < 4; ++a)
    if (idx[a] == i) w += tapv(h, t[a]);
  return w;
}

// Adjoint of level j on 16x16 tiles of grid j (inputs), all channels.
// With R = column adjoint of dU_j (rows: outputs, columns: inputs) and
// Bm = row adjoint (rows: inputs, columns: outputs), the input gradient is
// the row adjoint of R, and the tap gradient of the symmetric kernel is
//   sum over (output row oy, input column ix) of R[oy][ix] * d/dh of the row
//   taps of oy applied to T, plus sum over (input row iy, output column ox)
//   of Bm[iy][ox] * d/dh of the column taps of ox applied to T,
// each (oy, ix) / (iy, ox) pair owned by exactly one tile (the tile of ix /
// iy whose output rows / columns 2*tile .. 2*tile+31 contain oy / ox).
// Channel 0 of dT_j is the distortion gradient of yhat^(j), channels >= 1 are
// dU_{j+1}.  One workgroup per (channel, tile); one partial row of 4 tap
// gradients per workgroup.
constexpr int UT = CC_UPS_TILE;   // input tile side
constexpr int UG = 2 * UT + 6;   // output window side (2*UT + 3 + 3)
constexpr int UTW = UT + 4;      // input window side (2 each side)
static_assert(UT * 8 <= 256, "one thread per (tile row, tap) for the axis weights");

__global__ __launch_bounds__(256) void k_ups_bwd(Launch L, int j) {
  __shared__ float g[UG][UG + 1];
  __shared__ float t[UTW][UTW + 1];
  __shared__ float R[UG][UT + 1];
  __shared__ float Bm[UT][2 * UT + 1];
  __shared__ float wxs[UT][8], wys[UT][8];
  __shared__ float sh[4][4];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int wgi = cc_xcd_index(L, im);
  const int ho = d->gh[j - 1], wo = d->gw[j - 1], hi = d->gh[j], wi = d->gw[j];
  const int ntx = (wi + UT - 1) / UT, ntile = ntx * ((hi + UT - 1) / UT);
  const int ch = wgi / ntile, tile = wgi - ch * ntile;   // one channel of one tile
  const int iy0 = (tile / ntx) * UT, ix0 = (tile % ntx) * UT;
  const CF* hp = (const CF*)(d->theta + d->n_lat + d->p_ups[j]);
  const float hv[4] = {hp[0], hp[1], hp[2], hp[3]};
  const int tid = threadIdx.x;
  if (tid < UT * 8) {
    const int a = tid & 7, q = tid >> 3;
    const int iy = iy0 + q, ix = ix0 + q;
    const int oy = 2 * iy - 3 + a, ox = 2 * ix - 3 + a;
    wys[q][a] = (iy < hi && oy >= 0 && oy < ho) ? axis_w(hv, oy, iy, hi) : 0.0f;
    wxs[q][a] = (ix < wi && ox >= 0 && ox < wo) ? axis_w(hv, ox, ix, wi) : 0.0f;
  }
  float dh[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  {
    const float* gsrc = d->dU + d->uoff[j] + (size_t)ch * ho * wo;
    const float* tsrc = usrc(d, j, ch);
    // every load of the thread is issued before the first LDS store, so
    // their latencies overlap
    constexpr int NG = (UG * UG + 255) / 256, NT = (UTW * UTW + 255) / 256;
    float gv[NG], tv[NT];
#pragma unroll
    for (int u = 0; u < NG; ++u) {
      const int i = tid + 256 * u;
      const int r = i / UG, c = i - r * UG;
      const int oy = 2 * iy0 - 3 + r, ox = 2 * ix0 - 3 + c;
      gv[u] = (i < UG * UG && oy >= 0 && oy < ho && ox >= 0 && ox < wo) ? gsrc[oy * wo + ox] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int i = tid + 256 * u;
      const int r = i / UTW, c = i - r * UTW;
      tv[u] = i < UTW * UTW ? tsrc[clampi(iy0 - 2 + r, 0, hi - 1) * wi + clampi(ix0 - 2 + c, 0, wi - 1)] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < NG; ++u) {
      const int i = tid + 256 * u;
      if (i < UG * UG) (&g[0][0])[(i / UG) * (UG + 1) + i % UG] = gv[u];
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int i = tid + 256 * u;
      if (i < UTW * UTW) (&t[0][0])[(i / UTW) * (UTW + 1) + i % UTW] = tv[u];
    }
    __syncthreads();
    for (int i = tid; i < UG * UT; i += 256) {
      const int r = i / UT, q = i - r * UT;
      float a = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) a += wxs[q][b] * g[r][2 * q + b];
      R[r][q] = a;
    }
    for (int i = tid; i < UT * 2 * UT; i += 256) {
      const int q = i / (2 * UT), c = i - q * (2 * UT);
      float a = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) a += wys[q][b] * g[2 * q + b][c + 3];
      Bm[q][c] = a;
    }
    __syncthreads();
    for (int i = tid; i < UT * UT; i += 256) {
      const int q = i / UT, p = i - q * UT;
      const int iy = iy0 + q, ix = ix0 + p;
      if (iy < hi && ix < wi) {
        float a = 0.0f;
#pragma unroll
        for (int b = 0; b < 8; ++b) a += wys[q][b] * R[2 * q + b][p];
        if (d->ups_conv)
          d->dV[d->voff[j] + (size_t)ch * hi * wi + iy * wi + ix] = a;
        else if (ch == 0)
          d->dyq[d->goff[j] + iy * wi + ix] = a;
        else
          d->dU[d->uoff[j + 1] + (size_t)(ch - 1) * hi * wi + iy * wi + ix] = a;
      }
    }
    // tap gradients: term over (oy owned, ix in tile) and (iy in tile, ox owned)
    for (int i = tid; i < 2 * UT * UT; i += 256) {
      const int ol = i / UT, p = i - ol * UT;      // output row offset, input column
      const int oy = 2 * iy0 + ol, ix = ix0 + p;
      if (oy < ho && ix < wi) {
        int tt[4], idx[4];
        out_taps(oy, hi, tt, idx);
        const float rv = R[ol + 3][p];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float v = rv * t[idx[a] - (iy0 - 2)][p + 2];
          const int qq = tt[a] < 4 ? tt[a] : 7 - tt[a];
          dh[qq] += v;
        }
      }
      const int q = i / (2 * UT), oc = i - q * (2 * UT);   // input row, output column offset
      const int iy = iy0 + q, ox = 2 * ix0 + oc;
      if (iy < hi && ox < wo) {
        int tt[4], idx[4];
        out_taps(ox, wi, tt, idx);
        const float bv = Bm[q][oc];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float v = bv * t[q + 2][idx[a] - (ix0 - 2)];
          const int qq = tt[a] < 4 ? tt[a] : 7 - tt[a];
          dh[qq] += v;
        }
      }
    }
  }
  const int wv = tid >> 6, ln = tid & 63;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float s2 = wave_sum(dh[q]);
    if (ln == 0) sh[q][wv] = s2;
  }
  __syncthreads();
  if (tid < 4) {
    const float s2 = (sh[tid][0] + sh[tid][1]) + (sh[tid][2] + sh[tid][3]);
    const long long pg_off = d->prod[d->prod_ups1 + j - 1].off;
    d->wp[pg_off + (size_t)wgi * 4 + tid] = s2;
  }
}

// ------------------------------------------------- Conv refinement ----
// Both kernels take one workgroup (256 threads) per (channel of T_j, tile of
// CC_UPC_TH x CC_UPC_TW positions of grid j) and stage a window with a 3-wide
// halo in LDS, every load of a thread issued before the first LDS store.
constexpr int CTH = CC_UPC_TH, CTW = CC_UPC_TW;
constexpr int CWH = CTH + 6, CWW = CTW + 6;   // window with the 7-tap halo
constexpr int NWIN = (CWH * CWW + 255) / 256;
static_assert(CTW == 64, "the passes index tile columns by lane");

// 7-tap symmetric kernel k[0..6] = (c3 c2 c1 c0 c1 c2 c3) of level j.
__device__ __forceinline__ void conv_kernel7(const CDesc* d, int j, float* k) {
  const CF* c = (const CF*)(d->theta + d->n_lat + d->p_upc[j]);
  k[3] = c[0];
  k[2] = k[4] = c[1];
  k[1] = k[5] = c[2];
  k[0] = k[6] = c[3];
}

// Tile of workgroup wgi at level j: channel and top-left corner.
__device__ __forceinline__ void upc_tile(const CDesc* d, int j, int wgi, int& ch, int& y0, int& x0) {
  const int ntx = (d->gw[j] + CTW - 1) / CTW, nt = ntx * ((d->gh[j] + CTH - 1) / CTH);
  ch = wgi / nt;
  const int t = wgi - ch * nt;
  y0 = (t / ntx) * CTH;
  x0 = (t - (t / ntx) * ntx) * CTW;
}

// win[r][c] = src[clamp(y0 - 3 + r)][clamp(x0 - 3 + c)] (clamped = replicate
// edge) or, with zero_out, 0 outside the grid.
__device__ __forceinline__ void load_window(const float* src, int y0, int x0, int hi, int wi,
                                            bool zero_out, float (*win)[CWW + 1]) {
  float v[NWIN];
#pragma unroll
  for (int u = 0; u < NWIN; ++u) {
    const int i = threadIdx.x + 256 * u;
    const int r = i / CWW, c = i - r * CWW;
    const int y = y0 - 3 + r, x = x0 - 3 + c;
    const bool in = y >= 0 && y < hi && x >= 0 && x < wi;
    v[u] = (i < CWH * CWW && (in || !zero_out)) ? src[clampi(y, 0, hi - 1) * wi + clampi(x, 0, wi - 1)]
                                                : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < NWIN; ++u) {
    const int i = threadIdx.x + 256 * u;
    if (i < CWH * CWW) win[i / CWW][i % CWW] = v[u];
  }
}

// V_j = Conv_j(T_j): V[y][x] = sum_a k[a] sum_b k[b] T[clamp(y + a - 3)][clamp(x + b - 3)],
// rows pass into LDS, then the columns pass.
__global__ __launch_bounds__(256) void k_upc_fwd(Launch L, int j) {
  __shared__ float win[CWH][CWW + 1];
  __shared__ float rp[CWH][CTW + 1];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int hi = d->gh[j], wi = d->gw[j];
  int ch, y0, x0;
  upc_tile(d, j, cc_xcd_index(L, im), ch, y0, x0);
  float k[7];
  conv_kernel7(d, j, k);
  load_window(tchan(d, j, ch), y0, x0, hi, wi, false, win);
  __syncthreads();
  for (int i = threadIdx.x; i < CWH * CTW; i += 256) {
    const int r = i >> 6, x = i & 63;
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b < 7; ++b) s += k[b] * win[r][x + b];
    rp[r][x] = s;
  }
  __syncthreads();
  float* out = d->V + d->voff[j] + (size_t)ch * hi * wi;
  for (int i = threadIdx.x; i < CTH * CTW; i += 256) {
    const int y = i >> 6, x = i & 63;
    if (y0 + y < hi && x0 + x < wi) {
      float s = 0.0f;
#pragma unroll
      for (int a = 0; a < 7; ++a) s += k[a] * rp[y + a][x];
      out[(y0 + y) * wi + x0 + x] = s;
    }
  }
}

// Weights of the outputs o = i - 3 .. i + 3 on input i along one axis of
// length n (the clamped 7-tap filter's adjoint); 0 for outputs outside.
__device__ __forceinline__ void conv_adj_w(const float* k, int i, int n, float* w) {
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    const int o = i + a - 3;
    float s = 0.0f;
    if (o >= 0 && o < n) {
#pragma unroll
      for (int e = 0; e < 7; ++e)
        if (clampi(o + e - 3, 0, n - 1) == i) s += k[e];
    }
    w[a] = s;
  }
}

// Adjoint of Conv_j.  dT_j = Conv_j^T(dV_j) (columns pass into LDS, then the
// rows pass) goes to the distortion gradient of yhat^(j) (channel 0) or to
// dU_{j+1}.  The tap gradient of c_q is the sum over outputs o of dV[o] times
// (the row-filtered T at rows o_y -+ q plus the column-filtered T at columns
// o_x -+ q; once for q = 0).  One partial row of 4 tap gradients per workgroup.
__global__ __launch_bounds__(256) void k_upc_bwd(Launch L, int j) {
  __shared__ float gw[CWH][CWW + 1];    // dV window, 0 outside the grid
  __shared__ float tw[CWH][CWW + 1];    // T window, replicate edge
  __shared__ float c1[CWH][CTW + 1];    // dV through the columns adjoint
  __shared__ float rt[CWH][CTW + 1];    // T through the row taps
  __shared__ float ct[CTH][CWW + 1];    // T through the column taps
  __shared__ float awx[CTW][7], awy[CTH][7];
  __shared__ float sh[4][4];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int wgi = cc_xcd_index(L, im);
  const int hi = d->gh[j], wi = d->gw[j], n = hi * wi;
  const int tid = threadIdx.x;
  int ch, y0, x0;
  upc_tile(d, j, wgi, ch, y0, x0);
  float k[7];
  conv_kernel7(d, j, k);
  load_window(d->dV + d->voff[j] + (size_t)ch * n, y0, x0, hi, wi, true, gw);
  load_window(tchan(d, j, ch), y0, x0, hi, wi, false, tw);
  if (tid < CTW) conv_adj_w(k, x0 + tid, wi, awx[tid]);
  else if (tid < CTW + CTH) conv_adj_w(k, y0 + tid - CTW, hi, awy[tid - CTW]);
  __syncthreads();
  for (int i = tid; i < CWH * CTW; i += 256) {
    const int r = i >> 6, x = i & 63;
    float s = 0.0f, t = 0.0f;
#pragma unroll
    for (int b = 0; b < 7; ++b) {
      s += awx[x][b] * gw[r][x + b];
      t += k[b] * tw[r][x + b];
    }
    c1[r][x] = s;
    rt[r][x] = t;
  }
  for (int i = tid; i < CTH * CWW; i += 256) {
    const int y = i / CWW, c = i - y * CWW;
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 7; ++a) s += k[a] * tw[y + a][c];
    ct[y][c] = s;
  }
  __syncthreads();
  float dc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int i = tid; i < CTH * CTW; i += 256) {
    const int y = i >> 6, x = i & 63;
    const int iy = y0 + y, ix = x0 + x;
    if (iy < hi && ix < wi) {
      float g = 0.0f;
#pragma unroll
      for (int a = 0; a < 7; ++a) g += awy[y][a] * c1[y + a][x];
      if (ch == 0)
        d->dyq[d->goff[j] + iy * wi + ix] = g;
      else
        d->dU[d->uoff[j + 1] + (size_t)(ch - 1) * n + iy * wi + ix] = g;
      const float gv = gw[y + 3][x + 3];
      dc[0] += gv * (rt[y + 3][x] + ct[y][x + 3]);
#pragma unroll
      for (int q = 1; q < 4; ++q)
        dc[q] += gv * ((rt[y + 3 - q][x] + rt[y + 3 + q][x]) + (ct[y][x + 3 - q] + ct[y][x + 3 + q]));
    }
  }
  const int wv = tid >> 6, ln = tid & 63;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float s2 = wave_sum(dc[q]);
    if (ln == 0) sh[q][wv] = s2;
  }
  __syncthreads();
  if (tid < 4) {
    const float s2 = (sh[tid][0] + sh[tid][1]) + (sh[tid][2] + sh[tid][3]);
    d->wp[d->prod[d->prod_upc1 + j - 1].off + (size_t)wgi * 4 + tid] = s2;
  }
}

// ------------------------------------------- coarse levels, per source ----
// Channel c of U_j is source grid j + c upsampled through levels j + c, ...,
// j, so the sources are independent chains.  The levels from ups_jc up (each
// output grid at most CC_UPS_COARSE positions) run as one workgroup per
// source g: the forward takes yhat^(g) through levels g, g-1, ..., ups_jc
// with every intermediate in LDS (writing each U_j channel for the synthesis
// and the backward), the backward takes dU_{ups_jc} channel g - ups_jc
// through levels ups_jc, ..., g down to d yhat^(g) and the tap gradients (one
// partial row per (level, source)).  Rows then columns, in the same
// operation order as k_ups_fwd, so the forward values are identical.
constexpr int CT = CC_UPS_CHAIN_T;
constexpr int CW = CT / 64;   // wavefronts

// 2-D loops of the chain kernels: rows over the wavefronts, columns over the
// lanes (no division by a run-time width).
#define CC_FOR2D(rows, cols, r, c)                                  \
  for (int r = threadIdx.x >> 6; r < (rows); r += CW)               \
    for (int c = threadIdx.x & 63; c < (cols); c += 64)

// Rows pass: R[iy][ox] = sum_b w_x,b(ox) * A[iy][ix_b(ox)], for hi x wo.
__device__ __forceinline__ void rows_pass(const float* h, const float* A, float* R, int hi, int wi,
                                          int wo) {
  CC_FOR2D(hi, wo, iy, ox) {
    int tx[4], ix[4];
    out_taps(ox, wi, tx, ix);
    float r = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) r += tapv(h, tx[b]) * A[iy * wi + ix[b]];
    R[iy * wo + ox] = r;
  }
}

// Columns pass: B[oy][x] = sum_a w_y,a(oy) * R[iy_a(oy)][x], for ho x w.
__device__ __forceinline__ void cols_pass(const float* h, const float* R, float* B, int hi, int ho,
                                          int w) {
  CC_FOR2D(ho, w, oy, x) {
    int ty[4], iy[4];
    out_taps(oy, hi, ty, iy);
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) s += tapv(h, ty[a]) * R[iy[a] * w + x];
    B[oy * w + x] = s;
  }
}

// Adjoint weights of one axis: wa[i][b] = weight of input i in output
// 2 i - 3 + b (zero outside the output range).
__device__ __forceinline__ void adj_weights(const float* h, float (*wa)[8], int n_in, int n_out) {
  for (int e = threadIdx.x; e < 8 * n_in; e += CT) {
    const int i = e >> 3, b = e & 7, o = 2 * i - 3 + b;
    wa[i][b] = (o >= 0 && o < n_out) ? axis_w(h, o, i, n_in) : 0.0f;
  }
}

// Conv refinement passes of the chain kernels (h x w <= CC_UPS_COARSE / 4):
// rows R[y][x] = sum_b k[b] A[y][clamp(x + b - 3)], columns
// B[y][x] = sum_a k[a] R[clamp(y + a - 3)][x].
__device__ __forceinline__ void conv_rows(const float* k, const float* A, float* R, int h, int w) {
  CC_FOR2D(h, w, y, x) {
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b < 7; ++b) s += k[b] * A[y * w + clampi(x + b - 3, 0, w - 1)];
    R[y * w + x] = s;
  }
}
__device__ __forceinline__ void conv_cols(const float* k, const float* R, float* B, int h, int w) {
  CC_FOR2D(h, w, y, x) {
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 7; ++a) s += k[a] * R[clampi(y + a - 3, 0, h - 1) * w + x];
    B[y * w + x] = s;
  }
}

__global__ __launch_bounds__(CT) void k_ups_fwd_chain(Launch L) {
  __shared__ float bufA[CC_UPS_COARSE], bufB[CC_UPS_COARSE], rw[CC_UPS_COARSE / 2];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int jc = d->ups_jc;
  const int g = jc + (blockIdx.x - L.tile0[im]);   // source grid
  float* A = bufA;
  float* B = bufB;
  {
    const float* src = d->yhat + d->goff[g];
    for (int i = threadIdx.x; i < d->gh[g] * d->gw[g]; i += CT) A[i] = src[i];
  }
  for (int j = g; j >= jc; --j) {
    const int hi = d->gh[j], wi = d->gw[j], ho = d->gh[j - 1], wo = d->gw[j - 1];
    const CF* hc = (const CF*)(d->theta + d->n_lat + d->p_ups[j]);
    const float h[4] = {hc[0], hc[1], hc[2], hc[3]};
    const bool conv = d->ups_conv != 0;
    __syncthreads();
    const float* src = A;   // the transposed convolution's input
    if (conv) {
      float k7[7];
      conv_kernel7(d, j, k7);
      conv_rows(k7, A, rw, hi, wi);
      __syncthreads();
      conv_cols(k7, rw, B, hi, wi);
      __syncthreads();
      src = B;
    }
    rows_pass(h, src, rw, hi, wi, wo);
    __syncthreads();
    float* dst = conv ? A : B;
    cols_pass(h, rw, dst, hi, ho, wo);
    __syncthreads();
    float* out = d->U + d->uoff[j] + (size_t)(g - j) * ho * wo;
    for (int i = threadIdx.x; i < ho * wo; i += CT) out[i] = dst[i];
    if (!conv) {
      float* t = A;
      A = B;
      B = t;
    }
  }
}

__global__ __launch_bounds__(CT) void k_ups_bwd_chain(Launch L) {
  __shared__ float bufG[CC_UPS_COARSE], bufD[CC_UPS_COARSE];
  __shared__ float tin[CC_UPS_COARSE / 4], rc[CC_UPS_COARSE / 2], rf[CC_UPS_COARSE / 2],
      cf[CC_UPS_COARSE / 2];
  __shared__ float wxa[CC_UPS_COARSE / 4][8], wya[CC_UPS_COARSE / 4][8];
  // Conv refinement: T through the Conv's row taps and column taps, V_j,
  // d V_j and the columns adjoint of d V_j
  __shared__ float crt[CC_UPS_COARSE / 4], cct[CC_UPS_COARSE / 4], vin[CC_UPS_COARSE / 4],
      dvb[CC_UPS_COARSE / 4], ctmp[CC_UPS_COARSE / 4];
  __shared__ float sh[4][CW];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int jc = d->ups_jc;
  const int g = jc + (blockIdx.x - L.tile0[im]);   // source grid
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  float* G = bufG;
  float* D = bufD;
  {
    const int ho = d->gh[jc - 1], wo = d->gw[jc - 1];
    const float* src = d->dU + d->uoff[jc] + (size_t)(g - jc) * ho * wo;
    for (int i = tid; i < ho * wo; i += CT) G[i] = src[i];
  }
  for (int j = jc; j <= g; ++j) {
    const int hi = d->gh[j], wi = d->gw[j], ho = d->gh[j - 1], wo = d->gw[j - 1];
    const CF* hc = (const CF*)(d->theta + d->n_lat + d->p_ups[j]);
    const float h[4] = {hc[0], hc[1], hc[2], hc[3]};
    {
      const float* ts = tchan(d, j, g - j);
      for (int i = tid; i < hi * wi; i += CT) tin[i] = ts[i];
    }
    const bool conv = d->ups_conv != 0;
    float k7[7];
    if (conv) conv_kernel7(d, j, k7);
    adj_weights(h, wxa, wi, wo);
    adj_weights(h, wya, hi, ho);
    __syncthreads();
    const float* tsrc = tin;   // the transposed convolution's input
    if (conv) {
      conv_rows(k7, tin, crt, hi, wi);
      conv_cols(k7, tin, cct, hi, wi);
      __syncthreads();
      conv_cols(k7, crt, vin, hi, wi);
      __syncthreads();
      tsrc = vin;
    }
    // column adjoint of G: rc[oy][ix] over the outputs ox = 2 ix - 3 + b
    CC_FOR2D(ho, wi, oy, ix) {
      float a = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int ox = 2 * ix - 3 + b;
        a += wxa[ix][b] * G[oy * wo + clampi(ox, 0, wo - 1)];
      }
      rc[oy * wi + ix] = a;
    }
    rows_pass(h, tsrc, rf, hi, wi, wo);   // rf[iy][ox]: T through the row taps
    // cf[oy][ix]: T through the column taps
    CC_FOR2D(ho, wi, oy, ix) {
      int ty[4], iy[4];
      out_taps(oy, hi, ty, iy);
      float s = 0.0f;
#pragma unroll
      for (int a = 0; a < 4; ++a) s += tapv(h, ty[a]) * tsrc[iy[a] * wi + ix];
      cf[oy * wi + ix] = s;
    }
    __syncthreads();
    // row adjoint of rc: d T_j channel g - j
    CC_FOR2D(hi, wi, iy, ix) {
      float a = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int oy = 2 * iy - 3 + b;
        a += wya[iy][b] * rc[clampi(oy, 0, ho - 1) * wi + ix];
      }
      if (conv) {
        dvb[iy * wi + ix] = a;
      } else {
        D[iy * wi + ix] = a;
        if (j == g) d->dyq[d->goff[g] + iy * wi + ix] = a;
      }
    }
    // tap gradients: every output o contributes G[o] times the derivative of
    // U[o] in each tap, through the row taps (rf) and the column taps (cf)
    float dh[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    CC_FOR2D(ho, wo, oy, ox) {
      const float gv = G[oy * wo + ox];
      int ty[4], iy[4], tx[4], ix[4];
      out_taps(oy, hi, ty, iy);
      out_taps(ox, wi, tx, ix);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int qa = ty[a] < 4 ? ty[a] : 7 - ty[a];
        const int qb = tx[a] < 4 ? tx[a] : 7 - tx[a];
        const float va = gv * rf[iy[a] * wo + ox];
        const float vb = gv * cf[oy * wi + ix[a]];
#pragma unroll
        for (int q = 0; q < 4; ++q) dh[q] += (qa == q ? va : 0.0f) + (qb == q ? vb : 0.0f);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float s2 = wave_sum(dh[q]);
      if (ln == 0) sh[q][wv] = s2;
    }
    __syncthreads();
    if (tid < 4) {
      float s2 = 0.0f;
      for (int w2 = 0; w2 < CW; ++w2) s2 += sh[tid][w2];
      const long long pg_off = d->prod[d->prod_ups1 + j - 1].off;
      d->wp[pg_off + (size_t)(g - j) * 4 + tid] = s2;
    }
    if (conv) {
      // adjoint of the Conv (columns of the filter, then rows) into D, and
      // its tap gradients from T's row- and column-filtered copies
      __syncthreads();
      CC_FOR2D(hi, wi, y, x) {
        float aw[7];
        conv_adj_w(k7, x, wi, aw);
        float s = 0.0f;
#pragma unroll
        for (int b = 0; b < 7; ++b) {
          const int ox = x + b - 3;
          if (ox >= 0 && ox < wi) s += aw[b] * dvb[y * wi + ox];
        }
        ctmp[y * wi + x] = s;
      }
      __syncthreads();
      float dc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      CC_FOR2D(hi, wi, y, x) {
        float aw[7];
        conv_adj_w(k7, y, hi, aw);
        float s = 0.0f;
#pragma unroll
        for (int a = 0; a < 7; ++a) {
          const int oy = y + a - 3;
          if (oy >= 0 && oy < hi) s += aw[a] * ctmp[oy * wi + x];
        }
        D[y * wi + x] = s;
        if (j == g) d->dyq[d->goff[g] + y * wi + x] = s;
        const float gv = dvb[y * wi + x];
        dc[0] += gv * (crt[y * wi + x] + cct[y * wi + x]);
#pragma unroll
        for (int q = 1; q < 4; ++q)
          dc[q] += gv * ((crt[clampi(y - q, 0, hi - 1) * wi + x] + crt[clampi(y + q, 0, hi - 1) * wi + x]) +
                         (cct[y * wi + clampi(x - q, 0, wi - 1)] + cct[y * wi + clampi(x + q, 0, wi - 1)]));
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float s2 = wave_sum(dc[q]);
        if (ln == 0) sh[q][wv] = s2;
      }
      __syncthreads();
      if (tid < 4) {
        float s2 = 0.0f;
        for (int w2 = 0; w2 < CW; ++w2) s2 += sh[tid][w2];
        d->wp[d->prod[d->prod_upc1 + j - 1].off + (size_t)(g - j) * 4 + tid] = s2;
      }
    }
    float* t = G;
    G = D;
    D = t;
    __syncthreads();
  }
}

// ------------------------------------------------------------ synthesis ----
template <int NH, int W1, int W2>
struct SynShape {
  static constexpr int WL = NH == 2 ? W2 : W1;  // width of the last hidden layer
};

// Trunk of one pixel: z (L <= 8 values) -> hidden -> 3, plus stabilizer.
template <int NH, int W1, int W2>
__device__ __forceinline__ void syn_mlp(const CDesc* d, const CF* P, const float* z,
                                        float* h1, float* h2, float* out) {
  const int L = d->L;
  const CF* Wa = P + d->p_sw[0];
  const CF* Ba = P + d->p_sb[0];
#pragma unroll
  for (int a = 0; a < W1; ++a) {
    float s = Ba[a];
#pragma unroll
    for (int q = 0; q < CC_MAX_L; ++q)
      if (q < L) s += Wa[a * L + q] * z[q];
    h1[a] = fmaxf(s, 0.0f);
  }
  if constexpr (NH == 2) {
    const CF* Wb = P + d->p_sw[1];
    const CF* Bb = P + d->p_sb[1];
#pragma unroll
    for (int a = 0; a < W2; ++a) {
      float s = Bb[a];
#pragma unroll
      for (int q = 0; q < W1; ++q) s += Wb[a * W1 + q] * h1[q];
      h2[a] = fmaxf(s, 0.0f);
    }
  }
  constexpr int WL = SynShape<NH, W1, W2>::WL;
  const float* hl = NH == 2 ? h2 : h1;
  const CF* Wc = P + d->p_sw[NH];
  const CF* Bc = P + d->p_sb[NH];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float s = Bc[c];
#pragma unroll
    for (int q = 0; q < WL; ++q) s += Wc[c * WL + q] * hl[q];
    out[c] = s;
  }
  if (d->syn_stab) {
    const CF* Ws = P + d->p_ssw;
    const CF* Bs = P + d->p_ssb;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float s = Bs[c];
#pragma unroll
      for (int q = 0; q < CC_MAX_L; ++q)
        if (q < L) s += Ws[c * L + q] * z[q];
      out[c] += s;
    }
  }
}

__device__ __forceinline__ void load_z(const CDesc* d, int p, float* z) {
  const int n = d->H * d->W;
  z[0] = d->yhat[p];
#pragma unroll
  for (int q = 1; q < CC_MAX_L; ++q) z[q] = q < d->L ? d->U[d->uoff[1] + (size_t)(q - 1) * n + p] : 0.0f;
}

// Squared error of one pixel, its gradient into dXa and the per-workgroup
// FP64 partial sum.
__device__ __forceinline__ void mse_epilogue(const CDesc* d, int p, bool valid,
                                             const float* xo, int wgi, double* sh) {
  const int n = d->H * d->W;
  double sq = 0.0;
  if (valid) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = xo[c] - d->img[(size_t)c * n + p];
      d->dXa[(size_t)c * n + p] = d->mse_scale * e;
      sq += (double)e * (double)e;
    }
  }
  sq = wave_sum_d(sq);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wv] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < CC_PIX_TILE / 64; ++w) s += sh[w];
    d->lp_mse[wgi] = s;
  }
}

// Trunk weights staged in LDS with fixed strides, so that every read is a
// uniform-address (broadcast) vector load and no loop depends on the runtime L.
//   layer-1 record a (12 floats): W1[a][0..7] (zero beyond L), b1[a], and for a
//     one-hidden-layer trunk the output column Wo[0..2][a];
//   layer-2 record b (two hidden layers): W2[b][0..W1-1], b2[b], Wo[0..2][b];
//   tail: Ws[c][0..7] (stabilizer, zero beyond L or without stabilizer), then
//     the output bias bo[c] (+ bs[c] with a stabilizer).
template <int NH, int W1, int W2>
struct SynLds {
  static constexpr int R1 = 12;
  static constexpr int R2 = NH == 2 ? ((W1 + 4 + 3) & ~3) : 0;
  static constexpr int N1 = W1 * R1;
  static constexpr int N2 = NH == 2 ? W2 * R2 : 0;
  static constexpr int TAIL = N1 + N2;
  static constexpr int TOTAL = TAIL + 28;
};

template <int NH, int W1, int W2>
__device__ void stage_syn_weights(const CDesc* d, const CF* P, float* w) {
  using S = SynLds<NH, W1, W2>;
  const int L = d->L;
  for (int i = threadIdx.x; i < S::TOTAL; i += blockDim.x) {
    float v = 0.0f;
    if (i < S::N1) {
      const int a = i / S::R1, e = i % S::R1;
      if (e < 8)
        v = e < L ? P[d->p_sw[0] + a * L + e] : 0.0f;
      else if (e == 8)
        v = P[d->p_sb[0] + a];
      else if (NH == 1)
        v = P[d->p_sw[1] + (e - 9) * W1 + a];
    } else if (NH == 2 && i < S::TAIL) {
      constexpr int R2 = S::R2 > 0 ? S::R2 : 1;   // (no layer-2 records with one hidden layer)
      const int r = i - S::N1, b = r / R2, e = r % R2;
      if (e < W1)
        v = P[d->p_sw[1] + b * W1 + e];
      else if (e == W1)
        v = P[d->p_sb[1] + b];
      else if (e <= W1 + 3)
        v = P[d->p_sw[2] + (e - W1 - 1) * W2 + b];
    } else {
      const int e = i - S::TAIL;
      if (e < 24) {
        const int c = e >> 3, q = e & 7;
        v = (d->syn_stab && q < L) ? P[d->p_ssw + c * L + q] : 0.0f;
      } else if (e < 27) {
        const int c = e - 24;
        v = P[d->p_sb[NH] + c] + (d->syn_stab ? P[d->p_ssb + c] : 0.0f);
      }
    }
    w[i] = v;
  }
}

// zhat at pixel p: channel 0 = yhat^(0), channels 1..L-1 = U_1; zero beyond L
// and for p outside the image.
__device__ __forceinline__ void load_z8(const CDesc* d, int p, bool valid, float* z) {
  const int n = d->H * d->W;
  z[0] = valid ? d->yhat[p] : 0.0f;
#pragma unroll
  for (int q = 1; q < 8; ++q)
    z[q] = (valid && q < d->L) ? d->U[d->uoff[1] + (size_t)(q - 1) * n + p] : 0.0f;
}

template <int NH, int W1, int W2>
__global__ __launch_bounds__(CC_PIX_TILE) void k_syn_fwd(Launch Lc, int final_mse) {
  using S = SynLds<NH, W1, W2>;
  __shared__ __align__(16) float w[S::TOTAL];
  __shared__ double sh[CC_PIX_TILE / 64];
  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wgi = blockIdx.x - Lc.tile0[im];
  const int n = d->H * d->W;
  const int p = wgi * CC_PIX_TILE + threadIdx.x;
  const bool valid = p < n;
  stage_syn_weights<NH, W1, W2>(d, (const CF*)(d->theta + d->n_lat), w);
  float z[8];
  load_z8(d, p, valid, z);
  __syncthreads();
  const float4* w4 = (const float4*)w;
  float out[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float4 a = w4[(S::TAIL >> 2) + 2 * c], b = w4[(S::TAIL >> 2) + 2 * c + 1];
    out[c] = w[S::TAIL + 24 + c] + a.x * z[0] + a.y * z[1] + a.z * z[2] + a.w * z[3] + b.x * z[4] +
             b.y * z[5] + b.z * z[6] + b.w * z[7];
  }
  if constexpr (NH == 1) {
#pragma unroll 4
    for (int a = 0; a < W1; ++a) {
      const float4 r0 = w4[3 * a], r1 = w4[3 * a + 1], r2 = w4[3 * a + 2];
      float s = r2.x + r0.x * z[0] + r0.y * z[1] + r0.z * z[2] + r0.w * z[3] + r1.x * z[4] +
                r1.y * z[5] + r1.z * z[6] + r1.w * z[7];
      s = fmaxf(s, 0.0f);
      out[0] += r2.y * s;
      out[1] += r2.z * s;
      out[2] += r2.w * s;
    }
  } else {
    float h1[W1];
#pragma unroll
    for (int a = 0; a < W1; ++a) {
      const float4 r0 = w4[3 * a], r1 = w4[3 * a + 1], r2 = w4[3 * a + 2];
      const float s = r2.x + r0.x * z[0] + r0.y * z[1] + r0.z * z[2] + r0.w * z[3] + r1.x * z[4] +
                      r1.y * z[5] + r1.z * z[6] + r1.w * z[7];
      h1[a] = fmaxf(s, 0.0f);
    }
#pragma unroll 2
    for (int b = 0; b < W2; ++b) {
      const float* r = w + S::N1 + b * S::R2;
      float s = r[W1];
#pragma unroll
      for (int a = 0; a < W1; ++a) s += r[a] * h1[a];
      s = fmaxf(s, 0.0f);
      out[0] += r[W1 + 1] * s;
      out[1] += r[W1 + 2] * s;
      out[2] += r[W1 + 3] * s;
    }
  }
  if (valid) {
#pragma unroll
    for (int c = 0; c < 3; ++c) d->X[(size_t)c * n + p] = out[c];
  }
  if (final_mse) mse_epilogue(d, p, valid, out, wgi, sh);
}

// Backward of a one-hidden-layer trunk.  The NWV waves of a workgroup take
// the same 64 pixels and 1/NWV of the hidden units each: a wave recomputes
// its units' pre-activations, back-propagates the output gradient through
// them, accumulates its units' weight gradients in registers (one partial
// per lane, summed over the workgroup's chunks) and leaves its share of dzhat
// in LDS, where the NWV shares are added in a fixed order.  The per-lane
// partials are reduced once at the end (LDS transpose, then a fixed
// butterfly), giving one partial row per workgroup.  Eight waves halve the
// accumulators per wave, so four waves fit on a SIMD instead of two.
template <int W1, int NWV>
__global__ __launch_bounds__(NWV * 64, 2) void k_syn_bwd1(Launch Lc, int src_b) {
  static_assert(NWV == 4 || NWV == 8, "four or eight waves");
  using S = SynLds<1, W1, 0>;
  constexpr int UPW = (W1 + NWV - 1) / NWV;   // hidden units per wave
  constexpr int QPW = 8 / NWV;                // dzhat channels per wave
  constexpr int NF = (11 + NWV - 1) / NWV;    // chunk features loaded per wave
  constexpr int NU = UPW * 12;           // unit accumulators: dW1 row (8), db1, dWo column (3)
  constexpr int NACC = NU + 3 * QPW + 3;  // + stabilizer dWs[c][q] for the wave's q's, output bias
  constexpr int RS = 16 * 65;            // reduction region per wave
  constexpr int NRED = 2 * NWV * 8 * 64 > NWV * RS ? 2 * NWV * 8 * 64 : NWV * RS;
  __shared__ __align__(16) float w[S::TOTAL];
  __shared__ __align__(16) float zb[2][64][12];      // per lane: z[0..7], go[0..2]
  __shared__ __align__(16) float red[NRED];          // dz shares [2][NWV][8][64], then reduction
  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wg = blockIdx.x - Lc.tile0[im];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = d->H * d->W, L = d->L;
  const int nchunk = d->syn_nchunk, nwg = d->syn_nwg;
  const float* G = src_b ? d->dXb : d->dXa;
  stage_syn_weights<1, W1, 0>(d, (const CF*)(d->theta + d->n_lat), w);

  // feature f of a chunk (f = wv + NWV j): 0 yhat, 1..7 U planes (zero
  // beyond L), 8..10 output-gradient planes
  float pre[NF];
  auto load_chunk = [&](int ch) {
    const int p = ch * CC_SYN_CHUNK + lane;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int f = wv + NWV * j;
      float v = 0.0f;
      if (p < n) {
        if (f == 0)
          v = d->yhat[p];
        else if (f < 8) {
          if (f < L) v = d->U[d->uoff[1] + (size_t)(f - 1) * n + p];
        } else if (f < 11)
          v = G[(size_t)(f - 8) * n + p];
      }
      pre[j] = v;
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int f = wv + NWV * j;
      if (f < 11) zb[buf][lane][f] = pre[j];
    }
  };

  float acc[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = 0.0f;
  const float4* w4 = (const float4*)w;
  int buf = 0;
  if (wg < nchunk) {
    load_chunk(wg);
    store_chunk(0);
  }
  __syncthreads();
  for (int ch = wg; ch < nchunk; ch += nwg, buf ^= 1) {
    const int nxt = ch + nwg;
    if (nxt < nchunk) load_chunk(nxt);
    const float4 za = *(const float4*)&zb[buf][lane][0], zc = *(const float4*)&zb[buf][lane][4],
                 gg = *(const float4*)&zb[buf][lane][8];
    const float z[8] = {za.x, za.y, za.z, za.w, zc.x, zc.y, zc.z, zc.w};
    const float go[3] = {gg.x, gg.y, gg.z};
    float dz[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) dz[q] = 0.0f;
#pragma unroll
    for (int u = 0; u < UPW; ++u) {
      const int a = wv * UPW + u;
      if (UPW * NWV != W1 && a >= W1) continue;
      const float4 r0 = w4[3 * a], r1 = w4[3 * a + 1], r2 = w4[3 * a + 2];
      const float wr[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
      float s = r2.x;
#pragma unroll
      for (int q = 0; q < 8; ++q) s += wr[q] * z[q];
      const float h = fmaxf(s, 0.0f);
      const float dh = s > 0.0f ? r2.y * go[0] + r2.z * go[1] + r2.w * go[2] : 0.0f;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        dz[q] += wr[q] * dh;
        acc[12 * u + q] += dh * z[q];
      }
      acc[12 * u + 8] += dh;
      acc[12 * u + 9] += go[0] * h;
      acc[12 * u + 10] += go[1] * h;
      acc[12 * u + 11] += go[2] * h;
    }
    float* dzs = red + buf * (NWV * 8 * 64);
#pragma unroll
    for (int q = 0; q < 8; ++q) dzs[(wv * 8 + q) * 64 + lane] = dz[q];
    if (nxt < nchunk) store_chunk(buf ^ 1);
    __syncthreads();
    // dzhat channels q = wv + NWV qi: the NWV shares in wave order, plus the
    // stabilizer's term
    const int p = ch * CC_SYN_CHUNK + lane;
#pragma unroll
    for (int qi = 0; qi < QPW; ++qi) {
      const int q = wv + NWV * qi;
      if (q >= L) continue;
      float v = dzs[(0 * 8 + q) * 64 + lane];
#pragma unroll
      for (int sw = 1; sw < NWV; ++sw) v += dzs[(sw * 8 + q) * 64 + lane];
      v += w[S::TAIL + q] * go[0] + w[S::TAIL + 8 + q] * go[1] + w[S::TAIL + 16 + q] * go[2];
      if (p < n) {
        if (q == 0)
          d->dyq[p] = v;
        else
          d->dU[d->uoff[1] + (size_t)(q - 1) * n + p] = v;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[NU + 3 * qi + c] += go[c] * z[q];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[NU + 3 * QPW + c] += go[c];
  }

  // per-lane partials -> one value per parameter, in a fixed order
  __syncthreads();
  const long long g_off = d->prod[d->prod_syn].off;
  const int base = d->p_sw[0];
  float* outrow = d->wp + g_off + (size_t)wg * d->prod[d->prod_syn].pcnt;
  float* rw = red + wv * RS;
#pragma unroll
  for (int r0 = 0; r0 < NACC; r0 += 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (r0 + k < NACC) rw[k * 65 + lane] = acc[r0 + k];
    __syncthreads();
    const int pk = lane >> 2, qr = lane & 3;
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) v += rw[pk * 65 + qr * 16 + i];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    const int k = r0 + pk;
    if (qr == 0 && k < NACC) {
      int dst = -1, dst2 = -1;
      if (k < NU) {
        const int u = k / 12, e = k % 12, a = wv * UPW + u;
        if (a < W1) {
          if (e < 8)
            dst = e < L ? d->p_sw[0] + a * L + e : -1;
          else if (e == 8)
            dst = d->p_sb[0] + a;
          else
            dst = d->p_sw[1] + (e - 9) * W1 + a;
        }
      } else if (k < NU + 3 * QPW) {
        const int x = k - NU, q = wv + NWV * (x / 3), c = x % 3;
        if (d->syn_stab && q < L) dst = d->p_ssw + c * L + q;
      } else if (wv == 0) {
        const int c = k - NU - 3 * QPW;
        dst = d->p_sb[1] + c;
        if (d->syn_stab) dst2 = d->p_ssb + c;
      }
      if (dst >= 0) outrow[dst - base] = v;
      if (dst2 >= 0) outrow[dst2 - base] = v;
    }
    __syncthreads();
  }
}

// Backward of the trunk for one pixel per thread (recomputing the hidden
// activations from zhat); the weight gradient is reduced through LDS into one
// partial row per workgroup (one wavefront, chunks of 64 pixels).
template <int NH, int W1, int W2>
__global__ __launch_bounds__(64) void k_syn_bwd(Launch Lc, int src_b) {
  constexpr int WL = SynShape<NH, W1, W2>::WL;
  constexpr int HW2 = NH == 2 ? W2 : 0;
  constexpr int O_Z = 0, O_H1 = CC_MAX_L, O_H2 = O_H1 + W1, O_DH1 = O_H2 + HW2,
                O_DH2 = O_DH1 + W1, O_DO = O_DH2 + HW2, O_ONE = O_DO + 3;
  constexpr int AST = (O_ONE + 1) | 1;
  constexpr int PMAX = (CC_MAX_L + 1) * W1 + (W1 + 1) * HW2 + (WL + 1) * 3 + (CC_MAX_L + 1) * 3;
  constexpr int NQ = (PMAX + 63) / 64;
  __shared__ float lds[64 * AST];
  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wg = blockIdx.x - Lc.tile0[im];
  const int lane = threadIdx.x;
  const int n = d->H * d->W, L = d->L;
  const CF* P0 = (const CF*)(d->theta + d->n_lat);
  const float* G = src_b ? d->dXb : d->dXa;
  const int npar = d->prod[d->prod_syn].pcnt;
  float acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0f;
  for (int ch = wg; ch < d->syn_nchunk; ch += d->syn_nwg) {
    // re-read the weights per chunk (see the ARM kernel)
    const CF* P = P0;
    asm volatile("" : "+s"(P));
    const CF* Wa = P + d->p_sw[0];
    const CF* Wb = P + d->p_sw[1];
    const CF* Wc = P + d->p_sw[NH];
    const CF* Ws = P + d->p_ssw;
    const int p = ch * 64 + lane;
    const bool valid = p < n;
    float z[CC_MAX_L], h1[W1], h2[NH == 2 ? W2 : 1], out[3];
    float go[3] = {0.0f, 0.0f, 0.0f};
    if (valid) {
      load_z(d, p, z);
#pragma unroll
      for (int c = 0; c < 3; ++c) go[c] = G[(size_t)c * n + p];
    } else {
#pragma unroll
      for (int q = 0; q < CC_MAX_L; ++q) z[q] = 0.0f;
    }
    syn_mlp<NH, W1, W2>(d, P, z, h1, h2, out);
    const float* hl = NH == 2 ? h2 : h1;
    float dhl[WL], dh1[W1];
#pragma unroll
    for (int a = 0; a < WL; ++a) {
      const float s = Wc[a] * go[0] + Wc[WL + a] * go[1] + Wc[2 * WL + a] * go[2];
      dhl[a] = hl[a] > 0.0f ? s : 0.0f;
    }
    if constexpr (NH == 2) {
#pragma unroll
      for (int b = 0; b < W1; ++b) {
        float s = 0.0f;
#pragma unroll
        for (int a = 0; a < W2; ++a) s += Wb[a * W1 + b] * dhl[a];
        dh1[b] = h1[b] > 0.0f ? s : 0.0f;
      }
    } else {
#pragma unroll
      for (int b = 0; b < W1; ++b) dh1[b] = dhl[b];
    }
    float* row = lds + lane * AST;
#pragma unroll
    for (int q = 0; q < CC_MAX_L; ++q) {
      float s = 0.0f;
#pragma unroll
      for (int b = 0; b < W1; ++b)
        if (q < L) s += Wa[b * L + q] * dh1[b];
      if (d->syn_stab && q < L) s += Ws[q] * go[0] + Ws[L + q] * go[1] + Ws[2 * L + q] * go[2];
      if (valid && q < L) {
        if (q == 0)
          d->dyq[p] = s;
        else
          d->dU[d->uoff[1] + (size_t)(q - 1) * n + p] = s;
      }
      row[O_Z + q] = z[q];
    }
#pragma unroll
    for (int a = 0; a < W1; ++a) {
      row[O_H1 + a] = h1[a];
      row[O_DH1 + a] = dh1[a];
    }
    if constexpr (NH == 2) {
#pragma unroll
      for (int a = 0; a < W2; ++a) {
        row[O_H2 + a] = h2[a];
        row[O_DH2 + a] = dhl[a];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) row[O_DO + c] = go[c];
    row[O_ONE] = 1.0f;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int pq = lane + 64 * q;
      const unsigned e = pq < npar ? d->syn_gtab[pq] : 0xFFFFFFFFu;
      if (e == 0xFFFFFFFFu) continue;
      const int ia = e & 0xFF, ib = (e >> 8) & 0xFF;
      float s = 0.0f;
      for (int pos = 0; pos < 64; ++pos) s += lds[pos * AST + ia] * lds[pos * AST + ib];
      acc[q] += s;
    }
    __syncthreads();
  }
  const long long g_off = d->prod[d->prod_syn].off;
  float* out = d->wp + g_off + (size_t)wg * npar;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = lane + 64 * q;
    if (p < npar) out[p] = acc[q];
  }
}

// ------------------------------------------------------ residual layers ----
// X_{r+1} = X_r + b + Conv3x3(X_r), replicate padding; on the last layer
// also the MSE epilogue.
__global__ __launch_bounds__(CC_PIX_TILE) void k_res_fwd(Launch Lc, int r, int last_mse) {
  __shared__ double sh[CC_PIX_TILE / 64];
  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wgi = cc_xcd_index(Lc, im);
  const int H = d->H, W = d->W, n = H * W;
  const int p = wgi * CC_PIX_TILE + threadIdx.x;
  const bool valid = p < n;
  const CF* Wr = (const CF*)(d->theta + d->n_lat + d->p_rw[r]);
  const CF* Br = (const CF*)(d->theta + d->n_lat + d->p_rb[r]);
  const float* X = d->X + (size_t)r * 3 * n;
  float out[3] = {0.0f, 0.0f, 0.0f};
  if (valid) {
    const int y = p / W, x = p - y * W;
    float nb[3][9];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      const int yy = clampi(y + ky - 1, 0, H - 1);
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int xx = clampi(x + kx - 1, 0, W - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) nb[c][ky * 3 + kx] = X[(size_t)c * n + yy * W + xx];
      }
    }
#pragma unroll
    for (int co = 0; co < 3; ++co) {
      float s = Br[co];
#pragma unroll
      for (int ci = 0; ci < 3; ++ci)
#pragma unroll
        for (int t = 0; t < 9; ++t) s += Wr[(co * 3 + ci) * 9 + t] * nb[ci][t];
      out[co] = nb[co][4] + s;
      d->X[(size_t)(r + 1) * 3 * n + (size_t)co * n + p] = out[co];
    }
  }
  if (last_mse) mse_epilogue(d, p, valid, out, wgi, sh);
}

// Source positions p along one axis with clamp(p + o) == q, o in {-1, 0, 1}.
__device__ __forceinline__ int srcs(int q, int o, int n, int* ps) {
  int c = 0;
  const int p = q - o;
  if (p >= 0 && p < n) ps[c++] = p;
  if (o == -1 && q == 0) ps[c++] = 0;
  if (o == 1 && q == n - 1) ps[c++] = n - 1;
  return c;
}

// dX_r = dX_{r+1} + Conv3x3^T(dX_{r+1}) (adjoint of the replicate padding
// included), plus the layer's weight gradient as one partial row of 84 per
// workgroup.  A workgroup takes RES_TH x RES_TW tiles (stride: the number of
// workgroups); each tile stages X_r with a replicate-clamped halo and the
// incoming gradient with a zero halo in LDS.  In the image interior the
// adjoint is the plain correlation with the flipped kernel; on the image
// border the sources of every tap are enumerated per axis (srcs), which adds
// the clamped reads' contributions.  Weight-gradient partials stay in
// registers per lane and are reduced once, in a fixed order.
// src_b selects the input buffer; the output goes to the other.
// Two groups of four waves take every pixel of the tile: group 0 owns the
// weight-gradient entries [0, RG) and the input channel 0 of the adjoint,
// group 1 the entries [RG, 84) and the input channels 1, 2, which halves the
// per-lane accumulators (four waves per SIMD instead of two); the layer's
// weights are read through scalar loads.  A lane of either group sees the
// pixels a lane of a four-wave workgroup would.
constexpr int RG = 48;   // weight-gradient entries of group 0

template <int Q0, int NQ, int C0, int NC>
__device__ __forceinline__ void res_bwd_pixel(const float (*xs)[CC_RES_TH + 2][CC_RES_TW + 2],
                                              const float (*gs)[CC_RES_TH + 2][CC_RES_TW + 2],
                                              const CF* Wr, float* acc, int ly, int lx,
                                              int y, int x, int H, int W, int ty0, int tx0,
                                              float* O, int n) {
  float g[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) g[c] = gs[c][ly + 1][lx + 1];
  // weight gradient: g[co] * X_r[ci] at the tap's clamped position (entry
  // q = (co 3 + ci) 9 + t), and the bias g[co] (entry 81 + co)
#pragma unroll
  for (int q = Q0; q < Q0 + NQ; ++q) {
    if (q < 81) {
      const int co = q / 27, ci = (q / 9) % 3, t = q % 9;
      acc[q - Q0] += g[co] * xs[ci][ly + t / 3][lx + t % 3];
    } else {
      acc[q - Q0] += g[q - 81];
    }
  }
  // adjoint, input channels C0 .. C0 + NC - 1 (not interleaved with the
  // weight-gradient loop: that would hold both loops' LDS values at once)
  __builtin_amdgcn_sched_barrier(0);
  float o[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) o[c] = g[C0 + c];
  if (y > 0 && y < H - 1 && x > 0 && x < W - 1) {
#pragma unroll
    for (int co = 0; co < 3; ++co)
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const float gv = gs[co][ly + 2 - t / 3][lx + 2 - t % 3];
#pragma unroll
        for (int c = 0; c < NC; ++c) o[c] += Wr[(co * 3 + C0 + c) * 9 + t] * gv;
      }
  } else {
    for (int ky = 0; ky < 3; ++ky) {
      int py[2];
      const int cy = srcs(y, ky - 1, H, py);
      for (int kx = 0; kx < 3; ++kx) {
        int px[2];
        const int cx = srcs(x, kx - 1, W, px);
        const int t = ky * 3 + kx;
        for (int a2 = 0; a2 < cy; ++a2)
          for (int b2 = 0; b2 < cx; ++b2) {
            const int sy = py[a2] - ty0 + 1, sx = px[b2] - tx0 + 1;
#pragma unroll
            for (int co = 0; co < 3; ++co) {
              const float gv = gs[co][sy][sx];
#pragma unroll
              for (int c = 0; c < NC; ++c) o[c] += Wr[(co * 3 + C0 + c) * 9 + t] * gv;
            }
          }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) O[(size_t)(C0 + c) * n + y * W + x] = o[c];
}

__global__ __launch_bounds__(512, 4) void k_res_bwd(Launch Lc, int r, int src_b) {
  constexpr int TH = CC_RES_TH, TW = CC_RES_TW, SH = TH + 2, SW = TW + 2;
  constexpr int NT = 512;
  __shared__ float xs[3][SH][SW];
  __shared__ float gs[3][SH][SW];
  __shared__ float red[8 * 16 * 65];
  __shared__ float wsum[8][RG];
  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wgi = cc_xcd_index(Lc, im);
  const int nwg = d->res_nwg;
  const int H = d->H, W = d->W, n = H * W;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wv >> 2, wq = wv & 3;   // group, wave within the group
  const CF* Wr = (const CF*)(d->theta + d->n_lat + d->p_rw[r]);
  const float* G = src_b ? d->dXb : d->dXa;
  float* O = src_b ? d->dXa : d->dXb;
  const float* X = d->X + (size_t)r * 3 * n;
  float acc[RG];
#pragma unroll
  for (int q = 0; q < RG; ++q) acc[q] = 0.0f;
  const int ntx = (W + TW - 1) / TW, nty = (H + TH - 1) / TH;
  for (int tile = wgi; tile < ntx * nty; tile += nwg) {
    const int ty0 = (tile / ntx) * TH, tx0 = (tile % ntx) * TW;
    // stage X_r (replicate-clamped halo) and the incoming gradient (zero
    // halo): every load of the thread is issued before the first LDS store,
    // so their latencies overlap
    constexpr int NST = (SH * SW + NT - 1) / NT;
    float xv[NST][3], gv[NST][3];
#pragma unroll
    for (int u = 0; u < NST; ++u) {
      const int i = tid + NT * u;
      const int ly = i / SW, lx = i - ly * SW;
      const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
      const int cy = clampi(gy, 0, H - 1), cx = clampi(gx, 0, W - 1);
      const bool in = i < SH * SW && gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xv[u][c] = i < SH * SW ? X[(size_t)c * n + cy * W + cx] : 0.0f;
        gv[u][c] = in ? G[(size_t)c * n + gy * W + gx] : 0.0f;
      }
    }
    __syncthreads();   // previous tile's reads are done
#pragma unroll
    for (int u = 0; u < NST; ++u) {
      const int i = tid + NT * u;
      if (i < SH * SW) {
        const int ly = i / SW, lx = i - ly * SW;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xs[c][ly][lx] = xv[u][c];
          gs[c][ly][lx] = gv[u][c];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TH / 4; ++k) {
      const int ly = wq + 4 * k, lx = lane;
      const int y = ty0 + ly, x = tx0 + lx;
      if (y >= H || x >= W) continue;
      if (grp == 0)
        res_bwd_pixel<0, RG, 0, 1>(xs, gs, Wr, acc, ly, lx, y, x, H, W, ty0, tx0, O, n);
      else
        res_bwd_pixel<RG, 84 - RG, 1, 2>(xs, gs, Wr, acc, ly, lx, y, x, H, W, ty0, tx0, O, n);
    }
  }
  // per-lane partials -> per-wave sums (LDS transpose, fixed butterfly) ->
  // the group's sum in wave order
  __syncthreads();
  float* rw = red + wv * (16 * 65);
  const int nq = grp == 0 ? RG : 84 - RG;
#pragma unroll
  for (int r0 = 0; r0 < RG; r0 += 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (r0 + k < RG) rw[k * 65 + lane] = acc[r0 + k];
    __syncthreads();
    const int pk = lane >> 2, qr = lane & 3;
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) v += rw[pk * 65 + qr * 16 + i];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    __syncthreads();
    if (qr == 0 && r0 + pk < nq) wsum[wv][r0 + pk] = v;
  }
  __syncthreads();
  if (tid < 84) {
    const int g2 = tid < RG ? 0 : 4, q = tid < RG ? tid : tid - RG;
    const long long pg_off = d->prod[d->prod_res0 + r].off;
    d->wp[pg_off + (size_t)wgi * 84 + tid] =
        wsum[g2][q] + wsum[g2 + 1][q] + wsum[g2 + 2][q] + wsum[g2 + 3][q];
  }
}

inline int ok() { return hipGetLastError() == hipSuccess ? CC_OK : CC_EDEVICE; }

}  // namespace

#define CC_SYN_SHAPES(X) \
  X(2, 24, 24)           \
  X(1, 40, 0)            \
  X(1, 6, 0)             \
  X(1, 8, 0)             \
  X(1, 16, 0)            \
  X(1, 48, 0)            \
  X(1, 64, 0)

int cc_syn_shape_supported(int nh, int w1, int w2) {
#define X(a, b, c) if (nh == a && w1 == b && (a == 1 || w2 == c)) return 1;
  CC_SYN_SHAPES(X)
#undef X
  return 0;
}

int cc_launch_syn_fwd_plain(const Launch& l, const DevDesc& h, int final_mse, hipStream_t st) {
  const int w2 = h.n_syn_hidden == 2 ? h.syn_w[2] : 0;
#define X(a, b, c)                                                                             \
  if (h.n_syn_hidden == a && h.syn_w[1] == b && w2 == c) {                                     \
    hipLaunchKernelGGL((k_syn_fwd<a, b, c>), dim3(l.tile0[l.n]), dim3(CC_PIX_TILE), 0, st, l, \
                       final_mse);                                                             \
    return ok();                                                                               \
  }
  CC_SYN_SHAPES(X)
#undef X
  return CC_EINVAL;
}

int cc_launch_syn_bwd_plain(const Launch& l, const DevDesc& h, int src_b, hipStream_t st) {
  const int w2 = h.n_syn_hidden == 2 ? h.syn_w[2] : 0;
#define X(a, b, c)                                                                           \
  if (h.n_syn_hidden == a && h.syn_w[1] == b && w2 == c) {                                   \
    if constexpr (a == 1)                                                                    \
      hipLaunchKernelGGL((k_syn_bwd1<b, CC_SYN_BWD_WAVES>), dim3(l.tile0[l.n]),               \
                         dim3(CC_SYN_BWD_WAVES * 64), 0, st, l, src_b);                        \
    else                                                                                     \
      hipLaunchKernelGGL((k_syn_bwd<a, b, c>), dim3(l.tile0[l.n]), dim3(64), 0, st, l, src_b); \
    return ok();                                                                             \
  }
  CC_SYN_SHAPES(X)
#undef X
  return CC_EINVAL;
}

int cc_launch_ups_fwd(const Launch& l, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_ups_fwd, dim3(l.tile0[l.n]), dim3(CC_PIX_TILE), 0, st, l, j);
  return ok();
}
int cc_launch_upc_fwd(const Launch& l, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_upc_fwd, dim3(l.tile0[l.n]), dim3(256), 0, st, l, j);
  return ok();
}
int cc_launch_upc_bwd(const Launch& l, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_upc_bwd, dim3(l.tile0[l.n]), dim3(256), 0, st, l, j);
  return ok();
}
int cc_launch_ups_bwd(const Launch& l, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_ups_bwd, dim3(l.tile0[l.n]), dim3(256), 0, st, l, j);
  return ok();
}
int cc_launch_ups_fwd_chain(const Launch& l, hipStream_t st) {
  hipLaunchKernelGGL(k_ups_fwd_chain, dim3(l.tile0[l.n]), dim3(CT), 0, st, l);
  return ok();
}
int cc_launch_ups_bwd_chain(const Launch& l, hipStream_t st) {
  hipLaunchKernelGGL(k_ups_bwd_chain, dim3(l.tile0[l.n]), dim3(CT), 0, st, l);
  return ok();
}
int cc_launch_res_fwd(const Launch& l, int r, int last, int want_mse, hipStream_t st) {
  hipLaunchKernelGGL(k_res_fwd, dim3(l.tile0[l.n]), dim3(CC_PIX_TILE), 0, st, l, r,
                     (last && want_mse) ? 1 : 0);
  return ok();
}
int cc_launch_res_bwd2(const Launch& l, int r, int src_b, hipStream_t st) {
  hipLaunchKernelGGL(k_res_bwd, dim3(l.tile0[l.n]), dim3(512), 0, st, l, r, src_b);
  return ok();
}
