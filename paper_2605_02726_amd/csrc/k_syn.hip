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
// with the parity of o + 3.  zhat = [yhat^(0); U_1].
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
  const int p = (blockIdx.x - L.tile0[im]) * CC_PIX_TILE + threadIdx.x;
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
    const float* in = tchan(d, j, ch);
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
// dU_{j+1}.  One partial row of 4 tap gradients per workgroup.
constexpr int UT = CC_UPS_TILE;   // input tile side
constexpr int UG = 2 * UT + 6;   // output window side (2*UT + 3 + 3)
constexpr int UTW = UT + 4;      // input window side (2 each side)

__global__ __launch_bounds__(256) void k_ups_bwd(Launch L, int j) {
  __shared__ float g[UG][UG + 1];
  __shared__ float t[UTW][UTW + 1];
  __shared__ float R[UG][UT + 1];
  __shared__ float Bm[UT][2 * UT + 1];
  __shared__ float wxs[UT][8], wys[UT][8];
  __shared__ float sh[4][4];
  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int wgi = blockIdx.x - L.tile0[im];
  const int ho = d->gh[j - 1], wo = d->gw[j - 1], hi = d->gh[j], wi = d->gw[j];
  const int ntx = (wi + UT - 1) / UT;
  const int iy0 = (wgi / ntx) * UT, ix0 = (wgi % ntx) * UT;
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
  const int nch = d->L - j;
  float dh[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int ch = 0; ch < nch; ++ch) {
    const float* gsrc = d->dU + d->uoff[j] + (size_t)ch * ho * wo;
    const float* tsrc = tchan(d, j, ch);
    __syncthreads();
    for (int i = tid; i < UG * UG; i += 256) {
      const int r = i / UG, c = i - r * UG;
      const int oy = 2 * iy0 - 3 + r, ox = 2 * ix0 - 3 + c;
      g[r][c] = (oy >= 0 && oy < ho && ox >= 0 && ox < wo) ? gsrc[oy * wo + ox] : 0.0f;
    }
    for (int i = tid; i < UTW * UTW; i += 256) {
      const int r = i / UTW, c = i - r * UTW;
      t[r][c] = tsrc[clampi(iy0 - 2 + r, 0, hi - 1) * wi + clampi(ix0 - 2 + c, 0, wi - 1)];
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
    {
      const int q = tid / UT, p = tid - q * UT;   // 256 = 16 x 16 inputs
      const int iy = iy0 + q, ix = ix0 + p;
      if (iy < hi && ix < wi) {
        float a = 0.0f;
#pragma unroll
        for (int b = 0; b < 8; ++b) a += wys[q][b] * R[2 * q + b][p];
        if (ch == 0)
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

template <int NH, int W1, int W2>
__global__ __launch_bounds__(CC_PIX_TILE) void k_syn_fwd(Launch Lc, int final_mse) {
  __shared__ double sh[CC_PIX_TILE / 64];
  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wgi = blockIdx.x - Lc.tile0[im];
  const int n = d->H * d->W;
  const int p = wgi * CC_PIX_TILE + threadIdx.x;
  const bool valid = p < n;
  const CF* P = (const CF*)(d->theta + d->n_lat);
  float z[CC_MAX_L], h1[W1], h2[NH == 2 ? W2 : 1], out[3];
  if (valid) {
    load_z(d, p, z);
    syn_mlp<NH, W1, W2>(d, P, z, h1, h2, out);
#pragma unroll
    for (int c = 0; c < 3; ++c) d->X[(size_t)c * n + p] = out[c];
  }
  if (final_mse) mse_epilogue(d, p, valid, out, wgi, sh);
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
  const int wgi = blockIdx.x - Lc.tile0[im];
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
// workgroup; each thread handles RES_PPT pixels before the reduction.
// src_b selects the input buffer; the output goes to the other.
__global__ __launch_bounds__(CC_PIX_TILE) void k_res_bwd(Launch Lc, int r, int src_b) {
  __shared__ float sh[84][CC_PIX_TILE / 64];
  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wgi = blockIdx.x - Lc.tile0[im];
  const int H = d->H, W = d->W, n = H * W;
  const CF* Wr = (const CF*)(d->theta + d->n_lat + d->p_rw[r]);
  const float* G = src_b ? d->dXb : d->dXa;
  float* O = src_b ? d->dXa : d->dXb;
  const float* X = d->X + (size_t)r * 3 * n;
  float gw[84];
#pragma unroll
  for (int q = 0; q < 84; ++q) gw[q] = 0.0f;
  for (int k = 0; k < CC_RES_PPT; ++k) {
    const int p = (wgi * CC_RES_PPT + k) * CC_PIX_TILE + threadIdx.x;
    if (p >= n) break;
    const int y = p / W, x = p - y * W;
    float g[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = G[(size_t)c * n + p];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      const int yy = clampi(y + ky - 1, 0, H - 1);
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int xx = clampi(x + kx - 1, 0, W - 1);
#pragma unroll
        for (int ci = 0; ci < 3; ++ci) {
          const float v = X[(size_t)ci * n + yy * W + xx];
#pragma unroll
          for (int co = 0; co < 3; ++co) gw[(co * 3 + ci) * 9 + ky * 3 + kx] += g[co] * v;
        }
      }
    }
#pragma unroll
    for (int co = 0; co < 3; ++co) gw[81 + co] += g[co];
    float acc[3] = {g[0], g[1], g[2]};
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      int py[2];
      const int cy = srcs(y, ky - 1, H, py);
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        int px[2];
        const int cx = srcs(x, kx - 1, W, px);
        for (int a = 0; a < cy; ++a)
          for (int b = 0; b < cx; ++b) {
            const int s2 = py[a] * W + px[b];
#pragma unroll
            for (int co = 0; co < 3; ++co) {
              const float gv = G[(size_t)co * n + s2];
#pragma unroll
              for (int ci = 0; ci < 3; ++ci) acc[ci] += Wr[(co * 3 + ci) * 9 + ky * 3 + kx] * gv;
            }
          }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) O[(size_t)c * n + p] = acc[c];
  }
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 84; ++q) {
    const float s2 = wave_sum(gw[q]);
    if (ln == 0) sh[q][wv] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 84) {
    float s2 = 0.0f;
    for (int w2 = 0; w2 < CC_PIX_TILE / 64; ++w2) s2 += sh[threadIdx.x][w2];
    const long long pg_off = d->prod[d->prod_res0 + r].off;
    d->wp[pg_off + (size_t)wgi * 84 + threadIdx.x] = s2;
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
#define X(a, b, c)                                                                          \
  if (h.n_syn_hidden == a && h.syn_w[1] == b && w2 == c) {                                  \
    hipLaunchKernelGGL((k_syn_bwd<a, b, c>), dim3(l.tile0[l.n]), dim3(64), 0, st, l, src_b); \
    return ok();                                                                            \
  }
  CC_SYN_SHAPES(X)
#undef X
  return CC_EINVAL;
}

int cc_launch_ups_fwd(const Launch& l, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_ups_fwd, dim3(l.tile0[l.n]), dim3(CC_PIX_TILE), 0, st, l, j);
  return ok();
}
int cc_launch_ups_bwd(const Launch& l, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_ups_bwd, dim3(l.tile0[l.n]), dim3(256), 0, st, l, j);
  return ok();
}
int cc_launch_res_fwd(const Launch& l, int r, int last, int want_mse, hipStream_t st) {
  hipLaunchKernelGGL(k_res_fwd, dim3(l.tile0[l.n]), dim3(CC_PIX_TILE), 0, st, l, r,
                     (last && want_mse) ? 1 : 0);
  return ok();
}
int cc_launch_res_bwd2(const Launch& l, int r, int src_b, hipStream_t st) {
  hipLaunchKernelGGL(k_res_bwd, dim3(l.tile0[l.n]), dim3(CC_PIX_TILE), 0, st, l, r, src_b);
  return ok();
}
