// ARM entropy model, fused BF16 MFMA form (gfx950, v_mfma_f32_32x32x16_bf16).
//
// Same mathematics as the plain kernel (Section III-A: causal context,
// inter-feature context, MLP with stabilizer, Laplace rate; and its
// backward), with the three GEMM-shaped parts on the matrix cores:
//   forward   H1 = relu(W1 C + b1), H2 = relu(W2 H1 + b2)
//   backward  dH1 = W2^T dH2', dC = W1^T dH1'
//   weights   dW1 = dH1' C^T, dW2 = dH2' H1^T, dW3/dWs likewise
// with latent positions on the N axis: 32 positions per MFMA, operands in
// split BF16 (hi + lo), accumulation in FP32.  The output layer (2 units),
// the stabilizer, the rate and its derivatives run in FP32 on the vector
// ALUs.  The weight gradients need the positions on the K axis instead: each
// operand is transposed through the matrix cores (a product with a constant
// 0/1 permutation matrix, exact in FP32), so no activation passes through
// LDS, and the weight-gradient products are split BF16 as well.
//
// Work: one workgroup (4 wavefronts) per band of CC_FUSED_BAND rows of one
// grid, swept in segments of 128 columns; wavefront w owns columns
// [32 w, 32 w + 32) of the segment in every row of the band.  The quantised
// latents of the band and its causal halo (4 rows above, 4 columns each
// side) are staged in LDS.  The context
// gradient goes to the neighbours without atomics: a wavefront stages its
// tile's slot gradients in LDS and each lane gathers, for one destination
// column, the slots that reach it (fixed slot order), adding the sums to the
// wavefront's private window over the band rows plus that halo; the
// windows are merged in wavefront order at the end of each segment, so the
// result is deterministic.  Each band writes its own rows to plane 0 and
// the 4 halo rows above it to plane q for the rows of the band q above (two
// planes with 2-row bands, one with 4-row bands).  Weight gradients stay in
// MFMA accumulators across the band and are reduced over the 4 wavefronts
// in a fixed order into one partial row per band.
#include "cc_internal.h"

#include <math.h>

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr float INV_LN2 = 1.4426950408889634f;
constexpr int TH = CC_FUSED_BAND;  // band height (rows)
constexpr int HALO = CC_FUSED_HALO;   // causal reach: rows above, columns each side
constexpr int RP = TH / 2;            // row pairs of a band (IFCE inputs and pooling)
constexpr int NW = 4;              // wavefronts per workgroup
constexpr int SW = 32 * NW;        // segment width
constexpr int WR = SW + 2 * HALO;  // LDS row: segment plus the halo columns
constexpr int PW = 32 + 2 * HALO;  // private accumulator row of one wavefront
constexpr int GP = 32 + 4 * HALO;  // staged slot-gradient row (positions -8 .. 39)

// The first 24 causal neighbours in decoding order (half-plane {dy < 0, or
// dy = 0 and dx < 0} sorted by (dy^2 + dx^2, dy, dx)), as LDS offsets within
// the staged window; every fused shape uses a prefix of this list.  The host
// checks the state's neighbour list against it (cc_arm_fused_supported).
constexpr int NOFF = 24;
constexpr int CDY[NOFF] = {-1, 0, -1, -1, -2, 0, -2, -2, -1, -1, -2, -2,
                           -3, 0, -3, -3, -1, -1, -3, -3, -2, -2, -4, 0};
constexpr int CDX[NOFF] = {0, -1, -1, 1, 0, -2, -1, 1, -2, 2, -2, 2,
                           0, -3, -1, 1, -3, 3, -2, 2, -3, 3, 0, -4};
__host__ __device__ constexpr int coff(int m) { return m < NOFF ? CDY[m] * WR + CDX[m] : 0; }

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Data-path products in split BF16: x = hi + lo for both the weights and the
// activations, accumulating hi*hi + hi*lo + lo*hi (about 16 significant bits
// per product, FP32 accumulation).
__device__ __forceinline__ f32x16 mfma3(bf16x8 wh, bf16x8 wl, bf16x8 bh, bf16x8 bl, f32x16 c) {
  c = mfma(wl, bh, c);
  c = mfma(wh, bl, c);
  return mfma(wh, bh, c);
}

__device__ __forceinline__ void split8(const float* x, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    hi[i] = (__bf16)x[i];
    lo[i] = (__bf16)(x[i] - (float)hi[i]);
  }
}

// Row of the 32x32 output held by accumulator register i of a lane in half h.
__device__ __forceinline__ int mrow(int i, int h) { return (i >> 2) * 8 + 4 * h + (i & 3); }
// Hidden unit carried at K index k when the previous layer's output
// registers are fed back as the B operand: k = 16 s + 8 h + i <-> register
// 8 s + i of half h.
__device__ __forceinline__ int kunit(int k) {
  const int s = k >> 4, h = (k >> 3) & 1, i = k & 7;
  return mrow(8 * s + i, h);
}

__device__ __forceinline__ void laplace_bits(float dd, float ib, float& bits, float& gd, float& gl) {
  const float ad = fabsf(dd);
  if (ad >= 0.5f) {
    const float a = ad - 0.5f;
    bits = a * ib * INV_LN2 - log2f(-0.5f * expm1f(-ib));
    gd = copysignf(ib * INV_LN2, dd);
    gl = (ib / expm1f(ib) - a * ib) * INV_LN2;
  } else {
    // with E1 = exp(-x1), E2 = exp(-x2): p = 1 - (E1 + E2) / 2, and the
    // derivatives need E1 - E2 and E1 x1 + E2 x2; written with E's rather
    // than expm1(-x) = E - 1, whose low bits (where E is small, at small
    // scales b) FP32 cannot hold next to the -1
    const float x1 = (0.5f + dd) * ib, x2 = (0.5f - dd) * ib;
    const float E1 = expf(-x1), E2 = expf(-x2);
    const float h = 0.5f * (E1 + E2);
    const float p = 1.0f - h;
    bits = -log1pf(-h) * INV_LN2;
    const float q = INV_LN2 / p;
    // E1 - E2 = E2 expm1(x2 - x1) (dd >= 0) or -E1 expm1(x1 - x2) (dd < 0)
    const float dE = dd >= 0.0f ? E2 * expm1f(-2.0f * dd * ib) : -E1 * expm1f(2.0f * dd * ib);
    gd = -0.5f * ib * dE * q;
    gl = 0.5f * (E1 * x1 + E2 * x2) * q;
  }
}

// acc += A * B over 32 positions on K (two K-steps), split BF16:
// A_lo B_hi + A_hi B_lo + A_hi B_hi.
__device__ __forceinline__ f32x16 mma_split(const bf16x8* ah, const bf16x8* al, const bf16x8* bh,
                                            const bf16x8* bl, f32x16 acc) {
#pragma unroll
  for (int s = 0; s < 2; ++s) acc = mfma3(ah[s], al[s], bh[s], bl[s], acc);
  return acc;
}

// Transpose of a 32 x 32 block held as a B operand (lane = position, K index
// 16 s + 8 hh + i <-> feature) into the layout of an MFMA output with the
// positions as rows (lane = feature, register i <-> position mrow(i, hh)):
// D = X^T P with P the 0/1 matrix of the K index -> feature map, which an
// FP32 accumulation reproduces exactly.  Registers 8 s .. 8 s + 7 of the
// result, as BF16, are then an A or B operand with the positions on K.
__device__ __forceinline__ void transpose2(const bf16x8* x, const bf16x8* p, bf16x8* out) {
  f32x16 d = {};
  d = mfma(x[0], p[0], d);
  d = mfma(x[1], p[1], d);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 8; ++i) out[s][i] = (__bf16)d[8 * s + i];
}

// Lanes of column n of a transposed operand: all ones (a bias column), or
// zero.
__device__ __forceinline__ void set_column(bf16x8* hi, bf16x8* lo, float v) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      hi[s][i] = (__bf16)v;
      lo[s][i] = (__bf16)0.0f;
    }
}

template <int S, int F, int H1, int H2>
__global__ __launch_bounds__(256, 2) void k_arm_fused(Launch Lc, int bwd) {
  constexpr int CTX = S + F;
  static_assert(CTX + 1 <= 32 && H1 + 2 <= 32 && H2 + 1 <= 32 && CC_MAX_NIN + 1 <= 32, "shape");
  static_assert(TH % 2 == 0 && HALO >= TH, "row pairs; every halo row in a band above");
  // The linear stabilizer rides in the first layer's spare output rows H1,
  // H1 + 1 (and its backward in the same columns of the transposed layer):
  // register IS of half HS holds row H1, register IS + 1 row H1 + 1.
  static_assert((H1 & 3) != 3, "stabilizer rows must share a register group");
  constexpr int IS = (H1 / 8) * 4 + (H1 & 3), HS = (H1 & 7) / 4;
  __shared__ float ywin[HALO + TH][WR];
  // context-gradient accumulators: one private window per wavefront (its 32
  // columns plus HALO on each side, the band rows plus HALO above), merged
  // at the end of each segment; cin / cout carry the columns that spill into
  // the next segment
  __shared__ float pacc[NW][HALO + TH][PW];
  __shared__ float cin[HALO + TH][2 * HALO], cout[HALO + TH][2 * HALO];
  // per-wavefront staging of one tile's slot gradients for the gather:
  // [slot][position + 2 HALO], rows 0-31 the MFMA rows, row 32 the direct term
  __shared__ float gsc[NW][33][GP];
  // end-of-band weight-gradient sums of the three accumulators (the weights
  // are staged through the same storage at the start)
  __shared__ float wsum_raw[3 * 32 * 33];
  float(*wsum)[32][33] = reinterpret_cast<float(*)[32][33]>(wsum_raw);
  static_assert(H1 * CTX + H2 * H1 <= 3 * 32 * 33, "weight staging");
  __shared__ float pwin[RP][CC_MAX_NIN][SW / 2 + 1];   // IFCE inputs of the segment, per row pair
  __shared__ float fwin[RP][8][SW / 2];                 // IFCE features per 2 x 2 block
  __shared__ float dfs[NW][8][32];                  // top-row pair sums of the IFCE gradients
  __shared__ float vec[8][32];      // b1, b2, W3[0], W3[1], Ws[0], Ws[1] by row
  __shared__ float iw[8][CC_MAX_NIN], ib[8];  // IFCE weights [feature][input] (zero padded), biases
  __shared__ double bsh[NW];
  __shared__ bf16x8 wop[4][2][64], wopl[4][2][64];

  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wg = blockIdx.x - Lc.tile0[im];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, n = lane & 31, hh = lane >> 5;
  const CF* P = (const CF*)(d->theta + d->n_lat);
  const CF* W3 = P + d->p_aw[2];
  const bool stab = d->arm_stab != 0;
  const float rs = d->rate_scale;

  // ---- per-workgroup constants (the same for every band)
  if (tid < 32) {
    const int m = tid;
    vec[0][m] = m < H1 ? P[d->p_ab[0] + m] : 0.0f;
    vec[1][m] = m < H2 ? P[d->p_ab[1] + m] : 0.0f;
    vec[2][m] = m < H2 ? W3[m] : 0.0f;
    vec[3][m] = m < H2 ? W3[H2 + m] : 0.0f;
    vec[4][m] = (stab && m < CTX) ? P[d->p_asw + m] : 0.0f;
    vec[5][m] = (stab && m < CTX) ? P[d->p_asw + CTX + m] : 0.0f;
  }
  for (int i = tid; i < NW * 33 * GP; i += NW * 64) (&gsc[0][0][0])[i] = 0.0f;
  // A operands (weights, split BF16) per lane and K step, kept in LDS:
  // operand (matrix mat, step s) of lane l is wop[mat][s][l] (hi) and
  // wopl[mat][s][l] (lo).  W1 and W2 are first staged in FP32 through the
  // (not yet used) tile storage; wavefront mat then builds matrix mat.
  float* w1s = wsum_raw;
  float* w2s = w1s + H1 * CTX;
  for (int i = tid; i < H1 * CTX + H2 * H1; i += NW * 64)
    w1s[i] = i < H1 * CTX ? P[d->p_aw[0] + i] : P[d->p_aw[1] + i - H1 * CTX];
  __syncthreads();
  {
    const int mat = wave;
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      bf16x8 hi, lo;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int kk = 16 * s2 + 8 * hh + i, u = kunit(kk), m = n;
        float v = 0.0f;
        if (mat == 0)
          v = kk >= CTX ? 0.0f
              : m < H1 ? w1s[m * CTX + kk]
              : m < H1 + 2 ? vec[4 + m - H1][kk] : 0.0f;   // stabilizer rows
        else if (mat == 1)
          v = (m < H2 && u < H1) ? w2s[m * H1 + u] : 0.0f;
        else if (mat == 2)
          v = (m < H1 && u < H2) ? w2s[u * H1 + m] : 0.0f;
        else
          v = m >= CTX ? 0.0f
              : u < H1 ? w1s[u * CTX + m]
              : u < H1 + 2 ? vec[4 + u - H1][m] : 0.0f;    // stabilizer columns
        hi[i] = (__bf16)v;
        lo[i] = (__bf16)(v - (float)hi[i]);
      }
      wop[mat][s2][lane] = hi;
      wopl[mat][s2][lane] = lo;
    }
  }
  // 0/1 operands of the transposes: K index 16 s + 8 hh + i -> feature n
  // (the hidden-unit registers carry unit kunit(k); the context and the IFCE
  // inputs carry slot k)
  bf16x8 pu[2], pc[2];
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int kk = 16 * s2 + 8 * hh + i;
      pu[s2][i] = (__bf16)(kunit(kk) == n ? 1.0f : 0.0f);
      pc[s2][i] = (__bf16)(kk == n ? 1.0f : 0.0f);
    }
  const float b30 = P[d->p_ab[2]], b31 = P[d->p_ab[2] + 1];
  const float bs0 = stab ? P[d->p_asb] : 0.0f, bs1 = stab ? P[d->p_asb + 1] : 0.0f;
  // this workgroup's bands (band index: grid 0's bands first, then grid
  // 1's, ...), packed by the host so that the workgroups' loads are even;
  // every band writes its own partial row and bits partial, so the results
  // do not depend on the packing
  const int e0 = __builtin_amdgcn_readfirstlane(d->arm_wbeg[wg]);
  const int e1 = __builtin_amdgcn_readfirstlane(d->arm_wbeg[wg + 1]);
  for (int e = e0; e < e1; ++e) {
  const int bidx = __builtin_amdgcn_readfirstlane(d->arm_blist[e]);
  int k = 0, band = bidx;
  for (;;) {
    const int nb = (d->gh[k] + TH - 1) / TH;
    if (band < nb || k == d->NG - 1) break;
    band -= nb;
    ++k;
  }
  const int h = d->gh[k], w = d->gw[k], nk = h * w;
  const int y0 = band * TH;
  const bool has_ifce = F > 0 && k < d->G;
  const int nin = has_ifce ? d->nin[k] : 0;
  const float* yg = d->yhat + d->goff[k];
  // per-thread indices of the band-level code are recomputed from an opaque
  // copy of the thread index rather than kept in registers across the band
  int tb = threadIdx.x;
  __asm__ volatile("" : "+v"(tb));
  if (tb < 8 * CC_MAX_NIN) {
    const int f = tb / CC_MAX_NIN, q = tb - f * CC_MAX_NIN;
    iw[f][q] = (has_ifce && f < F && q < nin) ? P[d->p_iw[k] + f * nin + q] : 0.0f;
    if (q == 0) ib[f] = (has_ifce && f < F) ? P[d->p_ib[k] + f] : 0.0f;
  }

  // weight-gradient accumulators (rows x columns, positions summed):
  // acc1 = dH1 C^T (+ stabilizer rows H1, H1 + 1; bias column CTX),
  // acc2 = dH2 H1^T (bias column H1), acc3 = the same dH1 rows H1, H1 + 1
  // (d mu, d l) against H2^T: the output layer (bias column H2).  The IFCE
  // weight gradients come from the pooling of the per-position IFCE
  // gradients written below (they multiply the pooled sums by the inputs).
  f32x16 acc1 = {}, acc2 = {}, acc3 = {};
  double bsum = 0.0;
  for (int i = tb; i < NW * (HALO + TH) * PW; i += NW * 64) (&pacc[0][0][0])[i] = 0.0f;
  if (tb < (HALO + TH) * 2 * HALO) (&cin[0][0])[tb] = 0.0f;

  const int nseg = (w + SW - 1) / SW;
  // latent window of a segment: rows y0-4 .. y0+TH-1, columns x0-4 ..
  // x0+SW+3 (zero outside), loaded into registers (every load issued before
  // any use, so their latencies overlap); the next segment's window is
  // loaded while the current one's context gradients are merged
  constexpr int NY = ((HALO + TH) * WR + NW * 64 - 1) / (NW * 64);
  float yv[NY];
  auto load_window = [&](int xs, int t0) {
#pragma unroll
    for (int u = 0; u < NY; ++u) {
      const int i = t0 + NW * 64 * u;
      const int r = i / WR, c = i - r * WR;
      const int gy = y0 - HALO + r, gx = xs - HALO + c;
      yv[u] = (i < (HALO + TH) * WR && gy >= 0 && gy < h && gx >= 0 && gx < w) ? yg[gy * w + gx] : 0.0f;
    }
  };
  // IFCE inputs of the segment: every input grid is coarser (shift >= 1)
  // and y0 is even, so each row pair of the band shares one input row;
  // prefetched into registers with the window
  constexpr int NPW = CC_MAX_NIN * (SW / 2 + 1);
  constexpr int NQ = (RP * NPW + NW * 64 - 1) / (NW * 64);
  float pv[NQ];
  auto load_inputs = [&](int xs, int t0) {
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int i = t0 + NW * 64 * u;
      const int rp = i / NPW, iq = i - rp * NPW;
      const int q = iq / (SW / 2 + 1), c = iq - q * (SW / 2 + 1);
      float v = 0.0f;
      if (rp < RP && q < nin) {
        const int j = d->isrc[k][q], sh = d->ish[k][q];
        const int py = (y0 + 2 * rp) >> sh, px = (xs >> sh) + c;
        if (py < d->gh[j] && px < d->gw[j]) v = d->yhat[d->goff[j] + py * d->gw[j] + px];
      }
      pv[u] = v;
    }
  };
  load_window(0, tb);
  if (has_ifce) load_inputs(0, tb);
  for (int seg = 0; seg < nseg; ++seg) {
    const int x0 = seg * SW;
    int tq = threadIdx.x;   // opaque copy, as for the band-level code
    __asm__ volatile("" : "+v"(tq));
#pragma unroll
    for (int u = 0; u < NY; ++u) {
      const int i = tq + NW * 64 * u;
      if (i < (HALO + TH) * WR) (&ywin[0][0])[i] = yv[u];
    }
    if (has_ifce) {
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const int i = tq + NW * 64 * u;
        if (i < RP * NPW) (&pwin[0][0][0])[i] = pv[u];
      }
      __syncthreads();
      // IFCE features, once per 2 x 2 block (the inputs are constant over
      // each): f = b + W r, inputs in order
      for (int i = tq; i < RP * F * (SW / 2); i += NW * 64) {
        const int rp = i / (F * (SW / 2)), fi = i - rp * (F * (SW / 2));
        const int f = fi / (SW / 2), c2 = fi - f * (SW / 2);
        const int xp = x0 + 2 * c2;
        float a = ib[f];
        for (int q = 0; q < nin; ++q) {
          const int sh = d->ish[k][q];
          a += iw[f][q] * pwin[rp][q][(xp >> sh) - (x0 >> sh)];
        }
        fwin[rp][f][c2] = a;
      }
    }
    __syncthreads();

#pragma unroll 1
    for (int r = 0; r < TH; ++r) {
      const int y = y0 + r, x = x0 + 32 * wave + n;
      // an opaque zero added to the LDS indices of the weights and biases:
      // they are read again every tile instead of being held in registers
      // across the band, which keeps the kernel at two wavefronts per SIMD
      int zq = 0;
      __asm__ volatile("" : "+s"(zq));
      const bool valid = y < h && x < w;
      const int lc = HALO + 32 * wave + n;       // LDS column of this position
      // ---- context (FP32) in operand order: slot kk = 16 s + 8 hh + i
      float cf[2][8];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int kk = 16 * s + 8 * hh + i;
          float v = 0.0f;
          const int k0 = 16 * s + i, k1 = k0 + 8;   // slot of this lane's half
          if (kk < S) {
            v = (&ywin[HALO + r][lc])[hh ? coff(k1) : coff(k0)];
          } else if (kk < CTX && has_ifce) {
            v = fwin[r >> 1][kk - S][(32 * wave + n) >> 1];
          }
          cf[s][i] = v;
        }
      bf16x8 bc[2], bcl[2];
      split8(cf[0], bc[0], bcl[0]);
      split8(cf[1], bc[1], bcl[1]);
      const bool do_bwd = bwd > 0;
      // ---- layer 1 (with the stabilizer in rows H1, H1 + 1) and 2
      f32x16 z = {};
      f32x16 D = mfma3(wop[0][0][lane + zq], wopl[0][0][lane + zq], bc[0], bcl[0], z);
      if (CTX > 16) D = mfma3(wop[0][1][lane + zq], wopl[0][1][lane + zq], bc[1], bcl[1], D);
      float o0 = hh == HS ? D[IS] : 0.0f, o1 = hh == HS ? D[IS + 1] : 0.0f;
      unsigned m1 = 0, m2 = 0;
      bf16x8 bh[2], bhl[2];
      {
        float hv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          hv[i] = fmaxf(D[i] + vec[0][mrow(i, hh) + zq], 0.0f);
          m1 |= (hv[i] > 0.0f ? 1u : 0u) << i;
        }
        split8(hv, bh[0], bhl[0]);
        split8(hv + 8, bh[1], bhl[1]);
      }
      D = mfma3(wop[1][0][lane + zq], wopl[1][0][lane + zq], bh[0], bhl[0], z);
      D = mfma3(wop[1][1][lane + zq], wopl[1][1][lane + zq], bh[1], bhl[1], D);
      bf16x8 vh[2], vl[2];   // H2 (split, for the output layer's weight gradient)
      {
        float v2[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const float v = fmaxf(D[i] + vec[1][mrow(i, hh) + zq], 0.0f);
          m2 |= (v > 0.0f ? 1u : 0u) << i;
          o0 += vec[2][mrow(i, hh) + zq] * v;
          o1 += vec[3][mrow(i, hh) + zq] * v;
          v2[i] = v;
        }
        split8(v2, vh[0], vl[0]);
        split8(v2 + 8, vh[1], vl[1]);
      }
      const float p0 = __shfl_xor(o0, 32), p1 = __shfl_xor(o1, 32);
      const float mu = (o0 + p0) + (b30 + bs0);
      const float ls = (o1 + p1) + (b31 + bs1);
      // ---- rate (FP32)
      // the clamp and the floor below let a NaN through (it then reaches the loss)
      const float lcl = ls != ls ? ls : fminf(fmaxf(ls, d->lmin), d->lmax);
      const bool lin = ls >= d->lmin && ls <= d->lmax;
      const float yv = ywin[HALO + r][lc];
      float bits, gd, gl;
      laplace_bits(yv - mu, expf(-lcl), bits, gd, gl);
      if (bits > d->bits_max) {
        bits = d->bits_max;
        gd = 0.0f;
        gl = 0.0f;
      }
      if (!lin) gl = 0.0f;
      if (!valid) {
        bits = 0.0f;
        gd = 0.0f;
        gl = 0.0f;
      }
      if (hh == 0) bsum += (double)bits;
      if (!do_bwd) continue;

      // ---- backward
      const float dmu = -gd * rs, dl = gl * rs;
      bf16x8 b2[2], b2l[2];   // dH2 (B operand, split)
      {
        float gv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i)
          gv[i] = ((m2 >> i) & 1u) ? vec[2][mrow(i, hh) + zq] * dmu + vec[3][mrow(i, hh) + zq] * dl : 0.0f;
        split8(gv, b2[0], b2l[0]);
        split8(gv + 8, b2[1], b2l[1]);
      }
      D = mfma3(wop[2][0][lane + zq], wopl[2][0][lane + zq], b2[0], b2l[0], z);
      D = mfma3(wop[2][1][lane + zq], wopl[2][1][lane + zq], b2[1], b2l[1], D);
      bf16x8 b1[2], b1l[2];   // dH1 with (d mu, d l) in the stabilizer rows
      {
        float gv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) gv[i] = ((m1 >> i) & 1u) ? D[i] : 0.0f;
        // (d mu, d l) enter at the stabilizer rows: the transposed first layer
        // then adds the stabilizer's context gradient, and the weight
        // gradients get rows H1, H1 + 1 (only in half HS: the same registers
        // of the other half hold hidden units H1 - 4, H1 - 3 when HS = 1)
        if (hh == HS) {
          gv[IS] = dmu;
          gv[IS + 1] = dl;
        }
        split8(gv, b1[0], b1l[0]);
        split8(gv + 8, b1[1], b1l[1]);
      }
      D = mfma3(wop[3][0][lane + zq], wopl[3][0][lane + zq], b1[0], b1l[0], z);
      D = mfma3(wop[3][1][lane + zq], wopl[3][1][lane + zq], b1[1], b1l[1], D);
      float dc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) dc[i] = D[i];
      // IFCE gradients, summed over each 2 x 2 block (column pairs of both
      // band rows, in the order (top pair) + (bottom pair)) and written at
      // the next coarser resolution: the first level of the IFCE pooling
      // (the per-position values are not needed; grids with IFCEs have even
      // sides, and outside the grid the gradients are exactly zero)
      if (has_ifce) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int m = mrow(i, hh);
          if (m >= S && m < CTX) {
            const float pr = dc[i] + __shfl_xor(dc[i], 1);
            if ((r & 1) == 0) {
              dfs[wave][m - S][n] = pr;
            } else if ((n & 1) == 0 && x < w) {
              const int w1 = d->gw[k + 1], n1 = d->gh[k + 1] * w1;
              d->df[d->dfoff[k][1] + (m - S) * n1 + (y >> 1) * w1 + (x >> 1)] = dfs[wave][m - S][n] + pr;
            }
          }
        }
      }


      // ---- context gradient to the neighbours, without atomics: this
      // wavefront stages the slot gradients as [slot][position] (the direct
      // term as slot 32; positions padded with 2*HALO zeros on each side;
      // outside the grid they are exactly zero), then each lane owns one
      // destination column of the rows r - HALO .. r, sums the slots that
      // reach it in slot order and adds the sums to its window
      {
        float* g = &gsc[wave][0][0] + (hh ? 4 * GP : 0) + 2 * HALO + n;
#pragma unroll
        for (int i = 0; i < 16; ++i) g[mrow(i, 0) * GP] = dc[i];
        if (hh == 0) gsc[wave][32][2 * HALO + n] = gd * rs;
      }
      if (lane < PW) {
        const float* g = &gsc[wave][0][0] + lane + HALO;
        float sr[HALO + 1];
        sr[0] = g[32 * GP];
#pragma unroll
        for (int q = 1; q <= HALO; ++q) sr[q] = 0.0f;
#pragma unroll
        for (int m = 0; m < S; ++m) sr[-CDY[m]] += g[m * GP - CDX[m]];
        float* pw = &pacc[wave][HALO + r][lane];
#pragma unroll
        for (int q = 0; q <= HALO; ++q) pw[-q * PW] += sr[q];
      }

      // ---- weight gradients, positions on K: every operand transposed
      // through the matrix cores, hi and lo parts apart (exact)
      bf16x8 ah[2], al[2], xh[2], xl[2];
      transpose2(b1, pu, ah);                // dH1^T (+ stabilizer rows)
      transpose2(b1l, pu, al);
      transpose2(bc, pc, xh);                // C^T, ones in column CTX
      transpose2(bcl, pc, xl);
      if (n == CTX) set_column(xh, xl, 1.0f);
      acc1 = mma_split(ah, al, xh, xl, acc1);
      transpose2(vh, pu, xh);                // H2^T, ones in column H2
      transpose2(vl, pu, xl);
      if (n == H2) set_column(xh, xl, 1.0f);
      acc3 = mma_split(ah, al, xh, xl, acc3);
      transpose2(b2, pu, ah);                // dH2^T
      transpose2(b2l, pu, al);
      transpose2(bh, pu, xh);                // H1^T, ones in column H1, zero beyond
      transpose2(bhl, pu, xl);
      if (n >= H1) set_column(xh, xl, n == H1 ? 1.0f : 0.0f);
      acc2 = mma_split(ah, al, xh, xl, acc2);
    }
    __syncthreads();
    if (seg + 1 < nseg) {   // in flight during the merge
      load_window(x0 + SW, tq);
      if (has_ifce) load_inputs(x0 + SW, tq);
    }
    // ---- merge the wavefront windows (fixed order) with the carried
    // columns, write the finished columns of this segment and carry the last
    // 2*HALO columns into the next one.  Row rr of the window is grid row
    // y0 - HALO + rr: rows >= HALO belong to this band (plane 0), the
    // others to the band q = ceil((HALO - rr) / TH) above (plane q).
    if (bwd > 0) {
      const bool last = seg == nseg - 1;
      for (int i = tq; i < (HALO + TH) * WR; i += NW * 64) {
        const int rr = i / WR, c = i - rr * WR;
        float v = c < 2 * HALO ? cin[rr][c] : 0.0f;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
          const int cc = c - 32 * q;
          if (cc >= 0 && cc < PW) {
            v += pacc[q][rr][cc];
            pacc[q][rr][cc] = 0.0f;
          }
        }
        if (c >= SW && !last) {
          cout[rr][c - SW] = v;
          continue;
        }
        const int gy = y0 - HALO + rr, gx = x0 - HALO + c;
        if (gx < 0 || gx >= w || gy < 0 || gy >= h) continue;
        // plane 0: this band's rows; plane q: the rows of the band q above
        const int plane = rr >= HALO ? 0 : (HALO - rr + TH - 1) / TH;
        d->dc[(size_t)plane * d->n_lat + d->goff[k] + gy * w + gx] = v;
      }
      __syncthreads();
      if (tq < (HALO + TH) * 2 * HALO) (&cin[0][0])[tq] = (&cout[0][0])[tq];
    }
  }

  // ---- bits of this workgroup
  for (int off = 32; off > 0; off >>= 1) bsum += __shfl_xor(bsum, off);
  if (lane == 0) bsh[wave] = bsum;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int q = 0; q < NW; ++q) s += bsh[q];
    d->lp_bits[bidx] = s;
  }
  if (bwd > 0) {

  // ---- weight gradients: fixed-order sum over wavefronts, one partial row
  for (int q = 0; q < NW; ++q) {
    if (wave == q) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int m = mrow(i, hh);
        if (q == 0) {
          wsum[0][m][n] = acc1[i];
          wsum[1][m][n] = acc2[i];
          wsum[2][m][n] = acc3[i];
        } else {
          wsum[0][m][n] += acc1[i];
          wsum[1][m][n] += acc2[i];
          wsum[2][m][n] += acc3[i];
        }
      }
    }
    __syncthreads();
  }
  // the ARM parameters only (the row ends before the IFCE parameters)
  const int pcnt = d->prod[d->prod_arm].pcnt;
  float* out = d->wp + d->prod[d->prod_arm].off + (size_t)bidx * pcnt;
  int te = threadIdx.x;
  __asm__ volatile("" : "+v"(te));
  for (int p = te; p < pcnt; p += NW * 64) {
    const unsigned e = d->arm_ftab[p];
    const int a = (e >> 10) & 3, row = (e >> 5) & 31, col = e & 31;
    out[p] = wsum[a][row][col];
  }
  }
  // LDS of this band (window, accumulators, sums, IFCE weights) is reused
  // by the next one
  __syncthreads();
  }
}

template <int S, int F, int H1, int H2>
int launch_t(const Launch& l, int bwd, hipStream_t st) {
  hipLaunchKernelGGL((k_arm_fused<S, F, H1, H2>), dim3(l.tile0[l.n]), dim3(NW * 64), 0, st, l, bwd);
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EDEVICE;
}

}  // namespace

#define CC_FUSED_SHAPES(X) \
  X(16, 0, 16, 16)         \
  X(24, 6, 24, 24)         \
  X(18, 6, 24, 24)         \
  X(6, 2, 5, 4)            \
  X(6, 2, 8, 8)            \
  X(10, 4, 10, 10)         \
  X(14, 6, 20, 20)         \
  X(20, 6, 26, 26)

int cc_arm_fused_supported(const DevDesc& h) {
  if (h.S > NOFF) return 0;
  // the context (spatial slots and IFCE features) and its bias column fit
  // one 32-row tile
  if (h.S + h.F > 31) return 0;
  for (int k = 0; k < h.G; ++k)
    if (h.nin[k] > CC_MAX_NIN) return 0;
  for (int m = 0; m < h.S; ++m)
    if (h.dy[m] != CDY[m] || h.dx[m] != CDX[m]) return 0;
#define X(a, b, c, e) if (h.S == a && h.F == b && h.H1 == c && h.H2 == e) return 1;
  CC_FUSED_SHAPES(X)
#undef X
  return 0;
}

int cc_launch_arm_fused(const Launch& l, const DevDesc& h, int bwd, hipStream_t st) {
#define X(a, b, c, e) \
  if (h.S == a && h.F == b && h.H1 == c && h.H2 == e) return launch_t<a, b, c, e>(l, bwd, st);
  CC_FUSED_SHAPES(X)
#undef X
  return CC_EINVAL;
}
