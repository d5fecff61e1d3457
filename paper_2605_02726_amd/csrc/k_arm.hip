// ARM entropy model, plain FP32 form: one thread per latent position.
//
// For every position i of every grid k (Section III-A): causal spatial
// context s_i and, on grids k < G, the inter-feature context f_i = W r_i + b
// of the co-located coarser-grid values r_i (Section III-A.2); the MLP with
// linear stabilizer gives (mu, l); the Laplace bin probability of yhat_i
// (eq. laplace-distribution) gives its bits.  With BWD the kernel also runs
// the backward pass: d loss / d (mu, l, yhat_i) -> MLP backward -> context
// gradient dc (written per neighbour slot, gathered later by reversed offsets)
// and the IFCE gradient df; the weight gradient of the workgroup's positions
// is reduced through LDS into one partial row per workgroup.
//
// Weights are read through uniform addresses (scalar loads feeding the FMA
// operands); one workgroup is one wavefront looping over chunks of 64
// positions that never straddle two grids.
#include "cc_internal.h"

#include <math.h>

namespace {

constexpr float INV_LN2 = 1.4426950408889634f;

// Bits of one latent under Laplace(mu, b) on the unit bin around yhat, with
// the derivatives d bits / d (yhat - mu) and b * d bits / d b, in FP32 with
// expm1 forms that avoid cancellation:
//   |d| >= 1/2:  bits = (|d| - 1/2) / (b ln 2) - log2(-expm1(-1/b) / 2)
//   |d| <  1/2:  p = 1 - (exp(-(1/2 + d)/b) + exp(-(1/2 - d)/b)) / 2
__device__ __forceinline__ void laplace_bits(float dd, float ib, float& bits, float& gd,
                                             float& gl) {
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

template <int S, int F, int H1, int H2, bool BWD>
__global__ __launch_bounds__(64) void k_arm_plain(Launch Lc) {
  constexpr int CTX = S + F;
  constexpr int RM = CC_MAX_NIN;
  constexpr int O_H1 = CTX, O_H2 = O_H1 + H1, O_R = O_H2 + H2, O_DH1 = O_R + RM,
                O_DH2 = O_DH1 + H1, O_DO = O_DH2 + H2, O_DF = O_DO + 2, O_ONE = O_DF + F;
  constexpr int AST = (O_ONE + 1) | 1;
  constexpr int PMAX = (CTX + 1) * H1 + (H1 + 1) * H2 + (H2 + 1) * 2 + (CTX + 1) * 2 +
                       3 * F * (CC_MAX_NIN + 1);
  constexpr int NQ = (PMAX + 63) / 64;
  __shared__ float lds[BWD ? 64 * AST : 1];

  const int im = cc_find_img(Lc, blockIdx.x);
  const CDesc* d = (const CDesc*)Lc.d[im];
  const int wg = blockIdx.x - Lc.tile0[im];
  const int lane = threadIdx.x;
  const CF* P0 = (const CF*)(d->theta + d->n_lat);
  const bool stab = d->arm_stab != 0;
  const float rs = d->rate_scale;

  float acc[BWD ? NQ : 1];
  if constexpr (BWD) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0f;
  }
  double bsum = 0.0;

  for (int ch = wg; ch < d->arm_nchunk; ch += d->arm_nwg) {
    // The weights are re-read (scalar loads) in every chunk: laundering the
    // base pointer keeps the compiler from hoisting ~1.5k loop-invariant
    // weights into vector registers.
    const CF* P = P0;
    asm volatile("" : "+s"(P));
    const CF* W1 = P + d->p_aw[0];
    const CF* B1 = P + d->p_ab[0];
    const CF* W2 = P + d->p_aw[1];
    const CF* B2 = P + d->p_ab[1];
    const CF* W3 = P + d->p_aw[2];
    const CF* B3 = P + d->p_ab[2];
    const CF* Ws = P + d->p_asw;
    const CF* Bs = P + d->p_asb;
    int k = 0, c0 = ch;
    for (;;) {
      const int nck = (d->gh[k] * d->gw[k] + 63) >> 6;
      if (c0 < nck || k == d->NG - 1) break;
      c0 -= nck;
      ++k;
    }
    const int w = d->gw[k], nk = d->gh[k] * w;
    const int li = c0 * 64 + lane;
    const bool valid = li < nk;
    const int y = valid ? li / w : 0, x = valid ? li - y * w : 0;
    const float* yg = d->yhat + d->goff[k];

    float c[CTX];
#pragma unroll
    for (int m = 0; m < S; ++m) {
      const int yy = y + d->dy[m], xx = x + d->dx[m];
      c[m] = (valid && yy >= 0 && xx >= 0 && xx < w) ? yg[yy * w + xx] : 0.0f;
    }
    float r[RM];
#pragma unroll
    for (int q = 0; q < RM; ++q) r[q] = 0.0f;
    const bool has_ifce = (F > 0) && (k < d->G);
    if constexpr (F > 0) {
#pragma unroll
      for (int f = 0; f < F; ++f) c[S + f] = 0.0f;
      if (has_ifce) {
        const int nin = d->nin[k];
#pragma unroll
        for (int q = 0; q < RM; ++q) {
          if (q < nin && valid) {
            const int j = d->isrc[k][q], sh = d->ish[k][q];
            r[q] = d->yhat[d->goff[j] + (y >> sh) * d->gw[j] + (x >> sh)];
          }
        }
        const CF* Wi = P + d->p_iw[k];
        const CF* Bi = P + d->p_ib[k];
#pragma unroll
        for (int f = 0; f < F; ++f) {
          float s = Bi[f];
#pragma unroll
          for (int q = 0; q < RM; ++q)
            if (q < nin) s += Wi[f * nin + q] * r[q];
          c[S + f] = s;
        }
      }
    }

    float h1[H1], h2[H2];
#pragma unroll
    for (int a = 0; a < H1; ++a) {
      float s = B1[a];
#pragma unroll
      for (int q = 0; q < CTX; ++q) s += W1[a * CTX + q] * c[q];
      h1[a] = fmaxf(s, 0.0f);
    }
#pragma unroll
    for (int a = 0; a < H2; ++a) {
      float s = B2[a];
#pragma unroll
      for (int q = 0; q < H1; ++q) s += W2[a * H1 + q] * h1[q];
      h2[a] = fmaxf(s, 0.0f);
    }
    float o0 = B3[0], o1 = B3[1];
#pragma unroll
    for (int q = 0; q < H2; ++q) {
      o0 += W3[q] * h2[q];
      o1 += W3[H2 + q] * h2[q];
    }
    if (stab) {
      float s0 = Bs[0], s1 = Bs[1];
#pragma unroll
      for (int q = 0; q < CTX; ++q) {
        s0 += Ws[q] * c[q];
        s1 += Ws[CTX + q] * c[q];
      }
      o0 += s0;
      o1 += s1;
    }

    // the clamp and the floor below let a NaN through (it then reaches the loss)
    const float lcl = o1 != o1 ? o1 : fminf(fmaxf(o1, d->lmin), d->lmax);
    const bool lin = o1 >= d->lmin && o1 <= d->lmax;
    const float ib = expf(-lcl);
    const float yv = valid ? yg[li] : 0.0f;
    float bits, gd, gl;
    laplace_bits(yv - o0, ib, bits, gd, gl);
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
    bsum += (double)bits;

    if constexpr (BWD) {
      const float dmu = -gd * rs, dl = gl * rs;
      float dh2[H2], dh1[H1];
#pragma unroll
      for (int a = 0; a < H2; ++a) dh2[a] = h2[a] > 0.0f ? W3[a] * dmu + W3[H2 + a] * dl : 0.0f;
#pragma unroll
      for (int b = 0; b < H1; ++b) {
        float s = 0.0f;
#pragma unroll
        for (int a = 0; a < H2; ++a) s += W2[a * H1 + b] * dh2[a];
        dh1[b] = h1[b] > 0.0f ? s : 0.0f;
      }
      float* row = lds + lane * AST;
      const int gi = d->goff[k] + li;
#pragma unroll
      for (int q = 0; q < CTX; ++q) {
        float s = 0.0f;
#pragma unroll
        for (int b = 0; b < H1; ++b) s += W1[b * CTX + q] * dh1[b];
        if (stab) s += Ws[q] * dmu + Ws[CTX + q] * dl;
        if (q < S) {
          if (valid) d->dc[(size_t)q * d->n_lat + gi] = s;
        } else {
          const float dfv = has_ifce ? s : 0.0f;
          if (has_ifce && valid) d->df[d->dfoff[k][0] + (q - S) * nk + li] = dfv;
          row[O_DF + q - S] = dfv;
        }
        row[q] = c[q];
      }
      if (valid) d->dyd[gi] = gd * rs;
#pragma unroll
      for (int a = 0; a < H1; ++a) {
        row[O_H1 + a] = h1[a];
        row[O_DH1 + a] = dh1[a];
      }
#pragma unroll
      for (int a = 0; a < H2; ++a) {
        row[O_H2 + a] = h2[a];
        row[O_DH2 + a] = dh2[a];
      }
#pragma unroll
      for (int q = 0; q < RM; ++q) row[O_R + q] = r[q];
      row[O_DO] = dmu;
      row[O_DO + 1] = dl;
      row[O_ONE] = 1.0f;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int pq = lane + 64 * q;
        const unsigned e = pq < d->n_arm_par ? d->arm_gtab[pq] : 0xFFFFFFFFu;
        if (e == 0xFFFFFFFFu) continue;
        const int ia = e & 0xFF, ibb = (e >> 8) & 0xFF, kr = (e >> 16) & 0xFF;
        if (kr != 0xFF && kr != k) continue;
        float s = 0.0f;
        for (int pos = 0; pos < 64; ++pos) s += lds[pos * AST + ia] * lds[pos * AST + ibb];
        acc[q] += s;
      }
      __syncthreads();
    }
  }

  if constexpr (BWD) {
    float* out = d->wp + d->prod[d->prod_arm].off + (size_t)wg * d->n_arm_par;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int p = lane + 64 * q;
      if (p < d->n_arm_par) out[p] = acc[q];
    }
  }
  for (int off = 32; off > 0; off >>= 1) bsum += __shfl_xor(bsum, off);
  if (lane == 0) d->lp_bits[wg] = bsum;
}

template <int S, int F, int H1, int H2>
int launch_arm_t(const Launch& l, int bwd, hipStream_t st) {
  if (bwd)
    hipLaunchKernelGGL((k_arm_plain<S, F, H1, H2, true>), dim3(l.tile0[l.n]), dim3(64), 0, st, l);
  else
    hipLaunchKernelGGL((k_arm_plain<S, F, H1, H2, false>), dim3(l.tile0[l.n]), dim3(64), 0, st, l);
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EDEVICE;
}

}  // namespace

// Supported ARM shapes (s, F, hidden1, hidden2).
#define CC_ARM_SHAPES(X) \
  X(16, 0, 16, 16)       \
  X(24, 6, 24, 24)       \
  X(18, 6, 24, 24)       \
  X(6, 2, 5, 4)          \
  X(6, 2, 8, 8)          \
  X(10, 4, 10, 10)       \
  X(14, 6, 20, 20)       \
  X(20, 6, 26, 26)

int cc_arm_shape_supported(int S, int F, int H1, int H2) {
#define X(a, b, c, e) if (S == a && F == b && H1 == c && H2 == e) return 1;
  CC_ARM_SHAPES(X)
#undef X
  return 0;
}

int cc_launch_arm_plain(const Launch& l, const DevDesc& h, int bwd, hipStream_t st) {
#define X(a, b, c, e) \
  if (h.S == a && h.F == b && h.H1 == c && h.H2 == e) return launch_arm_t<a, b, c, e>(l, bwd, st);
  CC_ARM_SHAPES(X)
#undef X
  return CC_EINVAL;
}
