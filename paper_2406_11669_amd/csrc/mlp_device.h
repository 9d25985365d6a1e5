// mlp_device.h -- device code of the learned c2p guess's network, shared by the point kernels
// and the grid c2p kernel: parameter packing, bfloat16 rounding, the input features and the
// forward pass of one wavefront on the matrix cores.  Hidden activations: ReLU.  (See learned_c2p.hip for the design.)
#ifndef ASTERX_MLP_DEVICE_H
#define ASTERX_MLP_DEVICE_H

#include <hip/hip_runtime.h>

#include <cstdint>

#include "asterx.h"
#include "grmhd_device.h"

namespace mlpd {
using namespace ax;

constexpr int NI = 8, NH = 64, NO = 2;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH;
constexpr int OB3 = OW3 + NO * NH, NP = OB3 + NO;
static_assert(NP == ASTERX_MLP_NPARAMS, "parameter packing");

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

DEV short bf16(float x) {  // round to nearest even: one v_cvt_pk_bf16_f32 on gfx950
  return __builtin_bit_cast(short, (__bf16)x);
}

DEV float act(float x) {  // ReLU: one instruction per activation, where tanh would cost an exp and a reciprocal
  return fmaxf(x, 0.0f);
}

DEV f4 mfma(bf4 a, bf4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

// Two 16-deep K tiles in one v_mfma_f32_16x16x32_bf16 (twice the K of the 16-deep instruction per
// issue on gfx950).  Lane group g supplies K slots 8g..8g+7; taking slots 0-3 from tile (a0, b0) and
// 4-7 from tile (a1, b1) -- the same logical k for A and B in every slot -- leaves the contraction
// unchanged and lets a layer's 16 x 16 accumulator tiles feed the next layer as they are.
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
DEV f4 mfma32(s8 a, s8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// A operand of mfma32: row r of W (row length ld), K tiles kt and kt + 1, this lane group's 4 + 4.
DEV s8 ld8(const float* __restrict__ P, int o, int kt, int lg, bool on) {
  s8 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i] = on ? bf16(P[o + kt * 16 + 4 * lg + i]) : (short)0;
    r[4 + i] = on ? bf16(P[o + (kt + 1) * 16 + 4 * lg + i]) : (short)0;
  }
  return r;
}

DEV bf4 ld4(const float* __restrict__ P, int o, bool on) {
  bf4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = on ? bf16(P[o + i]) : (short)0;
  return r;
}

struct Stdz {
  float is[NI], isc[NI], os[NO], osc[NO];
};

// Features of a conserved state (undensitized input c): log D, log(tau/D), log(1 + S^2/D^2),
// log(1 + B^2/D), log(1 + (B.S)^2/D^3), det(gamma) - 1, alpha - 1, Gamma.  usable = false when
// the state cannot be fed to the network (non-positive D or tau, non-finite values).
DEV void features(const Geo& G, const C2PIn& c, double gam, float f[NI], bool& usable) {
  double D = c.D;
  usable = D > 0.0 && c.tau > 0.0 && isfinite(c.S2) && isfinite(c.B2) && isfinite(c.tau);
  if (!usable) {
#pragma unroll
    for (int k = 0; k < NI; ++k) f[k] = 0.0f;
    return;
  }
  // single precision is plenty for a network input (hardware logarithm)
  const double iD = 1.0 / D;
  f[0] = __logf((float)D);
  f[1] = __logf((float)(c.tau * iD));
  f[2] = __logf(1.0f + (float)(c.S2 * iD * iD));
  f[3] = __logf(1.0f + (float)(c.B2 * iD));
  f[4] = __logf(1.0f + (float)(c.BS * c.BS * iD * iD * iD));
  f[5] = (float)(G.sqrtg * G.sqrtg - 1.0);
  f[6] = (float)(G.alp - 1.0);
  f[7] = (float)gam;
}

// ---- one wavefront, 64 samples ------------------------------------------------------------------
// feat: LDS [64][8] standardised inputs.  y[nt]: output tile nt (lanes 0..15 hold rows 0, 1 =
// outputs of sample nt*16 + lane).  With TRAIN the FP32 activations and the bfloat16 operands of
// every layer are kept for the backward pass.
struct Acts {
  f4 t1[4][4], t2[4][4];
  bf4 x1[4], x2[4][4], x3[4][4];
};

template <bool TRAIN>
DEV void mlp_fwd(const float* __restrict__ P, const float (*feat)[NI], f4 y[4], Acts* A) {
  const int l = __lane_id(), lr = l & 15, lg = l >> 4;
  bf4 x1[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) x1[nt][i] = lg < 2 ? bf16(feat[nt * 16 + lr][4 * lg + i]) : (short)0;
  f4 h[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    bf4 a = ld4(P, OW1 + (mt * 16 + lr) * NI + 4 * lg, lg < 2);
    f4 bias;
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[i] = P[OB1 + mt * 16 + 4 * lg + i];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) h[mt][nt] = mfma(a, x1[nt], bias);
  }
  // activations in the packed operand layout of mfma32: x2[q][nt] holds K tiles 2q (slots 0-3) and
  // 2q + 1 (slots 4-7), i.e. the accumulator tiles mt = 2q, 2q + 1 of the layer before
  s8 x2[2][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float t = act(h[mt][nt][i]);
        if (TRAIN) A->t1[mt][nt][i] = t;
        x2[mt >> 1][nt][4 * (mt & 1) + i] = bf16(t);
      }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f4 bias;
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[i] = P[OB2 + mt * 16 + 4 * lg + i];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) h[mt][nt] = bias;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      s8 a = ld8(P, OW2 + (mt * 16 + lr) * NH, 2 * q, lg, true);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) h[mt][nt] = mfma32(a, x2[q][nt], h[mt][nt]);
    }
  }
  s8 x3[2][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float t = act(h[mt][nt][i]);
        if (TRAIN) A->t2[mt][nt][i] = t;
        x3[mt >> 1][nt][4 * (mt & 1) + i] = bf16(t);
      }
  f4 b3;
#pragma unroll
  for (int i = 0; i < 4; ++i) b3[i] = (4 * lg + i < NO) ? P[OB3 + 4 * lg + i] : 0.0f;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) y[nt] = b3;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    s8 a = ld8(P, OW3 + lr * NH, 2 * q, lg, lr < NO);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) y[nt] = mfma32(a, x3[q][nt], y[nt]);
  }
  if (TRAIN) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) A->x1[nt] = x1[nt];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          A->x2[mt][nt][i] = x2[mt >> 1][nt][4 * (mt & 1) + i];
          A->x3[mt][nt][i] = x3[mt >> 1][nt][4 * (mt & 1) + i];
        }
  }
}

}  // namespace mlpd

#endif
