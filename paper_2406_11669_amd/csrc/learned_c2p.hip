// learned_c2p.hip -- learned initial guess for the conservative-to-primitive recovery (gfx950).
//
// A multilayer perceptron 8 -> 64 -> 64 -> 2 (ReLU hidden activations) maps eight features of
// a conserved state to (log W, log(z / D)), z = rho h W^2, which seed Noble's 2D Newton
// iteration (Sec. 3.5).  The FP64 iteration polishes the guess to the same tolerance as the
// plain recovery; if it does not converge, the plain warm/cold start, Palenzuela's 1D
// solver and the atmosphere follow as usual, so the network never decides the result.
//
// Arithmetic of the network: weights, inputs and hidden activations are rounded to bfloat16
// (round to nearest even) and contracted on the matrix cores (FP32 accumulate): the forward
// pass's 64-deep layers with v_mfma_f32_16x16x32_bf16, the 8-deep input layer and the backward
// pass with v_mfma_f32_16x16x16_bf16; biases, activations and the loss are FP32.  ReLU rather than tanh: the
// network runs inside the recovery, where a tanh (exponential and reciprocal, quarter-rate) per
// hidden unit cost more than the Newton iterations the guess saves.  One wavefront evaluates 64
// samples: every layer is computed transposed (H^T = W X^T), so that the accumulator layout
// of one layer (lane l holds rows 4(l/16)..4(l/16)+3 of column l%16) is exactly the B-operand
// layout of the next and activations never leave registers; the weight gradients, which
// contract over samples, take their operands through a transpose in LDS.
//
// Training: asterx_mlp_grad evaluates the loss (1/n) sum_i |y_i - t_i|^2 / 2 on standardised
// outputs and its gradient with respect to the FP32 master parameters (per-wavefront partial
// sums reduced in a fixed order: deterministic); asterx_mlp_adam applies one Adam step.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "asterx.h"
#include "grmhd_device.h"
#include "host_internal.h"
#include "mlp_device.h"

using namespace ax;

namespace {

using namespace mlpd;

// Sum over the 16 lanes that share l / 16 (the sample index within a tile).
DEV float sum16(float v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Writes a D-layout tile set (rows base + 4(l/16) + i, column = sample nt*16 + l%16) into an LDS
// matrix T[row][sample] of bfloat16.
DEV void tile_to_lds(short (*T)[64], const bf4 v[4][4], int mtiles) {
  const int l = __lane_id(), lr = l & 15, lg = l >> 4;
  for (int mt = 0; mt < mtiles; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) T[mt * 16 + 4 * lg + i][nt * 16 + lr] = v[mt][nt][i];
}

// A/B operand read of rows r0 + l%16, samples kt*16 + 4(l/16) .. +3 from T[row][sample].
DEV bf4 lds_op(const short (*T)[64], int r0, int kt) {
  const int l = __lane_id(), lr = l & 15, lg = l >> 4;
  bf4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = T[r0 + lr][kt * 16 + 4 * lg + i];
  return r;
}

struct LdsTrain {
  float feat[64][NI];
  short A[64][64];
  short B[64][64];
};

// ---- kernels -------------------------------------------------------------------------------------

// Per-wavefront loss and gradient partial sums: part[w * (NP + 1) + p], p < NP the parameter
// gradient, p = NP the loss.  feat: raw features (NI x n), tgt: raw targets (NO x n).
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ P, long long n, const float* feat,
                                                 const float* tgt, Stdz z, float inv_n, float* part) {
  __shared__ LdsTrain S;
  const int l = __lane_id(), lr = l & 15, lg = l >> 4;
  const long long s0 = (long long)blockIdx.x * 64;
  {
    long long s = s0 + l;
#pragma unroll
    for (int k = 0; k < NI; ++k) S.feat[l][k] = s < n ? (feat[k * n + s] - z.is[k]) * z.isc[k] : 0.0f;
  }
  __syncthreads();
  Acts A;
  f4 y[4];
  mlp_fwd<true>(P, S.feat, y, &A);
  // output cotangent (lanes of row group 0 hold outputs 0, 1 of sample nt*16 + lr)
  f4 d3[4];
  float loss = 0.0f;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      long long s = s0 + nt * 16 + lr;
      float d = 0.0f;
      if (lg == 0 && i < NO && s < n) {
        float t = (tgt[i * n + s] - z.os[i]) * z.osc[i];
        float e = y[nt][i] - t;
        loss += 0.5f * e * e;
        d = e * inv_n;
      }
      d3[nt][i] = d;
    }
  float* out = part + (size_t)blockIdx.x * (NP + 1);
  // bias 3 and loss
  {
    float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      g0 += d3[nt][0];
      g1 += d3[nt][1];
    }
    g0 = sum16(g0);
    g1 = sum16(g1);
    float L = loss;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) L += __shfl_xor(L, o, 64);
    if (l == 0) {
      out[OB3] = g0;
      out[OB3 + 1] = g1;
      out[NP] = L * inv_n;
    }
  }
  bf4 d3b[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) d3b[nt][i] = bf16(d3[nt][i]);
  // dW3 = delta3 x3^T: A = delta3 [o][s] (rows 0, 1), B = x3 [h][s]
  {
    bf4 tmp[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) tmp[0][nt] = d3b[nt];
    tile_to_lds(S.A, tmp, 1);
    tile_to_lds(S.B, A.x3, 4);
    __syncthreads();
    f4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      bf4 a = lds_op(S.A, 0, kt);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma(a, lds_op(S.B, nt * 16, kt), acc[nt]);
    }
    if (lg == 0)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < NO; ++i) out[OW3 + i * NH + nt * 16 + lr] = acc[nt][i];
    __syncthreads();
  }
  // delta2 = (W3^T delta3) * ReLU'(t2)
  bf4 d2b[4][4];
  {
    float gb2[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      bf4 a;
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (4 * lg + i < NO) ? bf16(P[OW3 + (4 * lg + i) * NH + mt * 16 + lr]) : (short)0;
      // lane l supplies A[m = mt*16 + lr][k = 4 lg + i] = W3[k][m]
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f4 g = mfma(a, d3b[nt], f4{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float t = A.t2[mt][nt][i];
          float d = t > 0.0f ? g[i] : 0.0f;  // ReLU'
          d2b[mt][nt][i] = bf16(d);
          gb2[mt][i] = (nt == 0 ? 0.0f : gb2[mt][i]) + d;
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = sum16(gb2[mt][i]);
        if (lr == 0) out[OB2 + mt * 16 + 4 * lg + i] = v;
      }
  }
  // dW2 = delta2 x2^T: A = delta2 [h2][s], B = x2 [h1][s]
  {
    tile_to_lds(S.A, d2b, 4);
    tile_to_lds(S.B, A.x2, 4);
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f4 acc[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        bf4 a = lds_op(S.A, mt * 16, kt);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma(a, lds_op(S.B, nt * 16, kt), acc[nt]);
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[OW2 + (mt * 16 + 4 * lg + i) * NH + nt * 16 + lr] = acc[nt][i];
    }
    __syncthreads();
  }
  // delta1 = (W2^T delta2) * ReLU'(t1)
  bf4 d1b[4][4];
  {
    float gb1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f4 g[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) g[nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        bf4 a;  // A[m = mt*16 + lr][k = kt*16 + 4 lg + i] = W2[k][m]
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = bf16(P[OW2 + (kt * 16 + 4 * lg + i) * NH + mt * 16 + lr]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) g[nt] = mfma(a, d2b[kt][nt], g[nt]);
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float t = A.t1[mt][nt][i];
          float d = t > 0.0f ? g[nt][i] : 0.0f;  // ReLU'
          d1b[mt][nt][i] = bf16(d);
          gb1[mt][i] = (nt == 0 ? 0.0f : gb1[mt][i]) + d;
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = sum16(gb1[mt][i]);
        if (lr == 0) out[OB1 + mt * 16 + 4 * lg + i] = v;
      }
  }
  // dW1 = delta1 x1^T: A = delta1 [h1][s], B = x1 [f][s] (f < 8)
  {
    tile_to_lds(S.A, d1b, 4);
    {
      bf4 tmp[4][4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) tmp[0][nt] = A.x1[nt];
      // x1 tiles hold rows f = 4 lg + i for lg < 2 (zeros above): one 16-row tile
      tile_to_lds(S.B, tmp, 1);
    }
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f4 acc = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) acc = mfma(lds_op(S.A, mt * 16, kt), lds_op(S.B, 0, kt), acc);
      if (lr < NI)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[OW1 + (mt * 16 + 4 * lg + i) * NI + lr] = acc[i];
    }
  }
}

// grad[p] = sum over partials w (in order) of part[w][p], p <= NP (the last slot is the loss).
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int nw, float* __restrict__ grad) {
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p > NP) return;
  float s = 0.0f;
  for (int w = 0; w < nw; ++w) s += part[(size_t)w * (NP + 1) + p];
  grad[p] = s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int np, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  float gi = g[p];
  float mi = b1 * m[p] + (1.0f - b1) * gi;
  float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  w[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Inference: out (NO x n) = de-standardised network outputs of the raw features.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, long long n, const float* feat,
                                                     Stdz z, float* out) {
  __shared__ float F[4][64][NI];
  const int w = threadIdx.x >> 6, l = __lane_id(), lr = l & 15, lg = l >> 4;
  const long long s0 = ((long long)blockIdx.x * 4 + w) * 64;
  {
    long long s = s0 + l;
#pragma unroll
    for (int k = 0; k < NI; ++k) F[w][l][k] = s < n ? (feat[k * n + s] - z.is[k]) * z.isc[k] : 0.0f;
  }
  __syncthreads();
  f4 y[4];
  mlp_fwd<false>(P, F[w], y, nullptr);
  if (lg == 0)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      long long s = s0 + nt * 16 + lr;
      if (s < n)
#pragma unroll
        for (int i = 0; i < NO; ++i) out[i * n + s] = z.os[i] + y[nt][i] / z.osc[i];
    }
}

// ---- point kernels --------------------------------------------------------------------------------

struct PtsIn {
  long long n;
  const double* gam_pts;  // n or NULL
  double gam;
  const double* metric;   // 10 x n
  const double* Bt;       // 3 x n (densitized)
};

DEV double pt_gam(const PtsIn& a, long long i) { return a.gam_pts ? a.gam_pts[i] : a.gam; }

DEV void pt_geo(const PtsIn& a, long long i, Geo& G) {
  double m[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) m[q] = a.metric[q * a.n + i];
  geo_from(m, G);
}

__global__ __launch_bounds__(256) void k_prim2con_points(PtsIn a, const double* prim, double* cons, double* target) {
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  Geo G;
  pt_geo(a, i, G);
  double pr[5], Bt[3], U[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) pr[q] = prim[q * a.n + i];
#pragma unroll
  for (int q = 0; q < 3; ++q) Bt[q] = a.Bt[q * a.n + i];
  double gam = pt_gam(a, i);
  State S;
  state_make(G, pr, Bt, gam, S);
  cons_of(G, S, U);
#pragma unroll
  for (int q = 0; q < 5; ++q) cons[q * a.n + i] = U[q];
  if (target) {  // log W and log(z / D) with z = rho h W^2, D = rho W: log(h W)
    target[i] = log(S.W);
    target[a.n + i] = log(S.rhoh * S.W / S.rho);
  }
}

__global__ __launch_bounds__(256) void k_features_points(PtsIn a, const double* cons, float* feat) {
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  Geo G;
  pt_geo(a, i, G);
  double U[5], Bt[3];
#pragma unroll
  for (int q = 0; q < 5; ++q) U[q] = cons[q * a.n + i];
#pragma unroll
  for (int q = 0; q < 3; ++q) Bt[q] = a.Bt[q * a.n + i];
  C2PIn c;
  c2p_input(G, U, Bt, c);
  float f[NI];
  bool usable;
  features(G, c, pt_gam(a, i), f, usable);
#pragma unroll
  for (int k = 0; k < NI; ++k) feat[k * a.n + i] = f[k];
}

struct C2PPtsArgs {
  PtsIn in;
  C2PParams cp;
  double* cons;
  const double* guess;
  const float* mlp;
  Stdz z;
  double* prim;
  uint8_t* flags;
  int32_t* iters;
  unsigned long long* stats;
};

// c2p of independent points; with a network, each wavefront first evaluates it on its 64
// points (the whole wavefront takes part in the matrix instructions).
__global__ __launch_bounds__(256) void k_c2p_points(C2PPtsArgs a) {
  __shared__ float F[4][64][NI];
  __shared__ float Y[4][64][NO];
  const int w = threadIdx.x >> 6, l = __lane_id(), lr = l & 15, lg = l >> 4;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < a.in.n;
  Geo G;
  double U[5], Bt[3], prev[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double gam = 0.0;
  if (valid) {
    pt_geo(a.in, i, G);
#pragma unroll
    for (int q = 0; q < 5; ++q) U[q] = a.cons[q * a.in.n + i];
#pragma unroll
    for (int q = 0; q < 3; ++q) Bt[q] = a.in.Bt[q * a.in.n + i];
    if (a.guess)
#pragma unroll
      for (int q = 0; q < 5; ++q) prev[q] = a.guess[q * a.in.n + i];
    gam = pt_gam(a.in, i);
  }
  double zw[2];
  bool use_guess = false;
  if (a.mlp) {
    float f[NI];
    bool usable = false;
    C2PIn c;
    if (valid) {
      c2p_input(G, U, Bt, c);
      features(G, c, gam, f, usable);
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) F[w][l][k] = usable ? (f[k] - a.z.is[k]) * a.z.isc[k] : 0.0f;
    __syncthreads();
    f4 y[4];
    mlp_fwd<false>(a.mlp, F[w], y, nullptr);
    if (lg == 0)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int q = 0; q < NO; ++q) Y[w][nt * 16 + lr][q] = a.z.os[q] + y[nt][q] / a.z.osc[q];
    __syncthreads();
    if (usable) {
      double W = (double)__expf(Y[w][l][0]);
      const double wcap = 1.0 - 1.0 / (a.cp.wmax * a.cp.wmax);
      zw[0] = c.D * (double)__expf(Y[w][l][1]);
      zw[1] = fmin(fmax(1.0 - 1.0 / (W * W), 0.0), wcap);
      use_guess = isfinite(zw[0]) && zw[0] > 0.0;
    }
  }
  uint32_t fl = 0;
  int it = 0;
  if (valid) {
    C2PParams cp = a.cp;
    cp.gam = gam;
    double out[5];
    fl = c2p_point(G, U, Bt, prev, cp, out, it, use_guess ? zw : nullptr);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      a.prim[q * a.in.n + i] = out[q];
      a.cons[q * a.in.n + i] = U[q];
    }
    if (a.flags) a.flags[i] = (uint8_t)fl;
    if (a.iters) a.iters[i] = it;
  }
  if (a.stats) {
    // counters: Noble failed, fallback used, atmosphere, hard failure, NaN input, max
    // iterations, learned guess not converged, total iterations
    unsigned long long b[6] = {
        __ballot(valid && (fl & 1u)), __ballot(valid && (fl & 2u)), __ballot(valid && (fl & 4u)),
        __ballot(valid && (fl & 8u)), __ballot(valid && (fl & 16u)), __ballot(valid && (fl & 32u))};
    int mx = valid ? it : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    // counts are pushed only when non-zero and the maximum only when it grows: atomics to one
    // address serialize, and almost every wavefront has nothing new to report
    if (l == 0) {
      for (int q = 0; q < 5; ++q)
        if (b[q]) atomicAdd(&a.stats[q], (unsigned long long)__popcll(b[q]));
      if (mx && __hip_atomic_load(&a.stats[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned long long)mx)
        atomicMax(&a.stats[5], (unsigned long long)mx);
      if (b[5]) atomicAdd(&a.stats[6], (unsigned long long)__popcll(b[5]));
    }
  }
}

unsigned nblk(long long n, int per) { return (unsigned)((n + per - 1) / per); }

int launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return axh::set_error(ASTERX_ELAUNCH, what);
  return 0;
}

bool stdz_from(const asterx_mlp* m, Stdz& z) {
  for (int k = 0; k < NI; ++k) {
    z.is[k] = m->in_shift[k];
    z.isc[k] = m->in_scale[k];
    if (!(m->in_scale[k] > 0.0f)) return false;
  }
  for (int k = 0; k < NO; ++k) {
    z.os[k] = m->out_shift[k];
    z.osc[k] = 1.0f / m->out_scale[k];
    if (!(m->out_scale[k] > 0.0f)) return false;
  }
  return true;
}

int check_pts(long long n, const double* metric, const double* Bt, double gam, const double* gam_pts) {
  if (n < 0) return axh::set_error(ASTERX_EARG, "points: n must be >= 0");
  if (!metric || !Bt) return axh::set_error(ASTERX_EARG, "points: NULL metric or field");
  if (!gam_pts && !(gam > 1.0)) return axh::set_error(ASTERX_EARG, "points: gamma must be > 1");
  return 0;
}

}  // namespace

extern "C" {

int asterx_prim2con_points(int64_t n, const double* gam_pts, double gam, const double* metric, const double* Bt,
                           const double* prim, double* cons, double* target, void* stream) {
  int rc;
  if ((rc = check_pts(n, metric, Bt, gam, gam_pts))) return rc;
  if (!prim || !cons) return axh::set_error(ASTERX_EARG, "prim2con_points: NULL array");
  if (n == 0) return 0;
  PtsIn a{n, gam_pts, gam, metric, Bt};
  hipLaunchKernelGGL(k_prim2con_points, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, a, prim, cons, target);
  return launched("prim2con_points: launch failed");
}

int asterx_mlp_features(int64_t n, const double* gam_pts, double gam, const double* metric, const double* Bt,
                        const double* cons, float* feat, void* stream) {
  int rc;
  if ((rc = check_pts(n, metric, Bt, gam, gam_pts))) return rc;
  if (!cons || !feat) return axh::set_error(ASTERX_EARG, "mlp_features: NULL array");
  if (n == 0) return 0;
  PtsIn a{n, gam_pts, gam, metric, Bt};
  hipLaunchKernelGGL(k_features_points, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, a, cons, feat);
  return launched("mlp_features: launch failed");
}

int asterx_mlp_forward(const asterx_mlp* m, int64_t n, const float* feat, float* out, void* stream) {
  Stdz z;
  if (!m || !m->params || !feat || !out) return axh::set_error(ASTERX_EARG, "mlp_forward: NULL argument");
  if (!stdz_from(m, z)) return axh::set_error(ASTERX_EARG, "mlp_forward: scales must be > 0");
  if (n < 0) return axh::set_error(ASTERX_EARG, "mlp_forward: n must be >= 0");
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_mlp_forward, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, m->params, (long long)n, feat,
                     z, out);
  return launched("mlp_forward: launch failed");
}

size_t asterx_mlp_grad_workspace_size(int64_t n) {
  if (n <= 0) return 0;
  return (size_t)((n + 63) / 64) * (NP + 1) * sizeof(float);
}

int asterx_mlp_grad(const asterx_mlp* m, int64_t n, const float* feat, const float* target, float* grad,
                    void* workspace, size_t ws_bytes, void* stream) {
  Stdz z;
  if (!m || !m->params || !feat || !target || !grad || !workspace)
    return axh::set_error(ASTERX_EARG, "mlp_grad: NULL argument");
  if (!stdz_from(m, z)) return axh::set_error(ASTERX_EARG, "mlp_grad: scales must be > 0");
  if (n <= 0) return axh::set_error(ASTERX_EARG, "mlp_grad: n must be > 0");
  if (ws_bytes < asterx_mlp_grad_workspace_size(n)) return axh::set_error(ASTERX_EARG, "mlp_grad: workspace too small");
  int nw = (int)((n + 63) / 64);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nw), dim3(64), 0, s, m->params, (long long)n, feat, target, z, 1.0f / (float)n,
                     (float*)workspace);
  int rc;
  if ((rc = launched("mlp_grad: launch failed"))) return rc;
  hipLaunchKernelGGL(k_mlp_reduce, dim3(nblk(NP + 1, 256)), dim3(256), 0, s, (const float*)workspace, nw, grad);
  return launched("mlp_grad: reduce launch failed");
}

int asterx_mlp_adam(float* params, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                    float eps, int32_t step, void* stream) {
  if (!params || !grad || !m || !v) return axh::set_error(ASTERX_EARG, "mlp_adam: NULL argument");
  if (step < 1) return axh::set_error(ASTERX_EARG, "mlp_adam: step counts from 1");
  float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(NP, 256)), dim3(256), 0, (hipStream_t)stream, params, grad, m, v, NP, lr, beta1,
                     beta2, eps, c1, c2);
  return launched("mlp_adam: launch failed");
}

int asterx_c2p_points(const asterx_params* p, int64_t n, const double* gam_pts, const double* metric,
                      const double* Bt, double* cons, const double* guess, const asterx_mlp* mlp, double* prim,
                      uint8_t* flags, int32_t* iters, unsigned long long* stats, void* stream) {
  int rc;
  if (!p) return axh::set_error(ASTERX_EARG, "c2p_points: NULL params");
  if ((rc = check_pts(n, metric, Bt, p->gamma, gam_pts))) return rc;
  if (!cons || !prim) return axh::set_error(ASTERX_EARG, "c2p_points: NULL array");
  if (!(p->c2p_tol > 0.0) || p->c2p_maxit < 1 || p->brent_maxit < 1 || !(p->wmax > 1.0) || !(p->rho_atm >= 0.0) ||
      p->c2p_method < 0 || p->c2p_method > 2)
    return axh::set_error(ASTERX_EARG, "c2p_points: invalid c2p parameters");
  C2PPtsArgs a;
  a.in = PtsIn{n, gam_pts, p->gamma, metric, Bt};
  a.cp.gam = p->gamma;
  a.cp.rho_atm = p->rho_atm;
  a.cp.k_atm = p->k_atm;
  a.cp.tol = p->c2p_tol;
  a.cp.wmax = p->wmax;
  a.cp.maxit = p->c2p_maxit;
  a.cp.brent_maxit = p->brent_maxit;
  a.cp.method = p->c2p_method;
  a.cons = cons;
  a.guess = guess;
  a.mlp = nullptr;
  if (mlp) {
    if (!mlp->params) return axh::set_error(ASTERX_EARG, "c2p_points: NULL network parameters");
    if (!stdz_from(mlp, a.z)) return axh::set_error(ASTERX_EARG, "c2p_points: network scales must be > 0");
    a.mlp = mlp->params;
  }
  a.prim = prim;
  a.flags = flags;
  a.iters = iters;
  a.stats = stats;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_c2p_points, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, a);
  return launched("c2p_points: launch failed");
}

}  // extern "C"
