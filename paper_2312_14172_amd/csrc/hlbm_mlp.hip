// hlbm_mlp.hip -- BF16 matrix-core kernels of the signed-distance surrogate
// network used by the learned indicator (3 -> 64 -> 64 -> 64 -> 1, SiLU):
// exact-SDF training samples, forward + back-propagation, Adam, inference.
//
// Matrix products run on v_mfma_f32_16x16x32_bf16 in a transposed form:
// activations are kept as H^T (features x samples), one 16-sample tile per
// MFMA column block.  In that form a layer's accumulator layout (lane l holds
// rows 4(l/16)..4(l/16)+3 of a 16-row tile, column l%16) is already the B
// operand layout of the next layer's product once the contraction index is
// permuted: within a 32-feature chunk c, lane group g = l/16 and element
// e = 0..7 stand for feature kappa(c, g, e) = 32c + 4g + (e & 3) + 16 (e >> 2).
// The weight matrices are stored pre-permuted in that order, so no data moves
// between layers.  Weight-gradient products (contraction over samples) go
// through LDS to transpose activations and errors.
#include <algorithm>

#include "hlbm_device.h"
#include "hlbm_internal.h"
#include "hlbm_mlp.h"

namespace hlbm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline int kappa(int c, int g, int e) { return 32 * c + 4 * g + (e & 3) + 16 * (e >> 2); }

// SiLU and its derivative with the hardware reciprocal (1 ulp).
__device__ inline float sigm_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu_f(float z) { return z * sigm_f(z); }
__device__ inline float dsilu_f(float z) {
  const float s = sigm_f(z);
  return s * (1.0f + z * (1.0f - s));
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 16 C-layout values of a 64-feature column (index ot*4 + j = feature
// 16 ot + 4 g + j) -> the two bf16x8 B operands of chunks c = 0, 1.
__device__ inline void pack_b(const float *v, bf16x8 *b) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) b[c][e] = (__bf16)v[(2 * c + (e >> 2)) * 4 + (e & 3)];
}

// ---------------------------------------------------------------------------
// Weight packing (after every parameter update)
// ---------------------------------------------------------------------------
// wf[L][(ot*2 + c)*64 + lane][e] = W_L[16 ot + lane%16][kappa(c, lane/16, e)]  (forward, A = W)
// wb[L][(kt*2 + c)*64 + lane][e] = W_L[kappa(c, lane/16, e)][16 kt + lane%16]  (backward, A = W^T)
// followed by the FP32 parameters a lane of group g = lane/16 needs in the
// forward pass, as MLP_LANE_F4 float4 per group (features f = 16 ot + 4 g + j):
//   [4 ot + j] = (W1[f][0..2], b1[f]),  [16 + ot] = b2[f(j = 0..3)],
//   [20 + ot] = b3[..],  [24 + ot] = W4[..].
__global__ void k_mlp_pack(const float *__restrict__ theta, __bf16 *__restrict__ packed) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;  // 0 .. 4 * 4096 + 4 * MLP_LANE_F4 * 4
  if (t >= 4 * 4096) {
    const int r = t - 4 * 4096;
    if (r >= 4 * MLP_LANE_F4 * 4) return;
    const int comp = r % 4, slot = r / 4, g = slot / MLP_LANE_F4, k = slot % MLP_LANE_F4;
    float v;
    if (k < 16) {
      const int f = 16 * (k / 4) + 4 * g + k % 4;
      v = comp < 3 ? theta[MLP_OFF_W1 + 3 * f + comp] : theta[MLP_OFF_B1 + f];
    } else {
      const int ot = (k - 16) % 4, f = 16 * ot + 4 * g + comp;
      v = theta[(k < 20 ? MLP_OFF_B2 : (k < 24 ? MLP_OFF_B3 : MLP_OFF_W4)) + f];
    }
    ((float *)(packed + MLP_PACKED))[r] = v;
    return;
  }
  const int which = t / 4096;  // 0: wf2, 1: wf3, 2: wb2, 3: wb3
  const int r = t % 4096;
  const int e = r % 8, lane = (r / 8) % 64, c = (r / 512) % 2, tile = r / 1024;
  const float *W = theta + ((which & 1) ? MLP_OFF_W3 : MLP_OFF_W2);
  const int g = lane / 16, li = lane % 16;
  const int k = kappa(c, g, e);
  float v;
  if (which < 2) v = W[(16 * tile + li) * 64 + k];
  else v = W[k * 64 + 16 * tile + li];
  packed[t] = (__bf16)v;
}

struct MlpArgs {
  const float *theta;
  const bf16x8 *wf2, *wf3, *wb2, *wb3;
  const float4 *lane;  // per-lane-group forward parameters
};

__device__ inline MlpArgs mlp_args(const float *theta, const __bf16 *packed) {
  MlpArgs a;
  a.theta = theta;
  a.lane = (const float4 *)(packed + MLP_PACKED);
  a.wf2 = (const bf16x8 *)(packed);
  a.wf3 = (const bf16x8 *)(packed + 4096);
  a.wb2 = (const bf16x8 *)(packed + 2 * 4096);
  a.wb3 = (const bf16x8 *)(packed + 3 * 4096);
  return a;
}

// Forward pass of one 16-sample tile held by the wave: lane l holds sample
// l%16's input.  Outputs the pre-activations z1..z3 (C layout, 16 per lane)
// and y (replicated over the four lanes of each sample).
__device__ inline void mlp_forward_tile(const MlpArgs &A, float x0, float x1, float x2, float *z1, float *z2,
                                        float *z3, float &y) {
  const int l = threadIdx.x & 63, g = l >> 4;
  const float4 *P = A.lane + g * MLP_LANE_F4;
  float h[16];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float4 w = P[4 * ot + j];
      const float z = w.w + w.x * x0 + w.y * x1 + w.z * x2;
      z1[ot * 4 + j] = z;
      h[ot * 4 + j] = silu_f(z);
    }
  bf16x8 b[2];
  pack_b(h, b);
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(A.wf2[(ot * 2 + 0) * 64 + l], b[0], acc);
    acc = mfma(A.wf2[(ot * 2 + 1) * 64 + l], b[1], acc);
    const float4 bb = P[16 + ot];
    z2[ot * 4 + 0] = acc[0] + bb.x;
    z2[ot * 4 + 1] = acc[1] + bb.y;
    z2[ot * 4 + 2] = acc[2] + bb.z;
    z2[ot * 4 + 3] = acc[3] + bb.w;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) h[k] = silu_f(z2[k]);
  pack_b(h, b);
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(A.wf3[(ot * 2 + 0) * 64 + l], b[0], acc);
    acc = mfma(A.wf3[(ot * 2 + 1) * 64 + l], b[1], acc);
    const float4 bb = P[20 + ot];
    z3[ot * 4 + 0] = acc[0] + bb.x;
    z3[ot * 4 + 1] = acc[1] + bb.y;
    z3[ot * 4 + 2] = acc[2] + bb.z;
    z3[ot * 4 + 3] = acc[3] + bb.w;
  }
  float part = 0.f;
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    const float4 w4 = P[24 + ot];
    part += w4.x * silu_f(z3[ot * 4 + 0]) + w4.y * silu_f(z3[ot * 4 + 1]) + w4.z * silu_f(z3[ot * 4 + 2]) +
            w4.w * silu_f(z3[ot * 4 + 3]);
  }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  y = part + A.theta[MLP_OFF_B4];
}

// ---------------------------------------------------------------------------
// Inference: out[i] = network(pts[i]) for n points (normalised body frame).
// One wave per 64 points (four 16-point tiles).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_mlp_eval(const float *__restrict__ theta, const __bf16 *__restrict__ packed,
                                                 const float *__restrict__ pts, float *__restrict__ out, int n) {
  const MlpArgs A = mlp_args(theta, packed);
  const int l = threadIdx.x, g = l >> 4;
  for (int q = 0; q < 4; ++q) {
    const int s = blockIdx.x * 64 + q * 16 + (l & 15);
    const bool ok = s < n;
    const float x0 = ok ? pts[3 * s] : 0.f, x1 = ok ? pts[3 * s + 1] : 0.f, x2 = ok ? pts[3 * s + 2] : 0.f;
    float z1[16], z2[16], z3[16], y;
    mlp_forward_tile(A, x0, x1, x2, z1, z2, z3, y);
    if (ok && g == 0) out[s] = y;
  }
}

// ---------------------------------------------------------------------------
// Gradient of the mean-squared loss over a batch.  Two wavefronts per
// workgroup; workgroup b handles samples [b*per, (b+1)*per) in pairs of
// 16-sample tiles, wavefront q taking tile q of each pair, and writes its
// partial gradient (MLP_NPARAM floats) and squared-error sum.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_mlp_grad(const float *__restrict__ theta, const __bf16 *__restrict__ packed,
                                                  const float4 *__restrict__ samples, int n, int per, float scale,
                                                  float *__restrict__ partial) {
  __shared__ __attribute__((aligned(16))) __bf16 hT1[64][32], hT2[64][32], dT2[64][32], dT3[64][32];
  __shared__ float xfer[114 * 64];  // wavefront 1's per-lane sums
  const MlpArgs A = mlp_args(theta, packed);
  const float *th = theta;
  const int l = lane_id(), q = wave_id(), g = l >> 4, li = l & 15;
  float gW1[16][3], gb1[16], gb2[16], gb3[16], gW4[16], gb4 = 0.f, sse = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    gW1[k][0] = gW1[k][1] = gW1[k][2] = 0.f;
    gb1[k] = gb2[k] = gb3[k] = gW4[k] = 0.f;
  }
  // weight-gradient blocks (a, b) of the two 64x64 layers; wavefront q owns
  // the row blocks a = 2q, 2q + 1
  f32x4 dW2[2][4], dW3[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      dW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      dW3[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  const int s0 = blockIdx.x * per;
  const int s1 = min(n, s0 + per);
  for (int base = s0; base < s1; base += 32) {
    // the weight fragments and per-lane parameters are re-read (L1) for each
    // tile: hoisted out of the loop they would sit beside the 176 gradient
    // accumulators and push the kernel into scratch spills
    __asm__ volatile("" ::: "memory");
    {
      const int s = base + q * 16 + li;
      const bool ok = s < s1;
      const float4 smp = ok ? samples[s] : make_float4(0.f, 0.f, 0.f, 0.f);
      float z1[16], z2[16], z3[16], y;
      mlp_forward_tile(A, smp.x, smp.y, smp.z, z1, z2, z3, y);
      const float err = ok ? (y - smp.w) : 0.f;
      if (g == 0) sse += err * err;
      const float dy = scale * err;
      if (g == 0) gb4 += dy;
      // layer 4 and the error entering layer 3
      float d[16];
#pragma unroll
      for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = ot * 4 + j, f = 16 * ot + 4 * g + j;
          gW4[k] += dy * silu_f(z3[k]);
          d[k] = th[MLP_OFF_W4 + f] * dy * dsilu_f(z3[k]);
          gb3[k] += d[k];
          dT3[f][q * 16 + li] = (__bf16)d[k];
          hT2[f][q * 16 + li] = (__bf16)silu_f(z2[k]);
        }
      // error entering layer 2: W3^T d3
      bf16x8 b[2];
      pack_b(d, b);
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(A.wb3[(kt * 2 + 0) * 64 + l], b[0], acc);
        acc = mfma(A.wb3[(kt * 2 + 1) * 64 + l], b[1], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = kt * 4 + j, f = 16 * kt + 4 * g + j;
          d[k] = acc[j] * dsilu_f(z2[k]);
          gb2[k] += d[k];
          dT2[f][q * 16 + li] = (__bf16)d[k];
          hT1[f][q * 16 + li] = (__bf16)silu_f(z1[k]);
        }
      }
      // error entering layer 1: W2^T d2
      pack_b(d, b);
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(A.wb2[(kt * 2 + 0) * 64 + l], b[0], acc);
        acc = mfma(A.wb2[(kt * 2 + 1) * 64 + l], b[1], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = kt * 4 + j;
          const float d1 = acc[j] * dsilu_f(z1[k]);
          gb1[k] += d1;
          gW1[k][0] += d1 * smp.x;
          gW1[k][1] += d1 * smp.y;
          gW1[k][2] += d1 * smp.z;
        }
      }
    }
    // weight gradients of the two 64x64 layers: contraction over the 32
    // samples of the pair, operands transposed through LDS
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int ra = 16 * (2 * q + a) + li;
      const bf16x8 a3 = *(const bf16x8 *)&dT3[ra][8 * g];
      const bf16x8 a2 = *(const bf16x8 *)&dT2[ra][8 * g];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const bf16x8 b2 = *(const bf16x8 *)&hT2[16 * b + li][8 * g];
        const bf16x8 b1 = *(const bf16x8 *)&hT1[16 * b + li][8 * g];
        dW3[a][b] = mfma(a3, b2, dW3[a][b]);
        dW2[a][b] = mfma(a2, b1, dW2[a][b]);
      }
    }
    __syncthreads();
  }
  // ---- write this workgroup's partial gradient ------------------------
  float *out = partial + (size_t)blockIdx.x * MLP_PARTIAL;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * (2 * q + a) + 4 * g + j, col = 16 * b + li;
        out[MLP_OFF_W2 + row * 64 + col] = dW2[a][b][j];
        out[MLP_OFF_W3 + row * 64 + col] = dW3[a][b][j];
      }
  // per-lane sums of wavefront 1 added to wavefront 0's, then per-feature
  // sums over the 16 sample lanes of each lane group
  if (q == 1) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      xfer[(7 * k + 0) * 64 + l] = gb1[k];
      xfer[(7 * k + 1) * 64 + l] = gb2[k];
      xfer[(7 * k + 2) * 64 + l] = gb3[k];
      xfer[(7 * k + 3) * 64 + l] = gW4[k];
      xfer[(7 * k + 4) * 64 + l] = gW1[k][0];
      xfer[(7 * k + 5) * 64 + l] = gW1[k][1];
      xfer[(7 * k + 6) * 64 + l] = gW1[k][2];
    }
    xfer[112 * 64 + l] = gb4;
    xfer[113 * 64 + l] = sse;
  }
  __syncthreads();
  if (q == 1) return;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    float v[7] = {gb1[k], gb2[k], gb3[k], gW4[k], gW1[k][0], gW1[k][1], gW1[k][2]};
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      v[m] += xfer[(7 * k + m) * 64 + l];
      v[m] += __shfl_xor(v[m], 1, 64);
      v[m] += __shfl_xor(v[m], 2, 64);
      v[m] += __shfl_xor(v[m], 4, 64);
      v[m] += __shfl_xor(v[m], 8, 64);
    }
    if (li == 0) {
      const int f = 16 * (k / 4) + 4 * g + (k % 4);
      out[MLP_OFF_B1 + f] = v[0];
      out[MLP_OFF_B2 + f] = v[1];
      out[MLP_OFF_B3 + f] = v[2];
      out[MLP_OFF_W4 + f] = v[3];
      out[MLP_OFF_W1 + 3 * f + 0] = v[4];
      out[MLP_OFF_W1 + 3 * f + 1] = v[5];
      out[MLP_OFF_W1 + 3 * f + 2] = v[6];
    }
  }
  float v4[2] = {gb4 + xfer[112 * 64 + l], sse + xfer[113 * 64 + l]};
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v4[m] += __shfl_xor(v4[m], off, 64);
  if (l == 0) {
    out[MLP_OFF_B4] = v4[0];
    out[MLP_NPARAM] = v4[1];
  }
}

// Index within one packed 64x64 operand of the element that k_mlp_pack takes
// from row `tile` * 16 + li of its source and contraction index k (the
// inverse of kappa: k = 32 c + 16 (e >> 2) + 4 g + (e & 3)).
__device__ inline int packed_index(int tile, int li, int k) {
  const int c = k >> 5, rem = k & 31;
  const int g = (rem & 15) >> 2, e = (rem & 3) + 4 * (rem >> 4);
  return e + 8 * (16 * g + li) + 512 * c + 1024 * tile;
}

// Writes parameter p's value v to every place k_mlp_pack puts it (the same
// values and roundings as a full repack; b4 is read from theta directly).
__device__ inline void pack_param(__bf16 *__restrict__ packed, int p, float v) {
  float *lanef = (float *)(packed + MLP_PACKED);
  if ((p >= MLP_OFF_W2 && p < MLP_OFF_B2) || (p >= MLP_OFF_W3 && p < MLP_OFF_B3)) {
    const int L = p >= MLP_OFF_W3;
    const int q = p - (L ? MLP_OFF_W3 : MLP_OFF_W2), row = q >> 6, col = q & 63;
    const __bf16 b = (__bf16)v;
    packed[L * 4096 + packed_index(row >> 4, row & 15, col)] = b;        // forward, A = W
    packed[(2 + L) * 4096 + packed_index(col >> 4, col & 15, row)] = b;  // backward, A = W^T
  } else if (p < MLP_OFF_W2) {
    // W1[f][0..2] and b1[f]: float4 slot 4 ot + j of lane group g
    const int f = p < MLP_OFF_B1 ? p / 3 : p - MLP_OFF_B1, comp = p < MLP_OFF_B1 ? p % 3 : 3;
    const int g = (f & 15) >> 2, slot = g * MLP_LANE_F4 + 4 * (f >> 4) + (f & 3);
    lanef[4 * slot + comp] = v;
  } else if (p < MLP_OFF_B4) {
    // b2, b3, W4 [f]: component f & 3 of slot 16 / 20 / 24 + ot of group g
    const int which = p < MLP_OFF_W3 ? 0 : (p < MLP_OFF_W4 ? 1 : 2);
    const int f = p - (which == 0 ? MLP_OFF_B2 : (which == 1 ? MLP_OFF_B3 : MLP_OFF_W4));
    const int g = (f & 15) >> 2, slot = g * MLP_LANE_F4 + 16 + 4 * which + (f >> 4);
    lanef[4 * slot + (f & 3)] = v;
  }
}

// Sum the workgroup partials in a fixed order; optionally apply one Adam step
// (Kingma & Ba 2015, bias-corrected) to the FP32 master parameters and write
// the updated values into the packed operands (packed != NULL).  One
// workgroup per 64 parameters: wavefront w sums the partials w, w + 4, ...
// of its lane's parameter in increasing order (the loads issued 16 at a time
// ahead of the additions), and the four wavefront sums are added in order.
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(float *__restrict__ theta, float *__restrict__ m,
                                                         float *__restrict__ v, const float *__restrict__ partial,
                                                         int nblocks, float *__restrict__ grad_out, int do_step,
                                                         float lr, float b1, float b2, float eps, float bc1,
                                                         float bc2, __bf16 *__restrict__ packed) {
  __shared__ float part[4][64];
  const int lane = lane_id(), w = wave_id();
  const int p = blockIdx.x * 64 + lane;
  float gs = 0.f;
  if (p <= MLP_NPARAM) {
    int b = w;
    for (; b + 4 * 15 < nblocks; b += 4 * 16) {
      float x[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = partial[(size_t)(b + 4 * k) * MLP_PARTIAL + p];
#pragma unroll
      for (int k = 0; k < 16; ++k) gs += x[k];
    }
    for (; b < nblocks; b += 4) gs += partial[(size_t)b * MLP_PARTIAL + p];
  }
  part[w][lane] = gs;
  __syncthreads();
  if (w != 0 || p > MLP_NPARAM) return;
  const float gsum = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
  if (grad_out) grad_out[p] = gsum;
  if (!do_step || p == MLP_NPARAM) return;
  const float mn = b1 * m[p] + (1.f - b1) * gsum;
  const float vn = b2 * v[p] + (1.f - b2) * gsum * gsum;
  m[p] = mn;
  v[p] = vn;
  const float th = theta[p] - lr * (mn / bc1) / (sqrtf(vn / bc2) + eps);
  theta[p] = th;
  if (packed) pack_param(packed, p, th);
}

// ---------------------------------------------------------------------------
// Training samples from the exact signed distance (normalised units: the
// shape is scaled to circumradius 1).  Counter-based random numbers
// (splitmix64 of seed and sample index).  Samples are uniform in
// [-box, box]^3 except a share `band_share` that is redrawn until |d| <= band
// (at most 64 tries).
// ---------------------------------------------------------------------------
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__device__ inline double uniform01(uint64_t seed, uint64_t idx, int k) {
  return (double)(splitmix64(seed ^ splitmix64(idx * 64 + (uint64_t)k)) >> 11) * (1.0 / 9007199254740992.0);
}

__global__ void k_sdf_samples(int shape, double p0, double p1, const float4 *mesh, int mesh_nt, uint64_t seed, int n,
                              double box, double band, double clip, double band_share, float4 *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool want_band = uniform01(seed, i, 1000) < band_share;
  double x = 0, y = 0, z = 0, d = 0;
  for (int k = 0; k < 64; ++k) {
    x = (2.0 * uniform01(seed, i, 3 * k) - 1.0) * box;
    y = (2.0 * uniform01(seed, i, 3 * k + 1) - 1.0) * box;
    z = (2.0 * uniform01(seed, i, 3 * k + 2) - 1.0) * box;
    d = shape == 3 ? mesh_sdf<double>(mesh, mesh_nt, p0, x, y, z) : sdf_body<double>(shape, p0, p1, x, y, z);
    if (!want_band || fabs(d) <= band) break;
  }
  const double t = fmax(-clip, fmin(clip, d));
  out[i] = make_float4((float)x, (float)y, (float)z, (float)t);
}

// ---------------------------------------------------------------------------
// Band grid: the exact signed distance (FP64, stored in FP32) of the shape at
// unit circumradius at every voxel centre; one thread per voxel.
// ---------------------------------------------------------------------------
__global__ void k_band_grid(int shape, double p0, double p1, const float4 *mesh, int mesh_nt,
                            float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= BAND_G * BAND_G * BAND_G) return;
  const double h = 2.0 * BAND_HALF / BAND_G;
  const double x = -BAND_HALF + (i % BAND_G + 0.5) * h;
  const double y = -BAND_HALF + ((i / BAND_G) % BAND_G + 0.5) * h;
  const double z = -BAND_HALF + (i / (BAND_G * BAND_G) + 0.5) * h;
  out[i] = (float)(shape == 3 ? mesh_sdf<double>(mesh, mesh_nt, p0, x, y, z) : sdf_body<double>(shape, p0, p1, x, y, z));
}

// Settles a body-frame point b (in units of the circumradius rc) from the band
// grid: +1 where its distance is certainly above eps/2 (B = 0, outside), -1
// where certainly below -eps/2 (B = 1, inside), 0 where it must be evaluated.
// The signed distance is 1-Lipschitz, so it differs from the value d(v) at the
// voxel centre v by at most |b - v|; 1e-6 covers the FP32 rounding of d(v).
// Points off the grid are always evaluated.
__device__ inline int band_class(const float *__restrict__ band, double b0, double b1, double b2, double rc,
                                 double half_eps) {
  if (!band) return 0;
  const double ih = BAND_G / (2.0 * BAND_HALF), h = 2.0 * BAND_HALF / BAND_G;
  const double u0 = (b0 + BAND_HALF) * ih, u1 = (b1 + BAND_HALF) * ih, u2 = (b2 + BAND_HALF) * ih;
  if (!(u0 >= 0.0 && u0 < BAND_G && u1 >= 0.0 && u1 < BAND_G && u2 >= 0.0 && u2 < BAND_G)) return 0;
  const int i0 = (int)u0, i1 = (int)u1, i2 = (int)u2;
  const double v0 = b0 - (-BAND_HALF + (i0 + 0.5) * h), v1 = b1 - (-BAND_HALF + (i1 + 0.5) * h),
               v2 = b2 - (-BAND_HALF + (i2 + 0.5) * h);
  const double r2 = v0 * v0 + v1 * v1 + v2 * v2;
  const double d = (double)band[i0 + BAND_G * (i1 + BAND_G * i2)];
  const double e = half_eps / rc + 1e-6;
  // d - |b - v| > e  and  d + |b - v| < -e, without the square root
  const double out = d - e, in = -d - e;
  if (out > 0.0 && out * out > r2) return 1;
  if (in > 0.0 && in * in > r2) return -1;
  return 0;
}

// ---------------------------------------------------------------------------
// Distance tables over each particle's coupling box,
// tables[pid * cap + lx + sx (ly + sy lz)], for the particles read through a
// table (learned shapes, and mesh shapes without a network).  A cell is
// settled without evaluating the distance where it is certainly farther than
// eps/2 from the surface: outside R_c + eps/2 or, by the band grid, outside
// by more than eps/2 (entry +1e30, B = 0); inside r_in - eps/2 (r_in the
// inscribed radius) or, by the band grid, inside by more than eps/2 (entry
// -1e30, B = 1) -- the values the lattice kernel gives the cells it settles
// before reading a table.  The other cells are evaluated: by the network,
// R_c net(R^T (x - X) / R_c), or by the exact mesh distance.
//
// One workgroup of 256 threads per (chunk, particle); a particle's box is cut
// into nchunk contiguous chunks (more chunks when there are few particles, so
// that the launch fills the chip).  A chunk is classified 256 cells at a time,
// the cells to evaluate are appended to an LDS queue, and every 256 queued
// cells are evaluated by all threads at once (the network on full 16-cell
// tiles, the mesh distance on full wavefronts); the remainder at the end.
// Queue entries are box cell indices; the body-frame point is formed again
// from them in FP64.
// ---------------------------------------------------------------------------
constexpr int TAB_QUEUE = 512;

struct TableBox {
  int sx, sy, total;
  float isx, isxy;       // 1 / sx, 1 / (sx sy)
  double lo2, hi2, inv;  // early-out radii (as squares below), 1 / R_c
};

__device__ inline TableBox table_box(const Lattice &L, const DevParticle &p, double rin) {
  TableBox b;
  b.sx = p.hi[0] - p.lo[0] + 1;
  b.sy = p.hi[1] - p.lo[1] + 1;
  b.total = b.sx * b.sy * (p.hi[2] - p.lo[2] + 1);
  b.isx = 1.0f / (float)b.sx;
  b.isxy = 1.0f / (float)(b.sx * b.sy);
  b.lo2 = rin - 0.5 * L.eps;
  b.hi2 = p.rc + 0.5 * L.eps;
  b.inv = 1.0 / p.rc;
  return b;
}

// q = floor(i / m) for 0 <= i, 0 < m, from the FP32 product (i + 1/2) im
// (im = 1 / m in FP32) corrected by one step either way: the product is off
// by less than one while i < 2^22.
__device__ inline int div_fix(int i, int m, float im) {
  int q = (int)(((float)i + 0.5f) * im);
  const int r = i - q * m;
  q += r < 0 ? -1 : (r >= m ? 1 : 0);
  return q;
}

// Offset of box cell idx from the centre (box cells are unwrapped, so no
// minimum image is needed) and its body-frame image R^T d.
__device__ inline void table_point(const DevParticle &p, const TableBox &tb, int idx, double *d, double *bf) {
  const int zy = div_fix(idx, tb.sx, tb.isx), z = div_fix(idx, tb.sx * tb.sy, tb.isxy);
  d[0] = (p.lo[0] + (idx - zy * tb.sx) + 0.5) - p.X[0];
  d[1] = (p.lo[1] + (zy - z * tb.sy) + 0.5) - p.X[1];
  d[2] = (p.lo[2] + z + 0.5) - p.X[2];
  const double *R = p.R;
  bf[0] = R[0] * d[0] + R[3] * d[1] + R[6] * d[2];
  bf[1] = R[1] * d[0] + R[4] * d[1] + R[7] * d[2];
  bf[2] = R[2] * d[0] + R[5] * d[1] + R[8] * d[2];
}

// Classify the box cells [begin, end) and drain the queue through
// eval(queue, count): called by all 256 threads with count = 256 as the queue
// fills, then once with the rest (possibly 0).
template <class Eval>
__device__ inline void table_cells(const Lattice &L, const DevParticle &p, const TableBox &tb, int begin, int end,
                                   const float *__restrict__ band, float *__restrict__ tab, int *queue, int *wcnt,
                                   Eval eval) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  int queued = 0;  // uniform
  for (int base = begin; base < end; base += 256) {
    const int idx = base + t;
    bool q = false;
    if (idx < end) {
      double d[3], bf[3];
      table_point(p, tb, idx, d, bf);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      int cls;
      if (r2 > tb.hi2 * tb.hi2) cls = 1;
      else if (tb.lo2 > 0.0 && r2 < tb.lo2 * tb.lo2) cls = -1;
      else cls = band_class(band, bf[0] * tb.inv, bf[1] * tb.inv, bf[2] * tb.inv, p.rc, 0.5 * L.eps);
      if (cls != 0) tab[idx] = cls > 0 ? 1e30f : -1e30f;
      else q = true;
    }
    const unsigned long long mask = __ballot(q);
    if (l == 0) wcnt[w] = __popcll(mask);
    __syncthreads();
    int off = queued, added = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      off += k < w ? wcnt[k] : 0;
      added += wcnt[k];
    }
    if (q) queue[off + __popcll(mask & ((1ull << l) - 1ull))] = idx;
    queued += added;
    __syncthreads();
    if (queued >= 256) {
      eval(queue, 256);
      const int rest = queued - 256;
      const int keep = t < rest ? queue[256 + t] : 0;
      __syncthreads();
      if (t < rest) queue[t] = keep;
      queued = rest;
      __syncthreads();
    }
  }
  eval(queue, queued);
}

// Chunk blockIdx.x of nchunk of the box: [begin, end), whole 256-cell rounds.
__device__ inline void table_chunk(const TableBox &tb, int nchunk, int &begin, int &end) {
  const int per = ((tb.total + nchunk - 1) / nchunk + 255) / 256 * 256;
  begin = min(tb.total, (int)blockIdx.x * per);
  end = min(tb.total, begin + per);
}

// The occupancy hint caps the kernel at 86 VGPRs (no spills): 5 waves per SIMD
// instead of 4, 5 % faster on a 2000-particle 256^3 table launch.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_mlp_table(
    Lattice L, const DevParticle *__restrict__ parts, LearnedNets nets, int nchunk, float *__restrict__ tables,
    long long cap) {
  __shared__ int queue[TAB_QUEUE];
  __shared__ int wcnt[4];
  const DevParticle &p = parts[blockIdx.y];
  if (p.learned != 1) return;  // uniform per workgroup
  const int fam = min(max(p.shape - 1, 0), NFAM - 1);  // learned particles are shapes 1..3
  const MlpArgs A = mlp_args(nets.theta[fam], nets.packed[fam]);
  const double rin = p.shape == 2 ? fmin(p.prm[0], p.prm[1]) : (p.shape == 3 ? p.prm[2] : p.prm[0]);
  const TableBox tb = table_box(L, p, rin);
  int begin, end;
  table_chunk(tb, nchunk, begin, end);
  if (begin >= end) return;  // uniform per workgroup
  float *tab = tables + (size_t)blockIdx.y * cap;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, li = l & 15;
  // each wavefront evaluates its 64 queue entries as four 16-cell tiles
  table_cells(L, p, tb, begin, end, nets.band[fam], tab, queue, wcnt, [&](const int *qu, int count) {
    for (int q = 0; q < 4; ++q) {
      const int k = w * 64 + q * 16 + li;
      if (w * 64 + q * 16 >= count) break;  // uniform per wavefront
      // the per-lane parameters are re-read (L1) for every tile instead of
      // being hoisted out of the loop: that would hold ~110 more registers and
      // halve the waves per SIMD that hide the MFMA and SiLU latencies
      __asm__ volatile("" ::: "memory");
      const bool ok = k < count;
      const int idx = ok ? qu[k] : 0;
      float x0 = 0.f, x1 = 0.f, x2 = 0.f;
      if (ok) {
        double d[3], bf[3];
        table_point(p, tb, idx, d, bf);
        x0 = (float)(bf[0] * tb.inv);
        x1 = (float)(bf[1] * tb.inv);
        x2 = (float)(bf[2] * tb.inv);
      }
      float z1[16], z2[16], z3[16], y;
      mlp_forward_tile(A, x0, x1, x2, z1, z2, z3, y);
      if (ok && g == 0) tab[idx] = (float)(y * p.rc);
    }
  });
}

// Exact distance table of the mesh particles without a network (learned ==
// 2): the mesh's signed distance (FP64, stored in FP32), one queued cell per
// thread.
__global__ __launch_bounds__(256) void k_mesh_table(Lattice L, const DevParticle *__restrict__ parts,
                                                   const float *__restrict__ band, int nchunk,
                                                   float *__restrict__ tables, long long cap) {
  __shared__ int queue[TAB_QUEUE];
  __shared__ int wcnt[4];
  const DevParticle &p = parts[blockIdx.y];
  if (p.learned != 2) return;  // uniform per workgroup
  const TableBox tb = table_box(L, p, p.prm[2]);
  int begin, end;
  table_chunk(tb, nchunk, begin, end);
  if (begin >= end) return;  // uniform per workgroup
  float *tab = tables + (size_t)blockIdx.y * cap;
  table_cells(L, p, tb, begin, end, band, tab, queue, wcnt, [&](const int *qu, int count) {
    if ((int)threadIdx.x < count) {
      const int idx = qu[threadIdx.x];
      double d[3], bf[3];
      table_point(p, tb, idx, d, bf);
      tab[idx] = (float)mesh_sdf<double>(L.mesh, L.mesh_nt, p.prm[0], bf[0], bf[1], bf[2]);
    }
  });
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Chunks per particle box of the table kernels: about 2048 workgroups in all,
// at most one per 1024 cells of the largest box.
static int table_chunks(int n, long long cap) {
  const long long k = std::min<long long>((2048 + n - 1) / n, (cap + 1023) / 1024);
  return (int)std::max<long long>(1, k);
}

hipError_t launch_mesh_table(const Lattice &L, const DevParticle *parts, int n, const float *band, float *tables,
                             long long cap, hipStream_t s) {
  if (n <= 0 || !tables || L.mesh_nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mesh_table, dim3(table_chunks(n, cap), n), dim3(256), 0, s, L, parts, band,
                     table_chunks(n, cap), tables, cap);
  return hipGetLastError();
}

hipError_t band_grid(int shape, double p0, double p1, const float4 *mesh, int mesh_nt, float *out, hipStream_t s) {
  constexpr int nv = BAND_G * BAND_G * BAND_G;
  hipLaunchKernelGGL(k_band_grid, dim3((nv + 255) / 256), dim3(256), 0, s, shape, p0, p1, mesh, mesh_nt, out);
  return hipGetLastError();
}

hipError_t launch_mlp_table(const Lattice &L, const DevParticle *parts, int n, const LearnedNets &nets,
                            float *tables, long long cap, hipStream_t s) {
  if (n <= 0 || !tables) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_table, dim3(table_chunks(n, cap), n), dim3(256), 0, s, L, parts, nets,
                     table_chunks(n, cap), tables, cap);
  return hipGetLastError();
}

hipError_t mlp_pack(const float *theta, __bf16 *packed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((4 * 4096 + 4 * MLP_LANE_F4 * 4 + 255) / 256), dim3(256), 0, s, theta, packed);
  return hipGetLastError();
}

hipError_t mlp_eval(const float *theta, const __bf16 *packed, const float *pts, float *out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_eval, dim3((n + 63) / 64), dim3(64), 0, s, theta, packed, pts, out, n);
  return hipGetLastError();
}

hipError_t mlp_grad(const float *theta, const __bf16 *packed, const float4 *samples, int n, int nblocks,
                    float scale, float *partial, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int per = ((n + nblocks - 1) / nblocks + 31) / 32 * 32;
  const int nb = (n + per - 1) / per;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(128), 0, s, theta, packed, samples, n, per, scale, partial);
  return hipGetLastError();
}

int mlp_grad_blocks(int n, int nblocks) {
  const int per = ((n + nblocks - 1) / nblocks + 31) / 32 * 32;
  return (n + per - 1) / per;
}

hipError_t mlp_reduce_adam(float *theta, float *m, float *v, const float *partial, int nblocks, float *grad_out,
                           int do_step, float lr, int step, __bf16 *packed, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((MLP_NPARAM + 1 + 63) / 64), dim3(256), 0, s, theta, m, v, partial,
                     nblocks, grad_out, do_step, lr, b1, b2, 1e-8f, bc1, bc2, packed);
  return hipGetLastError();
}

hipError_t mlp_samples(int shape, double p0, double p1, const float4 *mesh, int mesh_nt, uint64_t seed, int n,
                       double box, double band, double clip, double band_share, float4 *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sdf_samples, dim3((n + 255) / 256), dim3(256), 0, s, shape, p0, p1, mesh, mesh_nt, seed, n,
                     box, band, clip, band_share, out);
  return hipGetLastError();
}

}  // namespace hlbm
