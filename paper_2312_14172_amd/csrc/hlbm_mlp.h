// hlbm_mlp.h -- parameter layout and launchers of the surrogate-network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlbm {

// flat parameter vector: W1 (64x3), b1, W2 (64x64), b2, W3 (64x64), b3, W4 (64), b4
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = 192;
constexpr int MLP_OFF_W2 = 256;
constexpr int MLP_OFF_B2 = 4352;
constexpr int MLP_OFF_W3 = 4416;
constexpr int MLP_OFF_B3 = 8512;
constexpr int MLP_OFF_W4 = 8576;
constexpr int MLP_OFF_B4 = 8640;
constexpr int MLP_NPARAM = 8641;
constexpr int MLP_PARTIAL = MLP_NPARAM + 1;  // gradient + squared-error sum
constexpr int MLP_PACKED = 4 * 4096;         // bf16 entries of the four packed 64x64 operands
constexpr int MLP_LANE_F4 = 28;              // float4 forward parameters per lane group (after them)
constexpr int MLP_PACKED_BYTES = MLP_PACKED * 2 + 4 * MLP_LANE_F4 * 16;
constexpr int MLP_MAX_BLOCKS = 512;          // workgroups of one gradient launch

// Band grid of a family: the exact signed distance of its shape scaled to
// unit circumradius, at the centres of BAND_G^3 voxels covering
// [-BAND_HALF, BAND_HALF]^3 of the body frame (x fastest).  The table kernels
// use it to settle the cells whose distance is certainly beyond +-eps/2.
constexpr int BAND_G = 64;
constexpr double BAND_HALF = 1.25;
constexpr size_t BAND_BYTES = (size_t)BAND_G * BAND_G * BAND_G * sizeof(float);
hipError_t band_grid(int shape, double p0, double p1, const float4 *mesh, int mesh_nt, float *out, hipStream_t s);

hipError_t mlp_pack(const float *theta, __bf16 *packed, hipStream_t s);
hipError_t mlp_eval(const float *theta, const __bf16 *packed, const float *pts, float *out, int n, hipStream_t s);
hipError_t mlp_grad(const float *theta, const __bf16 *packed, const float4 *samples, int n, int nblocks,
                    float scale, float *partial, hipStream_t s);
int mlp_grad_blocks(int n, int nblocks);
// packed: with do_step, the packed operands to update in place (replaces a
// k_mlp_pack launch after the step), or NULL
hipError_t mlp_reduce_adam(float *theta, float *m, float *v, const float *partial, int nblocks, float *grad_out,
                           int do_step, float lr, int step, __bf16 *packed, hipStream_t s);
hipError_t mlp_samples(int shape, double p0, double p1, const float4 *mesh, int mesh_nt, uint64_t seed, int n,
                       double box, double band, double clip, double band_share, float4 *out, hipStream_t s);

}  // namespace hlbm
