// Kernels of the learned displacement correction (a 3-level 3-D U-Net on the particle lattice; the network is
// defined in include/lpc.h). Activations and their gradients are BF16, channels-last: element (voxel v, channel c)
// of a tensor view sits at base[v * ld + off + c], with v = (x D + y) D + z on a periodic D^3 grid. Weights are kept
// in FP32 (canonical layout W[Cout][taps][Cin], then b[Cout]) and converted to BF16 for the MFMA convolutions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lpc {
namespace net {

typedef __bf16 bf16;

// Network input channels: the displacement from the lattice and Psi1, both in lattice units.
constexpr int kInputChannels = 6;

struct View {        // a BF16 tensor view: base[v * ld + off + c]
  bf16* p;
  int ld, off;
};

// 3^3 circular convolution on BF16 MFMA (v_mfma_f32_16x16x32_bf16), FP32 accumulation. Implicit GEMM: rows are
// output voxels, k = tap * cin + ci (taps x-major, cin a multiple of 8), columns are output channels.
//   w: BF16 [16 nb][kpad] (kpad = 27 cin rounded up to 32; padding rows / columns zero)
//   bias: FP32 [cout] or NULL; leaky: apply leaky ReLU (slope 0.1)
//   out: BF16 view, or outf (FP32 [V][cout]) when outf != NULL. Only channels < cout are written.
//   mask, mask_ch (BF16 out only; mask_ch a multiple of 8): out channels c < mask_ch are multiplied by the leaky-ReLU
//   slope where the activation mask[v][c] is not positive, after rounding (the leaky-ReLU gradient, fused).
// The same kernel computes the data gradient of a convolution with the flipped, transposed weights.
hipError_t conv3(View in, int cin, const bf16* w, int kpad, int nb, const float* bias, int leaky, View out,
                 float* outf, int cout, int D, hipStream_t s, View mask = View{nullptr, 0, 0}, int mask_ch = 0);

// 2^3 stride-2 convolution (down) and transposed convolution (up), FP32 weights in the canonical layout.
//   down: out[y][o] = b[o] + sum_{t, i} W[o][t][i] x[2y + t][i]     (x on D^3, out on (D/2)^3)
//   up:   out[2y + t][o] = b[o] + sum_i W[o][t][i] x[y][i]          (x on D^3, out on (2D)^3)
hipError_t down2(View x, int cin, const float* W, const float* b, int cout, View out, int D, hipStream_t s);
hipError_t up2(View x, int cin, const float* W, const float* b, int cout, View out, int D, hipStream_t s);
// Data gradients on the same MFMA kernels, from the transposed weights Wt[i][t][o] (transpose2), shapes (cin, cout)
// (16, 32) and (32, 64) for down, (32, 16) and (64, 32) for up; accumulate adds into dx instead of overwriting it.
//   down: dx[2y + t][i] (+)= sum_o Wt[i][t][o] dz[y][o]       (dx on D^3, dz on (D/2)^3)
//   up:   dx[y][i] = sum_{t, o} Wt[i][t][o] dz[2y + t][o]      (dx on D^3, dz on (2D)^3)
// mask, mask_ch: the fused leaky-ReLU gradient as for conv3 (applied after the accumulation).
hipError_t down2_dgrad(View dz, int cout, const float* Wt, int cin, View dx, int D, int accumulate, hipStream_t s,
                       View mask = View{nullptr, 0, 0}, int mask_ch = 0);
hipError_t up2_dgrad(View dz, int cout, const float* Wt, int cin, View dx, int D, hipStream_t s,
                     View mask = View{nullptr, 0, 0}, int mask_ch = 0);
// Wt[i][t][o] = W[o][t][i] (FP32, cout x 8 x cin values)
hipError_t transpose2(const float* W, int cout, int cin, float* Wt, hipStream_t s);

// Weight gradients as per-chunk partial sums (deterministic): partial[chunk][W (canonical, cin_real input channels),
// then nslot bias slots of cout] with nslot = 8 for up2 (one per tap) and 1 otherwise. x has cin (a multiple of 8)
// channels of which the first cin_real are real.
//   kind 0: conv3 (x and dz on D^3), 1: down2 (x on D^3, dz on (D/2)^3), 2: up2 (x on D^3, dz on (2D)^3)
// wgrad_chunks gives the number of chunks (partial rows) that wgrad writes for these arguments.
int wgrad_chunks(int kind, int cin, int cout, int D);
hipError_t wgrad(int kind, View x, int cin, int cin_real, View dz, int cout, int D, float* partial, hipStream_t s);
// grad[0..nW) = sum over chunks; grad[nW + o] = sum over chunks and slots (over wgrad_chunks(...) chunks)
hipError_t reduce_partials(const float* partial, int nchunk, int nW, int cout, int nslot, float* grad,
                           hipStream_t s);

// Canonical FP32 weights of a 3^3 conv -> BF16 MFMA layouts: forward [16 nbo][kpad] with k = t cinp + ci, and
// flipped [16 nbi][kpadb] with k = t' coutp + o holding W[o][26 - t'][i] (the data-gradient convolution).
hipError_t convert_conv3(const float* W, int cout, int cin, bf16* wf, int cinp, int nbo, int kpad, bf16* wb,
                         int coutp, int nbi, int kpadb, hipStream_t s);

// Net input: FP32 features [V][6] -> BF16 [V][8] (channels 6, 7 zero).
hipError_t pack_input(const float* feat, bf16* x, int V, hipStream_t s);
// Loss gradient: dout BF16 [V][8] = 2 (out - target) / (3 V) (channels 3..7 zero); per-block sums of squared
// errors (double) in loss_part[nblocks].
int loss_blocks(int V);
hipError_t loss_grad(const float* out, const float* target, bf16* dout, double* loss_part, int V, hipStream_t s);

// Adam (Kingma & Ba 2015) with bias correction; t counts from 1.
hipError_t adam(float* p, float* m, float* v, const float* g, int64_t count, float lr, double beta1, double beta2,
                float eps, int64_t t, hipStream_t s);

// Lattice features of particles pos[3][n] with lattice ids: out[id][d] = minimal image (pos - base) / (L / N), base
// the lattice point of id (ref == NULL) or ref[3][n]; with psi1, also out[id][3 + d] = psi1[d][p] / (L / N) (row
// stride 6, else 3). flags[0] is set if an id is out of range.
hipError_t features(const float* pos, const int32_t* id, int64_t n, const float* ref, const float* psi1, int N,
                    double box, float* out, int* flags, hipStream_t s);
// The same six features (lattice base, psi1 required) written as the network input x[id] = BF16 [8] (channels 6, 7
// zero): what features followed by pack_input gives, in one pass.
hipError_t features_packed(const float* pos, const int32_t* id, int64_t n, const float* psi1, int N, double box,
                           bf16* x, int* flags, hipStream_t s);
// p[i] *= g for i < count.
hipError_t scale(float* p, int64_t count, float g, hipStream_t s);
// out = the k-th (0..47) symmetry of the cube applied to the lattice field in[N^3][C] of C / 3 vectors per site (k =
// 8 p + f: axis permutation p, reflection bits f; see lpc_net_symmetry). out must not overlap in.
hipError_t symmetry(const float* in, float* out, int N, int C, int k, hipStream_t s);
// pos = wrap(pos + r[id] L / N) for every particle.
hipError_t apply_residual(float* pos, const int32_t* id, int64_t n, const float* r, int N, double box, int* flags,
                          hipStream_t s);

}  // namespace net
}  // namespace lpc
