// mlp.hip -- node-wise learned predictor (an extension on top of the
// predictor of Sec. 3.2; the paper names learned surrogates only as related
// work in Sec. 1).  A 15 -> 64 -> 64 -> 3 network with GELU (tanh form) after
// each hidden layer estimates, node by node, the error of the Adams-Bashforth
// increment (u - u_AB); the AB4 increment plus that estimate is a second
// candidate guess, judged against the snapshot guess by initial residual.
// Algorithm 1 still refines the kept guess to the tolerance, so the network
// only changes the iteration count.
//
//   inference: BF16 weights and activations on v_mfma_f32_16x16x16bf16_1k with
//     FP32 accumulation.  The layers are computed transposed, H^T = W X^T, so
//     the MFMA output layout of one layer (lane l holds rows 4*(l/16)+v of
//     column l%16) is exactly the B-operand layout of the next one: no shuffles.
//     Weights stay in registers for a wave's whole grid-stride loop.
//   training: FP32 arithmetic with the BF16-rounded weights (straight-through
//     to the FP32 master copy), mean squared error, Adam; every reduction in a
//     fixed order, so gradients are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace ebe {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kIn = kMlpIn, kHid = kMlpHid, kOut = kMlpOut;
constexpr int oW1 = 0, oB1 = kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid;
static_assert(oB3 + kOut == kMlpParams, "parameter layout");

// Round to nearest even: the native conversion (v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ uint16_t to_bf16(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// GELU, tanh form: z/2 (1 + tanh(c (z + 0.044715 z^3))) = z - z / (exp(2u) + 1),
// with the hardware reciprocal (one v_rcp_f32 instead of a full division).
constexpr float kGeluC = 0.7978845608028654f;
__device__ __forceinline__ float gelu(float z) {
    const float u = kGeluC * fmaf(0.044715f * z, z * z, z);
    const float e = __expf(2.0f * u);
    return fmaf(-z, __builtin_amdgcn_rcpf(e + 1.0f), z);
}
// derivative: (1 + t)/2 + z (1 - t^2) c (1 + 3 * 0.044715 z^2) / 2, t = tanh(u)
__device__ __forceinline__ float gelu_grad(float z) {
    const float u = kGeluC * fmaf(0.044715f * z, z * z, z);
    const float e = __expf(2.0f * u);
    const float t = fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
    const float du = kGeluC * fmaf(3.0f * 0.044715f, z * z, 1.0f);
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * du;
}

__device__ __forceinline__ float wave_sum_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Feature k (0..14) of internal node n from the state, not scaled: the newest
// displacement u^{it-1} (k < 3); the increments u^{it-1-q} - u^{it-2-q},
// q = 0, 1, 2 (3 <= k < 12), which the average-acceleration scheme gives
// exactly as dt/2 (v^{it-1-q} + v^{it-2-q}) -- together the same information
// as the last four displacements, without the cancellation their differences
// would suffer in BF16; the force of the new step (k >= 12).
__device__ __forceinline__ double state_feature(const MlpState& S, int64_t n, int k) {
    const int m = k / 3, c = k % 3;
    const int64_t i = 3 * n + c;
    if (m == 4) {
        double f = -S.msum[n] * (c == 0 ? S.g0 : (c == 1 ? S.g1 : S.g2));
        if (S.f_int) f += S.f_int[i];
        return f;
    }
    if (m == 0) return S.u[i];
    const double* va = m == 1 ? S.v1 : (m == 2 ? S.v2 : S.v3);
    const double* vb = m == 1 ? S.v2 : (m == 2 ? S.v3 : S.v4);
    return S.hdt * (va[i] + vb[i]);
}

// ---------------------------------------------------------------------------
// inference
// ---------------------------------------------------------------------------
template <int SRC>   // 0: scaled features from an array; 1: from the solver state
__global__ __launch_bounds__(256) void k_mlp_infer(const uint16_t* __restrict__ w, MlpState S, const float* x,
                                                   float* y, int64_t n) {
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // A operands: lane holds A[col][4g+v] of each 16x16 tile
    v4s a1[4], a2[4][4], a3[4];
    v4f c1[4], c2[4], c3;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = 4 * g + v;
            a1[rb][v] = (short)(k < kIn ? w[oW1 + (16 * rb + col) * kIn + k] : 0);
            c1[rb][v] = from_bf16(w[oB1 + 16 * rb + 4 * g + v]);
            c2[rb][v] = from_bf16(w[oB2 + 16 * rb + 4 * g + v]);
            a3[rb][v] = (short)(col < kOut ? w[oW3 + col * kHid + 16 * rb + k] : 0);
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) a2[rb][kb][v] = (short)w[oW2 + (16 * rb + col) * kHid + 16 * kb + k];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) c3[v] = (4 * g + v < kOut) ? from_bf16(w[oB3 + 4 * g + v]) : 0.0f;

    for (int64_t t = wave; t * 16 < n; t += nwaves) {
        const int64_t node = t * 16 + col;
        const bool ok = node < n;
        v4s bx;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = 4 * g + v;
            float f = 0.0f;
            if (ok && k < kIn) {
                if (SRC == 0) f = x[node * kIn + k];
                else f = (float)(state_feature(S, node, k) * S.inv_s[mlp_group(k)]);
            }
            bx[v] = (short)to_bf16(f);
        }
        v4s b2[4], b3[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const v4f h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[rb], bx, c1[rb], 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) b2[rb][v] = (short)to_bf16(gelu(h[v]));
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            v4f acc = c2[rb];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[rb][kb], b2[kb], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) b3[rb][v] = (short)to_bf16(gelu(acc[v]));
        }
        v4f out = c3;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) out = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3[kb], b3[kb], out, 0, 0, 0);
        if (g == 0 && ok) {   // rows 0..2 of column col: the outputs of this node
            if (SRC == 0) {
                y[node * kOut] = out[0]; y[node * kOut + 1] = out[1]; y[node * kOut + 2] = out[2];
            } else {
                const uint8_t fm = S.fixmask[node];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double xs = S.xs[3 * node + c];
                    S.xl[3 * node + c] = (fm >> c) & 1 ? xs : xs + S.s_t * (double)out[c];
                }
            }
        }
    }
}

int infer_grid(int64_t n) {
    const int64_t tiles = (n + 15) / 16;
    const int64_t wg = (tiles + 3) / 4;   // 4 waves per workgroup, one tile each at least
    return (int)(wg < 2048 ? (wg > 0 ? wg : 1) : 2048);
}

// ---------------------------------------------------------------------------
// training (FP32)
// ---------------------------------------------------------------------------
// Forward over a batch, one sample per thread: scaled inputs X[16][B],
// pre-activations Z1, Z2 and activations H1, H2 ([64][B] each, sample
// fastest), dY = 2 (y - t) / (3 B) ([3][B]) and per-workgroup partial sums of
// the squared error.  Weights: the BF16-rounded values, staged in LDS.
__global__ __launch_bounds__(256) void k_mlp_fwd(MlpTrain T, int B, const int64_t* idx) {
    __shared__ float W[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) W[i] = from_bf16(T.w[i]);
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    float se = 0.0f;
    if (b < B) {
        float x[kIn], t[kOut];
        if (idx) {
            const int64_t r = idx[b];
            const float* s = T.samples + (r >= 0 && r < T.n_samples ? r : 0) * kMlpSample;
#pragma unroll
            for (int k = 0; k < kIn; ++k) x[k] = s[k] * T.inv_s[mlp_group(k)];
#pragma unroll
            for (int o = 0; o < kOut; ++o) t[o] = s[kIn + o] * T.inv_st;
        } else {
#pragma unroll
            for (int k = 0; k < kIn; ++k) x[k] = T.x_in[(int64_t)b * kIn + k];
#pragma unroll
            for (int o = 0; o < kOut; ++o) t[o] = T.t_in[(int64_t)b * kOut + o];
        }
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            x[k] = from_bf16(to_bf16(x[k]));   // the inputs as the MFMA inference takes them
            T.X[k * B + b] = x[k];
        }
        float h1[kHid];
#pragma unroll
        for (int i = 0; i < kHid; ++i) {
            float z = W[oB1 + i];
#pragma unroll
            for (int k = 0; k < kIn; ++k) z = fmaf(W[oW1 + i * kIn + k], x[k], z);
            T.Z1[i * B + b] = z;
            h1[i] = gelu(z);
            T.H1[i * B + b] = h1[i];
        }
        float y[kOut];
#pragma unroll
        for (int o = 0; o < kOut; ++o) y[o] = W[oB3 + o];
        for (int i = 0; i < kHid; ++i) {
            float z = W[oB2 + i];
#pragma unroll
            for (int j = 0; j < kHid; ++j) z = fmaf(W[oW2 + i * kHid + j], h1[j], z);
            T.Z2[i * B + b] = z;
            const float h2 = gelu(z);
            T.H2[i * B + b] = h2;
#pragma unroll
            for (int o = 0; o < kOut; ++o) y[o] = fmaf(W[oW3 + o * kHid + i], h2, y[o]);
        }
        const float sc = 2.0f / (3.0f * (float)B);
#pragma unroll
        for (int o = 0; o < kOut; ++o) {
            const float r = y[o] - t[o];
            se = fmaf(r, r, se);
            T.dY[o * B + b] = sc * r;
        }
    }
    // partial sum of squared errors of this workgroup (fixed order)
    __shared__ float red[4];
    float v = wave_sum_f(se);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) T.loss_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Backward through the activations, one sample per thread: dZ2 = (W3^T dY) . g'(Z2),
// dZ1 = (W2^T dZ2) . g'(Z1).
__global__ __launch_bounds__(256) void k_mlp_bwd(MlpTrain T, int B) {
    __shared__ float W[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) W[i] = from_bf16(T.w[i]);
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float dy[kOut];
#pragma unroll
    for (int o = 0; o < kOut; ++o) dy[o] = T.dY[o * B + b];
    float dh1[kHid];
#pragma unroll
    for (int j = 0; j < kHid; ++j) dh1[j] = 0.0f;
    for (int i = 0; i < kHid; ++i) {
        float dh2 = 0.0f;
#pragma unroll
        for (int o = 0; o < kOut; ++o) dh2 = fmaf(W[oW3 + o * kHid + i], dy[o], dh2);
        const float dz2 = dh2 * gelu_grad(T.Z2[i * B + b]);
        T.dZ2[i * B + b] = dz2;
#pragma unroll
        for (int j = 0; j < kHid; ++j) dh1[j] = fmaf(W[oW2 + i * kHid + j], dz2, dh1[j]);
    }
#pragma unroll
    for (int j = 0; j < kHid; ++j) T.dZ1[j * B + b] = dh1[j] * gelu_grad(T.Z1[j * B + b]);
}

// Weight gradients as sums over the batch of outer products, G[i][j] =
// sum_b A[i][b] C[j][b] for a 16 x 16 tile per workgroup (batch staged in LDS
// in chunks of 64, fixed summation order), plus bias gradients sum_b A[i][b]
// when C is null.
__global__ __launch_bounds__(256) void k_mlp_outer(const float* A, int rows, const float* Cm, int cols, int B,
                                                   float* G, int ldg) {
    __shared__ float sa[16][65], sc[16][65];
    const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
    const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
    float acc = 0.0f;
    for (int b0 = 0; b0 < B; b0 += 64) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int r = e >> 6, q = e & 63, b = b0 + q;
            sa[r][q] = (i0 + r < rows && b < B) ? A[(int64_t)(i0 + r) * B + b] : 0.0f;
            sc[r][q] = (j0 + r < cols && b < B) ? (Cm ? Cm[(int64_t)(j0 + r) * B + b] : 1.0f) : 0.0f;
        }
        __syncthreads();
#pragma unroll 16
        for (int q = 0; q < 64; ++q) acc = fmaf(sa[ti][q], sc[tj][q], acc);
        __syncthreads();
    }
    if (i0 + ti < rows && j0 + tj < cols) G[(int64_t)(i0 + ti) * ldg + j0 + tj] = acc;
}

// Adam on the FP32 master weights; refreshes the BF16 copy.  Workgroup 0 also
// sums the loss partials of the last forward into loss[step] (fixed order).
__global__ __launch_bounds__(256) void k_mlp_adam(float* wm, float* m, float* v, uint16_t* wb, const float* grad,
                                                  float lr, float c1, float c2, const float* loss_part, int n_part,
                                                  int B, double* loss, int step) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (wm && p < kMlpParams) {
        const float g = grad[p];
        const float mm = fmaf(0.9f, m[p], 0.1f * g);
        const float vv = fmaf(0.999f, v[p], 0.001f * g * g);
        m[p] = mm;
        v[p] = vv;
        const float w = wm[p] - lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
        wm[p] = w;
        wb[p] = to_bf16(w);
    }
    if (loss && blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n_part; ++i) s += (double)loss_part[i];
        loss[step] = s / (3.0 * B);
    }
}

__global__ void k_mlp_round(const float* wm, uint16_t* wb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) wb[p] = to_bf16(wm[p]);
}

// ---------------------------------------------------------------------------
// sample collection and scales
// ---------------------------------------------------------------------------
// Before the solve: keep the Adams-Bashforth increment of the sampled nodes.
__global__ void k_collect_pre(const int32_t* nodes, int k, const double* xs, double* stage) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const int64_t n = nodes[i];
    for (int c = 0; c < 3; ++c) stage[3 * i + c] = xs[3 * n + c];
}
// After the solve (before the state update): raw features and the target
// du - du_AB of the sampled nodes, appended as float rows of 18 values.
__global__ void k_collect_post(MlpState S, const int32_t* nodes, int k, const double* du, const double* stage,
                               float* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const int64_t n = nodes[i];
    float* o = out + (int64_t)i * kMlpSample;
    for (int f = 0; f < kIn; ++f) o[f] = (float)state_feature(S, n, f);
    for (int c = 0; c < 3; ++c) o[kIn + c] = (float)(du[3 * n + c] - stage[3 * i + c]);
}

// Root mean squares of each input group (newest displacement, increments,
// force) and of the targets over the collected samples (one workgroup,
// fixed order).
__global__ __launch_bounds__(256) void k_sample_rms(const float* s, int64_t count, double* out4) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t r = threadIdx.x; r < count; r += blockDim.x) {
        const float* q = s + r * kMlpSample;
        for (int f = 0; f < kMlpSample; ++f) a[f < kIn ? mlp_group(f) : 3] += (double)q[f] * q[f];
    }
    __shared__ double red[4][4];
    for (int g = 0; g < 4; ++g) {
        const double v = wave_sum_d(a[g]);
        if ((threadIdx.x & 63) == 0) red[g][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double n = (double)(count > 0 ? count : 1);
        const double width[4] = {3.0, 9.0, 3.0, 3.0};
        for (int g = 0; g < 4; ++g)
            out4[g] = sqrt(((red[g][0] + red[g][1]) + (red[g][2] + red[g][3])) / (width[g] * n));
    }
}

// User node ids -> internal ids; out-of-range ids raise the flag (and map to 0).
__global__ void k_map_nodes(const int32_t* user, int k, const int32_t* u2i, int64_t n, int32_t* out, int32_t* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const int32_t u = user[i];
    if (u < 0 || u >= n) {
        *flag = 1;
        out[i] = 0;
    } else {
        out[i] = u2i[u];
    }
}

__global__ void k_check_index(const int64_t* idx, int64_t m, int64_t limit, int32_t* flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (idx[i] < 0 || idx[i] >= limit) *flag = 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_mlp_infer_array(hipStream_t s, const uint16_t* w, int64_t n, const float* x, float* y) {
    MlpState S{};
    hipLaunchKernelGGL(k_mlp_infer<0>, dim3(infer_grid(n)), dim3(256), 0, s, w, S, x, y, n);
}

void launch_mlp_infer_state(hipStream_t s, const uint16_t* w, const MlpState& S, int64_t n) {
    hipLaunchKernelGGL(k_mlp_infer<1>, dim3(infer_grid(n)), dim3(256), 0, s, w, S, (const float*)nullptr,
                       (float*)nullptr, n);
}

void launch_mlp_grads(hipStream_t s, const MlpTrain& T, int B, const int64_t* idx) {
    const int nb = (B + 255) / 256;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(nb), dim3(256), 0, s, T, B, idx);
    hipLaunchKernelGGL(k_mlp_bwd, dim3(nb), dim3(256), 0, s, T, B);
    // weight gradients: dW1 = dZ1 X^T, dW2 = dZ2 H1^T, dW3 = dY H2^T, biases = row sums
    hipLaunchKernelGGL(k_mlp_outer, dim3(1, 4), dim3(256), 0, s, T.dZ1, kHid, T.X, kIn, B, T.grad + oW1, kIn);
    hipLaunchKernelGGL(k_mlp_outer, dim3(4, 4), dim3(256), 0, s, T.dZ2, kHid, T.H1, kHid, B, T.grad + oW2, kHid);
    hipLaunchKernelGGL(k_mlp_outer, dim3(4, 1), dim3(256), 0, s, T.dY, kOut, T.H2, kHid, B, T.grad + oW3, kHid);
    hipLaunchKernelGGL(k_mlp_outer, dim3(1, 4), dim3(256), 0, s, T.dZ1, kHid, (const float*)nullptr, 1, B,
                       T.grad + oB1, 1);
    hipLaunchKernelGGL(k_mlp_outer, dim3(1, 4), dim3(256), 0, s, T.dZ2, kHid, (const float*)nullptr, 1, B,
                       T.grad + oB2, 1);
    hipLaunchKernelGGL(k_mlp_outer, dim3(1, 1), dim3(256), 0, s, T.dY, kOut, (const float*)nullptr, 1, B,
                       T.grad + oB3, 1);
}

void launch_mlp_adam(hipStream_t s, const MlpTrain& T, const float* grad, float lr, int t, int B, double* loss,
                     int step) {
    const double c1 = 1.0 / (1.0 - std::pow(0.9, t)), c2 = 1.0 / (1.0 - std::pow(0.999, t));
    const int nb = B > 0 ? (B + 255) / 256 : 0;
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, T.wm, T.m, T.v, T.w, grad, lr,
                       (float)c1, (float)c2, (const float*)T.loss_part, nb, B, loss, step);
}

void launch_mlp_loss(hipStream_t s, const MlpTrain& T, int B, double* loss) {
    // loss of the last forward (no update)
    const int nb = (B + 255) / 256;
    hipLaunchKernelGGL(k_mlp_adam, dim3(1), dim3(64), 0, s, (float*)nullptr, (float*)nullptr, (float*)nullptr,
                       (uint16_t*)nullptr, (const float*)nullptr, 0.0f, 1.0f, 1.0f, (const float*)T.loss_part, nb, B,
                       loss, 0);
}

void launch_mlp_round(hipStream_t s, const float* wm, uint16_t* wb) {
    hipLaunchKernelGGL(k_mlp_round, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, wm, wb);
}

void launch_collect_pre(hipStream_t s, const int32_t* nodes, int k, const double* xs, double* stage) {
    hipLaunchKernelGGL(k_collect_pre, dim3((k + 255) / 256), dim3(256), 0, s, nodes, k, xs, stage);
}

void launch_collect_post(hipStream_t s, const MlpState& S, const int32_t* nodes, int k, const double* du,
                         const double* stage, float* out) {
    hipLaunchKernelGGL(k_collect_post, dim3((k + 255) / 256), dim3(256), 0, s, S, nodes, k, du, stage, out);
}

void launch_map_nodes(hipStream_t s, const int32_t* user, int k, const int32_t* u2i, int64_t n, int32_t* out,
                      int32_t* flag) {
    (void)hipMemsetAsync(flag, 0, sizeof(int32_t), s);
    hipLaunchKernelGGL(k_map_nodes, dim3((k + 255) / 256), dim3(256), 0, s, user, k, u2i, n, out, flag);
}

void launch_check_index(hipStream_t s, const int64_t* idx, int64_t m, int64_t limit, int32_t* flag) {
    (void)hipMemsetAsync(flag, 0, sizeof(int32_t), s);
    int64_t nb = (m + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_check_index, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s, idx, m, limit, flag);
}

void launch_sample_rms(hipStream_t s, const float* samples, int64_t count, double* out4) {
    hipLaunchKernelGGL(k_sample_rms, dim3(1), dim3(256), 0, s, samples, count, out4);
}

}  // namespace ebe
