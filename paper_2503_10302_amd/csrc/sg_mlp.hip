// sg_mlp.hip -- FP32 kernels of the ladder-predictor network
// (4 -> 64 -> 64 -> 33, ReLU; outputs: log beta_0, softplus increments of
// log beta_1..31, log ICM cutoff).  Tiny dense layers: plain VALU FMAs, one
// 64-lane work-group per sample chunk, no matrix cores.
#include <mutex>

#include "sg_internal.h"

namespace sg {

constexpr int NI = 4, NH = 64, NO = 33;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH;
constexpr int OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH;
constexpr int NPARAM = OFF_B3 + NO;   // 6625; then mean[4], std[4]

__device__ __forceinline__ float softplus_f(float x) { return x > 20.f ? x : log1pf(expf(x)); }
__device__ __forceinline__ float sigmoid_f(float x) { return 1.f / (1.f + expf(-x)); }

// Forward (and, with y != null, backward) over samples [blockIdx.x * per, ...).
// Each work-group accumulates its gradient into grad_acc + blockIdx.x * NPARAM
// (every element owned by one lane: no atomics, fixed summation order).
__global__ __launch_bounds__(64) void mlp_fwd_bwd_kernel(const float *P, const float *x,
                                                         const float *y, const int *idx, int batch,
                                                         int per, float *grad_acc, float *loss_acc,
                                                         float *out)
{
    __shared__ float xs[NI], a1[NH], a2[NH], dO[NO], dz2[NH], ys[NO], os[NO];
    const int i = threadIdx.x;
    const float *mean = P + NPARAM, *sd = P + NPARAM + NI;
    float *G = grad_acc ? grad_acc + (size_t)blockIdx.x * NPARAM : nullptr;
    if (G) {
        for (int k = 0; k < NI; ++k) G[OFF_W1 + i * NI + k] = 0.f;
        G[OFF_B1 + i] = 0.f;
        for (int k = 0; k < NH; ++k) G[OFF_W2 + i * NH + k] = 0.f;
        G[OFF_B2 + i] = 0.f;
        if (i < NO) {
            for (int k = 0; k < NH; ++k) G[OFF_W3 + i * NH + k] = 0.f;
            G[OFF_B3 + i] = 0.f;
        }
    }
    float lsum = 0.f;
    const int s0 = blockIdx.x * per, s1 = min(batch, s0 + per);
    for (int sm = s0; sm < s1; ++sm) {
        const int b = idx ? idx[sm] : sm;
        if (i < NI) xs[i] = (x[b * NI + i] - mean[i]) / sd[i];
        __syncthreads();
        float z1 = P[OFF_B1 + i];
        for (int k = 0; k < NI; ++k) z1 += P[OFF_W1 + i * NI + k] * xs[k];
        a1[i] = z1 > 0.f ? z1 : 0.f;
        __syncthreads();
        float z2 = P[OFF_B2 + i];
        for (int k = 0; k < NH; ++k) z2 += P[OFF_W2 + i * NH + k] * a1[k];
        a2[i] = z2 > 0.f ? z2 : 0.f;
        __syncthreads();
        if (i < NO) {
            float o = P[OFF_B3 + i];
            for (int k = 0; k < NH; ++k) o += P[OFF_W3 + i * NH + k] * a2[k];
            os[i] = o;
        }
        __syncthreads();
        if (i == 0) {
            float acc = os[0];
            ys[0] = acc;
            for (int k = 1; k < 32; ++k) {
                acc += softplus_f(os[k]);
                ys[k] = acc;
            }
            ys[32] = os[32];
        }
        __syncthreads();
        if (out && i < NO) out[(size_t)b * NO + i] = ys[i];
        if (!y) continue;
        if (i == 0) {
            // dL/dy = 2 (y - t) / (B * 33); back through the cumulative softplus
            float dy[NO];
            for (int k = 0; k < NO; ++k) {
                const float d = ys[k] - y[(size_t)b * NO + k];
                lsum += d * d;
                dy[k] = 2.f * d / (float)(batch * NO);
            }
            float suffix = 0.f;
            for (int k = 31; k >= 1; --k) {
                suffix += dy[k];
                dO[k] = sigmoid_f(os[k]) * suffix;
            }
            dO[0] = suffix + dy[0];
            dO[32] = dy[32];
        }
        __syncthreads();
        if (i < NO) {
            G[OFF_B3 + i] += dO[i];
            for (int k = 0; k < NH; ++k) G[OFF_W3 + i * NH + k] += dO[i] * a2[k];
        }
        float da2 = 0.f;
        for (int o = 0; o < NO; ++o) da2 += dO[o] * P[OFF_W3 + o * NH + i];
        dz2[i] = a2[i] > 0.f ? da2 : 0.f;
        __syncthreads();
        G[OFF_B2 + i] += dz2[i];
        for (int k = 0; k < NH; ++k) G[OFF_W2 + i * NH + k] += dz2[i] * a1[k];
        float da1 = 0.f;
        for (int o = 0; o < NH; ++o) da1 += dz2[o] * P[OFF_W2 + o * NH + i];
        const float dz1 = a1[i] > 0.f ? da1 : 0.f;
        G[OFF_B1 + i] += dz1;
        for (int k = 0; k < NI; ++k) G[OFF_W1 + i * NI + k] += dz1 * xs[k];
        __syncthreads();
    }
    if (loss_acc && i == 0) loss_acc[blockIdx.x] = lsum;
}

// Sum the per-work-group gradients (fixed order) into grad.
__global__ void mlp_reduce_kernel(const float *grad_acc, int nblk, float *grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += grad_acc[(size_t)b * NPARAM + p];
    grad[p] = s;
}

// Adam (Kingma & Ba) with bias correction.
__global__ void mlp_adam_kernel(float *P, const float *g, float *m, float *v, int n, float lr,
                                float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

hipError_t launch_mlp_pass(const float *P, const float *x, const float *y, const int *idx,
                           int batch, int nblk, float *grad_acc, float *loss_acc, float *out,
                           float *grad, hipStream_t s)
{
    const int per = (batch + nblk - 1) / nblk;
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(nblk), dim3(64), 0, s, P, x, y, idx, batch, per,
                       grad_acc, loss_acc, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !grad) return e;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, grad_acc,
                       nblk, grad);
    return hipGetLastError();
}

// Device memory of the allocation-free prediction entry point: the staging area of the
// network inputs (raw features, [kPredictMax][NI]) followed by the network outputs
// ([kPredictMax][NO]).  One copy per GPU, held until the process ends.  In host code the
// name below is only a stand-in: every host-side use goes through the address that
// hipGetSymbolAddress returns for the current device (mlp_scratch).
static __device__ __align__(256) float scratch[kPredictMax * (NI + NO)];
static_assert(kPredictScratchFloats == kPredictMax * (NI + NO), "scratch layout");

namespace {
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t mlp_scratch(float **p)
{
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (float *)a;
    }
    *p = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_mlp_adam2(float *P, const float *g, float *m, float *v, float lr, float b1,
                            float b2, float eps, int step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, g, m, v,
                       NPARAM, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace sg
