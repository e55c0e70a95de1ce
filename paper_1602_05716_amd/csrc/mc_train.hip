// mc_train.hip -- training of the delayed-acceptance surrogate on the GPU:
// bfloat16 matrix-core (MFMA) products with float accumulation, float
// master weights and Adam, behind mc_mlp_grad and mc_train_surrogate.
//
// The network (see include/mc.h): eps(phi) = b3 + w3 . bf16(relu(Z2)),
// Z2 = bf16(relu(Z1)) W2 + b2, Z1 = phi W1 + b1, phi the 128 neighbour
// histogram counts of a position.  The training loss of a batch of logged
// moves is mean((eps(phi_new) - eps(phi_old) - dE / l_B)^2); its gradient is
// formed by backpropagation, with the derivative of the bfloat16 rounding
// taken as 1.  Not in the paper: the learned first stage of a two-stage
// Metropolis test whose second stage is the paper's exact dE.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mc.h"
#include "mc_internal.hpp"

namespace {

constexpr int kIn = 128, kHid = 128;
constexpr int kNP = MC_DA_NPARAM;
// offsets of the flat parameter vector
constexpr int oW1 = 0, oB1 = oW1 + kIn * kHid, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid;
static_assert(oB3 + 1 == kNP, "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float v) {
    uint32_t b = __builtin_bit_cast(uint32_t, v);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// C[M x N] = op(A)[M x K] op(B)[K x N] (+ C if accumulate), bfloat16 inputs,
// float sums on the matrix cores.  op(A)[m][k] = ta ? A[k * lda + m] :
// A[m * lda + k]; op(B)[k][n] = tb ? B[n * ldb + k] : B[k * ldb + n].  A
// workgroup of 4 waves computes a 64 x 64 block, each wave a 32 x 32 tile
// with v_mfma_f32_32x32x8bf16_1k (lane l holds A[l % 32][4 (l / 32) + v],
// B[4 (l / 32) + v][l % 32], v = 0..3, and D[8 (r / 4) + 4 (l / 32) + r % 4]
// [l % 32], r = 0..15).  M and N multiples of 64, K a multiple of 8.
__global__ void __launch_bounds__(256)
gemm_bf16_kernel(const uint16_t* __restrict__ A, int lda, int ta, const uint16_t* __restrict__ B, int ldb, int tb,
                 float* __restrict__ C, int ldc, int K, int accumulate)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + (wave & 1) * 32, n0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int i = lane & 31, kq = (lane >> 5) * 4;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int k0 = 0; k0 < K; k0 += 8) {
        bf16x4 a, b;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = k0 + kq + v;
            a[v] = (short)(ta ? A[(size_t)k * lda + (m0 + i)] : A[(size_t)(m0 + i) * lda + k]);
            b[v] = (short)(tb ? B[(size_t)(n0 + i) * ldb + k] : B[(size_t)k * ldb + (n0 + i)]);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        float* dst = C + (size_t)row * ldc + (n0 + i);
        *dst = accumulate ? *dst + acc[r] : acc[r];
    }
}

// Batch rows from logged moves: row b = phi(x_i) of pair b, row B + b =
// phi(x~_i); counts as bfloat16 (exact); y[b] = dE / l_B.
__global__ void gather_kernel(const uint32_t* __restrict__ feat, const double* __restrict__ de,
                              const int64_t* __restrict__ idx, int B, double inv_lB, uint16_t* __restrict__ X,
                              float* __restrict__ y)
{
    const int b = blockIdx.x;
    const int64_t m = idx[b];
    for (int k = threadIdx.x; k < 2 * kIn; k += blockDim.x) {
        const uint32_t w = feat[m * 64 + (k >> 2)];
        const float c = (float)((w >> (8 * (k & 3))) & 0xFFu);
        const int row = k < kIn ? b : B + b;
        X[(size_t)row * kIn + (k & (kIn - 1))] = to_bf16(c);
    }
    if (threadIdx.x == 0) y[b] = (float)(de[m] * inv_lB);
}

// Same from host-given byte histograms [B][256] (gradient checks).
__global__ void gather_bytes_kernel(const uint8_t* __restrict__ f, int B, uint16_t* __restrict__ X)
{
    const int b = blockIdx.x;
    for (int k = threadIdx.x; k < 2 * kIn; k += blockDim.x) {
        const int row = k < kIn ? b : B + b;
        X[(size_t)row * kIn + (k & (kIn - 1))] = to_bf16((float)f[(size_t)b * 2 * kIn + k]);
    }
}

// Z += bias (in place, float); H = bf16(relu(Z)).
__global__ void bias_relu_kernel(float* __restrict__ Z, const float* __restrict__ bias, uint16_t* __restrict__ H,
                                 int rows)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)rows * kHid) return;
    const float z = Z[t] + bias[t % kHid];
    Z[t] = z;
    H[t] = to_bf16(z > 0.f ? z : 0.f);
}

// out[r] = b3 + sum_k H2[r][k] w3[k], k ascending.
__global__ void out_kernel(const uint16_t* __restrict__ H2, const float* __restrict__ w3, float b3,
                           float* __restrict__ out, int rows)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float o = b3;
    for (int k = 0; k < kHid; ++k) o = __builtin_fmaf(from_bf16(H2[(size_t)r * kHid + k]), w3[k], o);
    out[r] = o;
}

// Residuals, loss and the gradient with respect to the outputs.
__global__ void loss_kernel(const float* __restrict__ out, const float* __restrict__ y, int B,
                            float* __restrict__ dout, double* __restrict__ loss)
{
    __shared__ double part[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const float r = out[B + b] - out[b] - y[b];
        acc += (double)r * (double)r;
        const float g = 2.f * r / (float)B;
        dout[B + b] = g;
        dout[b] = -g;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / (double)B;
}

// dZ2[r][h] = dout[r] w3[h] [Z2 > 0] (float and bfloat16 copies).
__global__ void back_out_kernel(const float* __restrict__ dout, const float* __restrict__ w3,
                                const float* __restrict__ Z2, float* __restrict__ dZ2, uint16_t* __restrict__ dZ2b,
                                int rows)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)rows * kHid) return;
    const float g = Z2[t] > 0.f ? dout[t / kHid] * w3[t % kHid] : 0.f;
    dZ2[t] = g;
    dZ2b[t] = to_bf16(g);
}

// dZ1 = dH1 [Z1 > 0] (in place in dH1) and its bfloat16 copy.
__global__ void back_relu_kernel(float* __restrict__ dH, const float* __restrict__ Z, uint16_t* __restrict__ dHb,
                                 int rows)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)rows * kHid) return;
    const float g = Z[t] > 0.f ? dH[t] : 0.f;
    dH[t] = g;
    dHb[t] = to_bf16(g);
}

// Column sums of a [rows x 128] float matrix (bias gradients), and
// sum_r dout[r] H2[r][k] (w3 gradient) when H2 is given; one block per column.
__global__ void colsum_kernel(const float* __restrict__ M, const float* __restrict__ dout,
                              const uint16_t* __restrict__ H2, int rows, float* __restrict__ g)
{
    __shared__ float part[256];
    const int k = blockIdx.x;
    float acc = 0.f;
    for (int r = threadIdx.x; r < rows; r += blockDim.x)
        acc += H2 ? dout[r] * from_bf16(H2[(size_t)r * kHid + k]) : M[(size_t)r * kHid + k];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) g[k] = part[0];
}

__global__ void sum_kernel(const float* __restrict__ v, int n, float* __restrict__ out)
{
    __shared__ float part[256];
    float acc = 0.f;
    for (int r = threadIdx.x; r < n; r += blockDim.x) acc += v[r];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

// Adam on the float master weights; refreshes the bfloat16-valued working
// copy (float) and the bfloat16 matrices of both hidden layers.
__global__ void adam_kernel(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                            float c2, float* __restrict__ Pw, uint16_t* __restrict__ W1b, uint16_t* __restrict__ W2b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float p = P[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    P[t] = p;
    const uint16_t hb = to_bf16(p);
    Pw[t] = from_bf16(hb);
    if (t >= oW1 && t < oB1) W1b[t - oW1] = hb;
    if (t >= oW2 && t < oB2) W2b[t - oW2] = hb;
}

// Working copies from float master weights (bfloat16 values).
__global__ void refresh_kernel(const float* __restrict__ P, int n, float* __restrict__ Pw, uint16_t* __restrict__ W1b,
                               uint16_t* __restrict__ W2b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint16_t hb = to_bf16(P[t]);
    Pw[t] = from_bf16(hb);
    if (t >= oW1 && t < oB1) W1b[t - oW1] = hb;
    if (t >= oW2 && t < oB2) W2b[t - oW2] = hb;
}

// Device workspace of the network for batches of up to Bmax pairs.
struct Net {
    int Bmax = 0;
    float *P = nullptr, *Pw = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t *W1b = nullptr, *W2b = nullptr;
    uint16_t *X = nullptr, *H1 = nullptr, *H2 = nullptr, *dZ2b = nullptr, *dZ1b = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *out = nullptr, *dout = nullptr, *dZ2 = nullptr, *dH1 = nullptr, *y = nullptr;
    int64_t* idx = nullptr;
    double* loss = nullptr;
    std::vector<void*> all;
    hipStream_t s = nullptr;

    template <typename Q>
    bool get(Q** p, size_t bytes) {
        void* q = nullptr;
        if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) return false;
        all.push_back(q);
        *p = (Q*)q;
        return true;
    }
    // every buffer of a batch of B moves (the optimizer's moments only when
    // training), each obtained from take(&pointer, bytes)
    template <typename Take>
    static bool layout(Net& n, int B, bool train, Take&& take) {
        const size_t R = 2 * (size_t)B;
        return take(&n.P, 4 * kNP) && take(&n.Pw, 4 * kNP) && (!train || (take(&n.m, 4 * kNP) && take(&n.v, 4 * kNP))) &&
               take(&n.g, 4 * kNP) && take(&n.W1b, 2 * kIn * kHid) && take(&n.W2b, 2 * kHid * kHid) &&
               take(&n.X, 2 * R * kIn) && take(&n.H1, 2 * R * kHid) && take(&n.H2, 2 * R * kHid) &&
               take(&n.dZ2b, 2 * R * kHid) && take(&n.dZ1b, 2 * R * kHid) && take(&n.Z1, 4 * R * kHid) &&
               take(&n.Z2, 4 * R * kHid) && take(&n.out, 4 * R) && take(&n.dout, 4 * R) &&
               take(&n.dZ2, 4 * R * kHid) && take(&n.dH1, 4 * R * kHid) && take(&n.y, 4 * (size_t)B) &&
               take(&n.idx, 8 * (size_t)B) && take(&n.loss, 8);
    }
    bool init(int B, hipStream_t stream) {
        Bmax = B;
        s = stream;
        return layout(*this, B, true, [this](auto** p, size_t bytes) { return get(p, bytes); });
    }
    // the buffers of a gradient pass (no optimizer moments) carved out of
    // caller-provided device memory [base, base + cap); nothing is allocated
    // and nothing is freed by the destructor
    bool carve(int B, unsigned char* base, size_t cap, size_t* used) {
        Bmax = B;
        size_t at = 0;
        auto take = [&](auto** p, size_t bytes) {
            const size_t a = (bytes + 255) & ~(size_t)255;
            if (at + a > cap) return false;
            *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(base + at);
            at += a;
            return true;
        };
        const bool ok = layout(*this, B, false, take);
        *used = at;
        return ok;
    }
    ~Net() {
        if (s) (void)hipStreamSynchronize(s);
        for (void* q : all) (void)hipFree(q);
    }
    bool upload_params(const std::vector<float>& p) {
        if (hipMemcpy(P, p.data(), 4 * kNP, hipMemcpyHostToDevice) != hipSuccess) return false;
        if (m && hipMemset(m, 0, 4 * kNP) != hipSuccess) return false;
        if (v && hipMemset(v, 0, 4 * kNP) != hipSuccess) return false;
        hipLaunchKernelGGL(refresh_kernel, dim3((kNP + 255) / 256), dim3(256), 0, s, P, kNP, Pw, W1b, W2b);
        return hipGetLastError() == hipSuccess;
    }
    void gemm(const uint16_t* A, int lda, int ta, const uint16_t* B, int ldb, int tb, float* C, int ldc, int M, int N,
              int K, int accumulate) {
        hipLaunchKernelGGL(gemm_bf16_kernel, dim3(M / 64, N / 64), dim3(256), 0, s, A, lda, ta, B, ldb, tb, C, ldc, K,
                           accumulate);
    }
    // forward over the R = 2B rows of X
    void forward(int B) {
        const int R = 2 * B;
        const int ew = (R * kHid + 255) / 256;
        gemm(X, kIn, 0, W1b, kHid, 0, Z1, kHid, R, kHid, kIn, 0);
        hipLaunchKernelGGL(bias_relu_kernel, dim3(ew), dim3(256), 0, s, Z1, Pw + oB1, H1, R);
        gemm(H1, kHid, 0, W2b, kHid, 0, Z2, kHid, R, kHid, kHid, 0);
        hipLaunchKernelGGL(bias_relu_kernel, dim3(ew), dim3(256), 0, s, Z2, Pw + oB2, H2, R);
    }
    void outputs(int B, float b3) {
        const int R = 2 * B;
        hipLaunchKernelGGL(out_kernel, dim3((R + 255) / 256), dim3(256), 0, s, H2, Pw + oW3, b3, out, R);
    }
    // loss and gradient (into g) of the batch in X / y
    void backward(int B) {
        const int R = 2 * B;
        const int ew = (R * kHid + 255) / 256;
        hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, out, y, B, dout, loss);
        hipLaunchKernelGGL(colsum_kernel, dim3(kHid), dim3(256), 0, s, nullptr, dout, H2, R, g + oW3);
        hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, dout, R, g + oB3);
        hipLaunchKernelGGL(back_out_kernel, dim3(ew), dim3(256), 0, s, dout, Pw + oW3, Z2, dZ2, dZ2b, R);
        hipLaunchKernelGGL(colsum_kernel, dim3(kHid), dim3(256), 0, s, dZ2, nullptr, nullptr, R, g + oB2);
        gemm(H1, kHid, 1, dZ2b, kHid, 0, g + oW2, kHid, kHid, kHid, R, 0);   // dW2 = H1^T dZ2
        gemm(dZ2b, kHid, 0, W2b, kHid, 1, dH1, kHid, R, kHid, kHid, 0);      // dH1 = dZ2 W2^T
        hipLaunchKernelGGL(back_relu_kernel, dim3(ew), dim3(256), 0, s, dH1, Z1, dZ1b, R);
        hipLaunchKernelGGL(colsum_kernel, dim3(kHid), dim3(256), 0, s, dH1, nullptr, nullptr, R, g + oB1);
        gemm(X, kIn, 1, dZ1b, kHid, 0, g + oW1, kHid, kIn, kHid, R, 0);      // dW1 = X^T dZ1
    }
};

float round_bf16_host(double v) {
    float f = (float)v;
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    b &= 0xFFFF0000u;
    std::memcpy(&f, &b, 4);
    return f;
}

thread_local std::string g_train_error = "no error";

// Records why a handle-free call failed, for mc_last_error(NULL); returns code.
int noalloc_fail(int code, const std::string& msg) {
    g_train_error = msg;
    mc_internal_note_error(msg.c_str());
    return code;
}

// Bytes of the buffers Net::carve takes for a gradient pass of B moves plus
// the staged byte histograms (each piece rounded up to 256 bytes).
constexpr size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t grad_pass_bytes(int B) {
    const size_t R = 2 * (size_t)B;
    return 3 * round256(4 * (size_t)kNP) + round256(2 * kIn * kHid) + round256(2 * kHid * kHid) +
           round256(2 * R * kIn) + 4 * round256(2 * R * kHid) + 4 * round256(4 * R * kHid) + 2 * round256(4 * R) +
           round256(4 * (size_t)B) + round256(8 * (size_t)B) + round256(8) + round256((size_t)B * 2 * kIn);
}

// Largest batch of mc_mlp_grad_noalloc and its device workspace: one
// file-scope array, about 2.2 MB, that every GPU the library runs on holds
// until the process ends.  Host code never names it directly: its device
// address comes from hipGetSymbolAddress, once per device.
constexpr int kNoAllocBatch = MC_NOALLOC_MAX_BATCH;
constexpr size_t kScratchBytes = grad_pass_bytes(kNoAllocBatch);
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up on the device's first
// call; nullptr (and the reason in g_train_error) on failure.
unsigned char* device_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        g_train_error = "no usable current HIP device";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_train_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_ptr[dev] = (unsigned char*)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int mc_mlp_grad(int32_t batch, const uint8_t* feats, const double* target, const double* params, double* loss,
                double* grad) {
    if (batch < 32 || batch % 32 != 0 || !feats || !target || !params)
        return MC_E_ARG;
    std::vector<float> p(kNP);
    for (int k = 0; k < kNP; ++k) {
        if (!std::isfinite(params[k])) return MC_E_ARG;
        p[k] = (float)params[k];
    }
    Net net;
    if (!net.init(batch, nullptr)) return MC_E_OOM;
    if (!net.upload_params(p)) return MC_E_DEVICE;
    uint8_t* dfeat = nullptr;
    if (!net.get(&dfeat, (size_t)batch * 2 * kIn)) return MC_E_OOM;
    std::vector<float> y(batch);
    for (int b = 0; b < batch; ++b) y[b] = (float)target[b];
    if (hipMemcpy(dfeat, feats, (size_t)batch * 2 * kIn, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net.y, y.data(), 4 * (size_t)batch, hipMemcpyHostToDevice) != hipSuccess)
        return MC_E_DEVICE;
    hipLaunchKernelGGL(gather_bytes_kernel, dim3(batch), dim3(256), 0, nullptr, dfeat, batch, net.X);
    net.forward(batch);
    net.outputs(batch, round_bf16_host(params[oB3]));
    net.backward(batch);
    if (hipDeviceSynchronize() != hipSuccess || hipGetLastError() != hipSuccess) return MC_E_DEVICE;
    std::vector<float> g(kNP);
    double l = 0.0;
    if (hipMemcpy(g.data(), net.g, 4 * kNP, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&l, net.loss, 8, hipMemcpyDeviceToHost) != hipSuccess)
        return MC_E_DEVICE;
    if (loss) *loss = l;
    if (grad)
        for (int k = 0; k < kNP; ++k) grad[k] = g[k];
    return MC_OK;
}

int mc_mlp_grad_noalloc(int32_t batch, const uint8_t* feats, const double* target, const double* params,
                        double* loss, double* grad) {
    if (batch < 32 || batch % 32 != 0 || !feats || !target || !params)
        return noalloc_fail(MC_E_ARG, "batch must be a positive multiple of 32, and feats, target and params given");
    if (batch > kNoAllocBatch)
        return noalloc_fail(MC_E_ARG, "batch " + std::to_string(batch) + " exceeds the workspace's " +
                                          std::to_string(kNoAllocBatch) + " moves (MC_NOALLOC_MAX_BATCH)");
    std::vector<float> p(kNP);
    for (int k = 0; k < kNP; ++k) {
        if (!std::isfinite(params[k])) return noalloc_fail(MC_E_ARG, "non-finite parameter");
        p[k] = (float)params[k];
    }
    unsigned char* ws = device_scratch();
    if (!ws) return noalloc_fail(MC_E_DEVICE, g_train_error);
    Net net;
    size_t used = 0;
    uint8_t* dfeat = nullptr;
    if (!net.carve(batch, ws, kScratchBytes, &used) ||
        used + round256((size_t)batch * 2 * kIn) > kScratchBytes)
        return noalloc_fail(MC_E_STATE, "the buffers of the pass do not fit the workspace");
    dfeat = ws + used;
    if (!net.upload_params(p)) return noalloc_fail(MC_E_DEVICE, "parameter upload failed");
    std::vector<float> y(batch);
    for (int b = 0; b < batch; ++b) y[b] = (float)target[b];
    if (hipMemcpy(dfeat, feats, (size_t)batch * 2 * kIn, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net.y, y.data(), 4 * (size_t)batch, hipMemcpyHostToDevice) != hipSuccess)
        return noalloc_fail(MC_E_DEVICE, "input upload failed");
    hipLaunchKernelGGL(gather_bytes_kernel, dim3(batch), dim3(256), 0, nullptr, dfeat, batch, net.X);
    net.forward(batch);
    net.outputs(batch, round_bf16_host(params[oB3]));
    net.backward(batch);
    if (hipDeviceSynchronize() != hipSuccess || hipGetLastError() != hipSuccess)
        return noalloc_fail(MC_E_DEVICE, "the gradient pass failed on the device");
    std::vector<float> g(kNP);
    double l = 0.0;
    if (hipMemcpy(g.data(), net.g, 4 * kNP, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&l, net.loss, 8, hipMemcpyDeviceToHost) != hipSuccess)
        return noalloc_fail(MC_E_DEVICE, "output download failed");
    if (loss) *loss = l;
    if (grad)
        for (int k = 0; k < kNP; ++k) grad[k] = g[k];
    return MC_OK;
}

int mc_train_surrogate(mc_handle* h, int32_t chain, int64_t n_moves, int32_t epochs, int32_t batch, double lr,
                       uint64_t seed, const double* params_in, double* params_out, double* loss_out,
                       double* val_loss, double* ref_stage2_reject) {
    if (!h) return MC_E_ARG;
    if (epochs < 1 || batch < 32 || batch % 32 != 0 || !(lr > 0) || !params_out)
        return mc_internal_fail(h, MC_E_ARG, "need epochs >= 1, batch a multiple of 32, lr > 0, params_out");
    MCLogView lg;
    int rc = mc_internal_log(h, chain, &lg);
    if (rc) return rc;
    if (n_moves < 1 || n_moves > lg.cap) return mc_internal_fail(h, MC_E_ARG, "n_moves exceeds the log");
    // usable moves: logged, no conflict, no wall or overlap rejection
    std::vector<uint8_t> flags((size_t)n_moves);
    std::vector<double> de((size_t)n_moves);
    if (hipMemcpy(flags.data(), lg.flags, (size_t)n_moves, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(de.data(), lg.de, 8 * (size_t)n_moves, hipMemcpyDeviceToHost) != hipSuccess)
        return mc_internal_fail(h, MC_E_DEVICE, "log download failed");
    std::vector<int64_t> use;
    for (int64_t k = 0; k < n_moves; ++k)
        if ((flags[k] & 0x80) && !(flags[k] & 0x07)) use.push_back(k);
    if ((int64_t)use.size() < 2 * batch) return mc_internal_fail(h, MC_E_ARG, "too few usable logged moves");
    // the last tenth of the usable moves is held out
    const int64_t n_val = std::max<int64_t>(batch, (int64_t)use.size() / 10) / batch * batch;
    const int64_t n_tr = ((int64_t)use.size() - n_val) / batch * batch;
    std::vector<int64_t> tr(use.begin(), use.begin() + n_tr), va(use.end() - n_val, use.end());
    std::mt19937_64 rng(seed);
    std::vector<float> p(kNP);
    if (params_in) {
        for (int k = 0; k < kNP; ++k) p[k] = (float)params_in[k];
    } else {
        // He initialisation of the weights, zero biases
        std::normal_distribution<double> nd(0.0, 1.0);
        for (int k = 0; k < kNP; ++k) {
            const double sd = k < oB1 ? std::sqrt(2.0 / kIn) : (k >= oW2 && k < oB2) ? std::sqrt(2.0 / kHid)
                              : (k >= oW3 && k < oB3) ? std::sqrt(1.0 / kHid) : 0.0;
            p[k] = (float)(sd * nd(rng));
        }
    }
    Net net;
    if (!net.init(batch, lg.stream)) return mc_internal_fail(h, MC_E_OOM, "training workspace");
    if (!net.upload_params(p)) return mc_internal_fail(h, MC_E_DEVICE, "parameter upload");
    const double inv_lB = lg.lB > 0 ? 1.0 / lg.lB : 1.0;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float c1 = 1.f, c2 = 1.f;
    double last = 0.0;
    for (int e = 0; e < epochs; ++e) {
        std::shuffle(tr.begin(), tr.end(), rng);
        double acc = 0.0;
        for (int64_t b0 = 0; b0 < n_tr; b0 += batch) {
            if (hipMemcpyAsync(net.idx, tr.data() + b0, 8 * (size_t)batch, hipMemcpyHostToDevice, net.s) != hipSuccess)
                return mc_internal_fail(h, MC_E_DEVICE, "index upload");
            hipLaunchKernelGGL(gather_kernel, dim3(batch), dim3(256), 0, net.s, lg.feat, lg.de, net.idx, batch, inv_lB,
                               net.X, net.y);
            net.forward(batch);
            // b3 cancels in the difference of the two outputs: keep it at its value
            net.outputs(batch, 0.f);
            net.backward(batch);
            c1 *= b1;
            c2 *= b2;
            hipLaunchKernelGGL(adam_kernel, dim3((kNP + 255) / 256), dim3(256), 0, net.s, net.P, net.m, net.v, net.g, kNP,
                               (float)lr, b1, b2, eps, 1.f - c1, 1.f - c2, net.Pw, net.W1b, net.W2b);
            double l = 0.0;
            if (hipMemcpyAsync(&l, net.loss, 8, hipMemcpyDeviceToHost, net.s) != hipSuccess ||
                hipStreamSynchronize(net.s) != hipSuccess)
                return mc_internal_fail(h, MC_E_DEVICE, "training step failed");
            acc += l;
        }
        last = acc / (double)(n_tr / batch);
        if (loss_out) loss_out[e] = last;
    }
    // held-out loss and the stage-2 rejection rate the trained network gives
    // on the held-out moves: sum a1 (1 - a2) / sum a1 with a1 = min(1, e^-dEh)
    // and a2 = min(1, e^-(dE - dEh)) (stage 1 pass probability and stage 2
    // rejection probability of each move)
    double vl = 0.0, s_a1 = 0.0, s_rej = 0.0;
    std::vector<float> outv(2 * (size_t)batch);
    for (int64_t b0 = 0; b0 < n_val; b0 += batch) {
        if (hipMemcpyAsync(net.idx, va.data() + b0, 8 * (size_t)batch, hipMemcpyHostToDevice, net.s) != hipSuccess)
            return mc_internal_fail(h, MC_E_DEVICE, "index upload");
        hipLaunchKernelGGL(gather_kernel, dim3(batch), dim3(256), 0, net.s, lg.feat, lg.de, net.idx, batch, inv_lB,
                           net.X, net.y);
        net.forward(batch);
        net.outputs(batch, 0.f);
        if (hipMemcpyAsync(outv.data(), net.out, 4 * outv.size(), hipMemcpyDeviceToHost, net.s) != hipSuccess ||
            hipStreamSynchronize(net.s) != hipSuccess)
            return mc_internal_fail(h, MC_E_DEVICE, "evaluation failed");
        for (int b = 0; b < batch; ++b) {
            const double dEh = lg.lB * ((double)outv[batch + b] - (double)outv[b]);
            const double dE = de[va[b0 + b]];
            const double r = dEh - dE;
            vl += (r * inv_lB) * (r * inv_lB);
            const double a1 = dEh <= 0 ? 1.0 : std::exp(-dEh);
            const double a2 = dE - dEh <= 0 ? 1.0 : std::exp(-(dE - dEh));
            s_a1 += a1;
            s_rej += a1 * (1.0 - a2);
        }
    }
    if (val_loss) *val_loss = vl / (double)n_val;
    if (ref_stage2_reject) *ref_stage2_reject = s_a1 > 0 ? s_rej / s_a1 : 0.0;
    std::vector<float> pf(kNP);
    if (hipMemcpy(pf.data(), net.Pw, 4 * kNP, hipMemcpyDeviceToHost) != hipSuccess)
        return mc_internal_fail(h, MC_E_DEVICE, "parameter download");
    for (int k = 0; k < kNP; ++k) params_out[k] = pf[k];
    (void)last;
    return MC_OK;
}

}  // extern "C"
