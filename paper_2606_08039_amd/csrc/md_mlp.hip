// md_mlp.hip -- training kernels of the aerodynamic-residual surrogate
// (64 -> 128 -> 128 -> 128 -> 6, SiLU, bfloat16 operands, fp32 accumulation).
//
// Every matrix product of the forward and backward passes runs through one
// tiled MFMA kernel (v_mfma_f32_16x16x32_bf16, 64x64 workgroup tiles, four
// waves of 32x32) with a fused epilogue: bias + SiLU (forward), bias only
// (output layer), SiLU' (backward data), or split-K partials (weight
// gradients, reduced afterwards in a fixed order so gradients are
// deterministic).  Master weights, gradients and Adam moments are fp32.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "md.h"
#include "md_mlp.h"

namespace md {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 32, KP = TK + 8;

__device__ __forceinline__ float ldf(const float *p) { return *p; }
__device__ __forceinline__ float ldf(const bf16 *p) { return (float)*p; }

enum Epi { EPI_HIDDEN = 0, EPI_LINEAR = 1, EPI_DSILU = 2, EPI_PARTIAL = 3 };

struct GemmArgs {
    int M, N, K;
    const void *A;
    long long lda;
    int a_trans;  // element (m, k) = a_trans ? A[k * lda + m] : A[m * lda + k]
    const void *B;
    long long ldb;
    int b_trans;  // element (k, n) = b_trans ? B[n * ldb + k] : B[k * ldb + n]
    int k_slice;  // K extent handled by one blockIdx.z
    int epi;
    const float *bias;
    float *out_f;
    bf16 *out_h;
    long long ldo;
    const float *aux;
    long long part_stride;
};

__device__ __forceinline__ float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

__device__ __forceinline__ float dsilu_f(float z) {
    const float s = __builtin_amdgcn_rcpf(1.f + __expf(-z));
    return s * (1.f + z * (1.f - s));
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) bf16 As[TM][KP];
    __shared__ __attribute__((aligned(16))) bf16 Bs[TN][KP];
    const TA *A = (const TA *)g.A;
    const TB *B = (const TB *)g.B;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int kbeg = blockIdx.z * g.k_slice;
    const int kend = min(g.K, kbeg + g.k_slice);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        for (int e = tid; e < TM * TK; e += 256) {
            const int r = e / TK, c = e % TK, m = m0 + r, k = k0 + c;
            float v = 0.f;
            if (m < g.M && k < kend) v = g.a_trans ? ldf(A + (long long)k * g.lda + m) : ldf(A + (long long)m * g.lda + k);
            As[r][c] = (bf16)v;
        }
        for (int e = tid; e < TN * TK; e += 256) {
            const int r = e / TK, c = e % TK, n = n0 + r, k = k0 + c;
            float v = 0.f;
            if (n < g.N && k < kend) v = g.b_trans ? ldf(B + (long long)n * g.ldb + k) : ldf(B + (long long)k * g.ldb + n);
            Bs[r][c] = (bf16)v;
        }
        __syncthreads();
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8 *)&As[wm + i * 16 + (lane & 15)][8 * (lane >> 4)];
        for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8 *)&Bs[wn + j * 16 + (lane & 15)][8 * (lane >> 4)];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // C layout of the 16x16 result: lane holds rows 4*(lane/16)+t, column lane%16
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + j * 16 + (lane & 15);
            for (int t = 0; t < 4; ++t) {
                const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + t;
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][t];
                const long long o = (long long)m * g.ldo + n;
                switch (g.epi) {
                    case EPI_HIDDEN: {
                        const float z = v + g.bias[n];
                        if (g.out_f) g.out_f[o] = z;  // pre-activations, kept for the backward pass
                        g.out_h[o] = (bf16)silu_f(z);
                        break;
                    }
                    case EPI_LINEAR:
                        g.out_f[o] = v + (g.bias ? g.bias[n] : 0.f);
                        break;
                    case EPI_DSILU:
                        g.out_f[o] = v * dsilu_f(g.aux[o]);
                        break;
                    default:
                        g.out_f[blockIdx.z * g.part_stride + o] = v;
                        break;
                }
            }
        }
    }
}

// standardised, bfloat16 network input: xb = bf16((x - mean) * inv_std)
__global__ void prep_input_kernel(const float *X, const float *mean, const float *inv_std, bf16 *Xb,
                                  long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int f = (int)(i % MLP_IN);
    Xb[i] = (bf16)((X[i] - mean[f]) * inv_std[f]);
}

// gradient of the mean squared error over B x OUT standardised targets;
// per-block partial sums of the squared error (fixed reduction order)
__global__ void __launch_bounds__(256) mse_grad_kernel(const float *Y, const float *T, const float *ymean,
                                                       const float *ystd, int B, float *dY, float *loss_part) {
    __shared__ float red[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    float e2 = 0.f;
    if (i < B * MLP_OUT) {
        const int o = i % MLP_OUT;
        const float ts = (T[i] - ymean[o]) / ystd[o];
        const float d = Y[i] - ts;
        dY[i] = d * (2.f / (float)(B * MLP_OUT));
        e2 = d * d;
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// out[i] = sum_z part[z * stride + i], z ascending
__global__ void reduce_parts_kernel(const float *part, int nz, long long stride, float *out, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int z = 0; z < nz; ++z) s += part[z * stride + i];
    out[i] = s;
}

// out[c] = sum_r X[r * ld + c]: one block per column, fixed tree order
__global__ void __launch_bounds__(256) col_sum_kernel(const float *X, int rows, long long ld, float *out) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) s += X[(long long)r * ld + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

// Adam (Kingma and Ba) on the flat fp32 parameters; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t
__global__ void adam_kernel(float *p, const float *g, float *m1, float *m2, int n, float lr, float b1,
                            float b2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float m = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = m;
    m2[i] = v;
    p[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

template <typename TA, typename TB>
hipError_t gemm(const GemmArgs &g, int nz, hipStream_t st) {
    dim3 grid((g.M + TM - 1) / TM, (g.N + TN - 1) / TN, nz);
    hipLaunchKernelGGL((gemm_kernel<TA, TB>), grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

GemmArgs base(int M, int N, int K) {
    GemmArgs g;
    std::memset(&g, 0, sizeof g);
    g.M = M;
    g.N = N;
    g.K = K;
    g.k_slice = K;
    return g;
}

}  // namespace

// Offsets of the flat parameter vector: W1, b1, W2, b2, W3, b3, W4, b4 (W row-major [out][in]).
const int kParamOff[8] = {0, 8192, 8320, 24704, 24832, 41216, 41344, 42112};

// Intermediates of md_mlp_forward_noalloc for up to MD_MLP_NOALLOC_MAX_BATCH
// samples: the standardised bfloat16 input, two bfloat16 hidden activations
// used in turn by the three hidden layers, and the standardised fp32
// outputs.  Every part is a multiple of 256 bytes.  One copy per GPU, held
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on each device.
constexpr size_t NA_B = MD_MLP_NOALLOC_MAX_BATCH;
constexpr size_t NA_XB = 0, NA_HA = NA_XB + 2 * NA_B * MLP_IN, NA_HB = NA_HA + 2 * NA_B * MLP_H,
                 NA_Y = NA_HB + 2 * NA_B * MLP_H, NA_BYTES = NA_Y + 4 * NA_B * MLP_OUT;
static_assert(NA_HA % 256 == 0 && NA_HB % 256 == 0 && NA_Y % 256 == 0, "scratch parts stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on device dev, which must be current;
// resolved once per device.
static hipError_t scratch_on(int dev, unsigned char **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace md

using md::bf16;
using md::kParamOff;

struct md_mlp {
    int max_batch = 0;
    int device = 0;
    float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
    int64_t t = 0;
    float *norm = nullptr;  // x_mean[64], x_inv_std[64], y_mean[6], y_std[6]
    bf16 *Xb = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *Y = nullptr, *dY = nullptr;
    float *dZa = nullptr, *dZb = nullptr, *part = nullptr, *loss_part = nullptr;
    int part_nz = 0;
    int last_B = 0, fwd_B = 0;
    bool have_fwd = false, have_bwd = false;
    std::vector<void *> allocs;
    unsigned char *scratch = nullptr;  // this device's static scratch (md_mlp_forward_noalloc)
    std::string scratch_err;
    std::string err;
};

namespace {

md_status mlp_fail(md_mlp *m, md_status st, const std::string &msg) {
    m->err = msg;
    return st;
}

template <typename T>
hipError_t mlp_alloc(md_mlp *m, T **p, size_t n) {
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (n > 0 ? n : 1));
    if (e == hipSuccess) {
        m->allocs.push_back(*p);
        e = hipMemset(*p, 0, sizeof(T) * (n > 0 ? n : 1));
    }
    return e;
}

constexpr int kSplitRows = 256;  // batch rows per split-K slice of a weight gradient

}  // namespace

extern "C" {

md_status md_mlp_create(int max_batch, md_mlp **out) {
    if (!out || max_batch < 1 || max_batch > (1 << 24)) return MD_E_INVALID_ARG;
    *out = nullptr;
    md_mlp *m = new (std::nothrow) md_mlp();
    if (!m) return MD_E_OOM;
    m->max_batch = max_batch;
    (void)hipGetDevice(&m->device);
    const size_t Bm = (size_t)max_batch;
    m->part_nz = (max_batch + kSplitRows - 1) / kSplitRows;
    hipError_t e = hipSuccess;
    auto A = [&](auto **p, size_t n) {
        if (e == hipSuccess) e = mlp_alloc(m, p, n);
    };
    A(&m->params, md::MLP_NPARAMS);
    A(&m->grads, md::MLP_NPARAMS);
    A(&m->m1, md::MLP_NPARAMS);
    A(&m->m2, md::MLP_NPARAMS);
    A(&m->norm, md::MLP_NORM);
    A(&m->Xb, Bm * md::MLP_IN);
    A(&m->H1, Bm * md::MLP_H);
    A(&m->H2, Bm * md::MLP_H);
    A(&m->H3, Bm * md::MLP_H);
    A(&m->Z1, Bm * md::MLP_H);
    A(&m->Z2, Bm * md::MLP_H);
    A(&m->Z3, Bm * md::MLP_H);
    A(&m->Y, Bm * md::MLP_OUT);
    A(&m->dY, Bm * md::MLP_OUT);
    A(&m->dZa, Bm * md::MLP_H);
    A(&m->dZb, Bm * md::MLP_H);
    A(&m->part, (size_t)m->part_nz * md::MLP_H * md::MLP_H);
    A(&m->loss_part, (Bm * md::MLP_OUT + 255) / 256);
    if (e != hipSuccess) {
        md_mlp_destroy(m);
        return MD_E_OOM;
    }
    // the address of this device's static scratch, resolved here (set-up)
    // rather than in the call that must not allocate
    const hipError_t se = md::scratch_on(m->device, &m->scratch);
    if (se != hipSuccess) m->scratch_err = md::hip_msg("hipGetSymbolAddress(scratch)", se);
    // identity normalisation until set
    std::vector<float> nrm(md::MLP_NORM, 0.f);
    for (int i = 0; i < md::MLP_IN; ++i) nrm[md::MLP_IN + i] = 1.f;
    for (int i = 0; i < md::MLP_OUT; ++i) nrm[2 * md::MLP_IN + md::MLP_OUT + i] = 1.f;
    if (hipMemcpy(m->norm, nrm.data(), sizeof(float) * nrm.size(), hipMemcpyHostToDevice) != hipSuccess) {
        md_mlp_destroy(m);
        return MD_E_HIP;
    }
    *out = m;
    return MD_OK;
}

void md_mlp_destroy(md_mlp *m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    for (void *p : m->allocs) (void)hipFree(p);
    delete m;
}

const char *md_mlp_last_error(const md_mlp *m) { return m ? m->err.c_str() : "null md_mlp"; }

md_status md_mlp_set_params(md_mlp *m, const float *h_params) {
    if (!m || !h_params) return MD_E_INVALID_ARG;
    hipError_t e = hipMemcpy(m->params, h_params, sizeof(float) * md::MLP_NPARAMS, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->m1, 0, sizeof(float) * md::MLP_NPARAMS);
    if (e == hipSuccess) e = hipMemset(m->m2, 0, sizeof(float) * md::MLP_NPARAMS);
    if (e != hipSuccess) return mlp_fail(m, MD_E_HIP, md::hip_msg("md_mlp_set_params", e));
    m->t = 0;
    return MD_OK;
}

md_status md_mlp_get_params(const md_mlp *m, float *h_params) {
    if (!m || !h_params) return MD_E_INVALID_ARG;
    (void)hipDeviceSynchronize();
    return hipMemcpy(h_params, m->params, sizeof(float) * md::MLP_NPARAMS, hipMemcpyDeviceToHost) == hipSuccess
               ? MD_OK
               : MD_E_HIP;
}

md_status md_mlp_set_norm(md_mlp *m, const float *h_norm) {
    if (!m || !h_norm) return MD_E_INVALID_ARG;
    for (int i = 0; i < md::MLP_IN; ++i)
        if (!(h_norm[md::MLP_IN + i] > 0.f)) return mlp_fail(m, MD_E_INVALID_ARG, "input scales must be > 0");
    for (int i = 0; i < md::MLP_OUT; ++i)
        if (!(h_norm[2 * md::MLP_IN + md::MLP_OUT + i] > 0.f))
            return mlp_fail(m, MD_E_INVALID_ARG, "output scales must be > 0");
    return hipMemcpy(m->norm, h_norm, sizeof(float) * md::MLP_NORM, hipMemcpyHostToDevice) == hipSuccess
               ? MD_OK
               : MD_E_HIP;
}

md_status md_mlp_get_norm(const md_mlp *m, float *h_norm) {
    if (!m || !h_norm) return MD_E_INVALID_ARG;
    return hipMemcpy(h_norm, m->norm, sizeof(float) * md::MLP_NORM, hipMemcpyDeviceToHost) == hipSuccess
               ? MD_OK
               : MD_E_HIP;
}

}  // extern "C"

namespace {

// The forward pass on buffers Xb [B][64], H[l] [B][128] (bf16), Z[l]
// [B][128] (fp32 pre-activations, or null to keep none) and Y [B][6]
// (standardised fp32); d_Y (nullable) receives the de-standardised outputs.
hipError_t mlp_forward_on(const md_mlp *m, const float *d_X, int B, bf16 *Xb, bf16 *const H[3],
                          float *const Z[3], float *Y, float *d_Y, hipStream_t st) {
    using namespace md;
    const float *P = m->params;
    const long long nx = (long long)B * MLP_IN;
    hipLaunchKernelGGL(prep_input_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, d_X, m->norm,
                       m->norm + MLP_IN, Xb, nx);
    hipError_t e = hipGetLastError();
    const bf16 *hin = Xb;
    int din = MLP_IN;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        GemmArgs g = base(B, MLP_H, din);
        g.A = hin;
        g.lda = din;
        g.B = P + kParamOff[2 * l];  // W[out][in]: element (k, n) = W[n][k]
        g.ldb = din;
        g.b_trans = 1;
        g.epi = EPI_HIDDEN;
        g.bias = P + kParamOff[2 * l + 1];
        g.out_f = Z[l];
        g.out_h = H[l];
        g.ldo = MLP_H;
        e = gemm<bf16, float>(g, 1, st);
        hin = H[l];
        din = MLP_H;
    }
    if (e == hipSuccess) {
        GemmArgs g = base(B, MLP_OUT, MLP_H);
        g.A = H[2];
        g.lda = MLP_H;
        g.B = P + kParamOff[6];
        g.ldb = MLP_H;
        g.b_trans = 1;
        g.epi = EPI_LINEAR;
        g.bias = P + kParamOff[7];
        g.out_f = Y;
        g.ldo = MLP_OUT;
        e = gemm<bf16, float>(g, 1, st);
    }
    if (e == hipSuccess && d_Y) e = mlp_destandardize(Y, m->norm + 2 * MLP_IN, d_Y, B, st);
    return e;
}

}  // namespace

extern "C" {

md_status md_mlp_forward(md_mlp *m, const float *d_X, int B, float *d_Y, void *stream) {
    using namespace md;
    if (!m || !d_X || B < 0) return MD_E_INVALID_ARG;
    if (B > m->max_batch) return mlp_fail(m, MD_E_INVALID_ARG, "batch exceeds max_batch");
    if (B == 0) return MD_OK;
    bf16 *const H[3] = {m->H1, m->H2, m->H3};
    float *const Z[3] = {m->Z1, m->Z2, m->Z3};
    const hipError_t e = mlp_forward_on(m, d_X, B, m->Xb, H, Z, m->Y, d_Y, (hipStream_t)stream);
    if (e != hipSuccess) return mlp_fail(m, MD_E_HIP, hip_msg("md_mlp_forward", e));
    m->fwd_B = B;
    m->have_fwd = true;
    return MD_OK;
}

md_status md_mlp_forward_noalloc(md_mlp *m, const float *d_X, int B, float *d_Y, void *stream) {
    using namespace md;
    if (!m || !d_X || !d_Y || B < 0) {
        if (m) m->err = "md_mlp_forward_noalloc: null input or output, or B < 0";
        return MD_E_INVALID_ARG;
    }
    if (B > MD_MLP_NOALLOC_MAX_BATCH)
        return mlp_fail(m, MD_E_INVALID_ARG,
                        "md_mlp_forward_noalloc: batch " + std::to_string(B) + " exceeds its static scratch of " +
                            std::to_string(MD_MLP_NOALLOC_MAX_BATCH) + " samples");
    if (!m->scratch) return mlp_fail(m, MD_E_HIP, "md_mlp_forward_noalloc: " + m->scratch_err);
    if (B == 0) return MD_OK;
    unsigned char *s = m->scratch;
    bf16 *Xb = (bf16 *)(s + NA_XB), *Ha = (bf16 *)(s + NA_HA), *Hb = (bf16 *)(s + NA_HB);
    // inference keeps no pre-activations: the hidden layers alternate between two buffers
    bf16 *const H[3] = {Ha, Hb, Ha};
    float *const Z[3] = {nullptr, nullptr, nullptr};
    const hipError_t e = mlp_forward_on(m, d_X, B, Xb, H, Z, (float *)(s + NA_Y), d_Y, (hipStream_t)stream);
    if (e != hipSuccess) return mlp_fail(m, MD_E_HIP, hip_msg("md_mlp_forward_noalloc", e));
    return MD_OK;
}

md_status md_mlp_backward(md_mlp *m, const float *d_T, int B, void *stream) {
    using namespace md;
    if (!m || !d_T) return MD_E_INVALID_ARG;
    if (!m->have_fwd || m->fwd_B != B || B < 1) return mlp_fail(m, MD_E_INVALID_ARG, "backward needs the forward of the same batch");
    hipStream_t st = (hipStream_t)stream;
    const float *P = m->params;
    float *G = m->grads;
    const int nblk = (B * MLP_OUT + 255) / 256;
    hipLaunchKernelGGL(mse_grad_kernel, dim3(nblk), dim3(256), 0, st, m->Y, d_T, m->norm + 2 * MLP_IN,
                       m->norm + 2 * MLP_IN + MLP_OUT, B, m->dY, m->loss_part);
    hipError_t e = hipGetLastError();
    const int nz = (B + kSplitRows - 1) / kSplitRows;
    // weight gradient dW[out][in] = sum_b dZ[b][out] * Hin[b][in]  (split-K over the batch)
    auto wgrad = [&](const float *dZ, int dout, const bf16 *Hin, int din, int l) {
        if (e != hipSuccess) return;
        GemmArgs g = base(dout, din, B);
        g.A = dZ;
        g.lda = dout;
        g.a_trans = 1;
        g.B = Hin;
        g.ldb = din;
        g.b_trans = 0;
        g.k_slice = kSplitRows;
        g.epi = EPI_PARTIAL;
        g.out_f = m->part;
        g.ldo = din;
        g.part_stride = (long long)dout * din;
        e = gemm<float, bf16>(g, nz, st);
        if (e != hipSuccess) return;
        const long long n = (long long)dout * din;
        hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m->part, nz, n,
                           G + kParamOff[2 * l], n);
        hipLaunchKernelGGL(col_sum_kernel, dim3(dout), dim3(256), 0, st, dZ, B, (long long)dout, G + kParamOff[2 * l + 1]);
        e = hipGetLastError();
    };
    // data gradient dZprev = (dZ W) * SiLU'(Zprev)
    auto dgrad = [&](const float *dZ, int dout, int l, const float *Zprev, float *outp) {
        if (e != hipSuccess) return;
        GemmArgs g = base(B, MLP_H, dout);
        g.A = dZ;
        g.lda = dout;
        g.B = P + kParamOff[2 * l];  // W[out][in]: element (k = out, n = in)
        g.ldb = MLP_H;
        g.b_trans = 0;
        g.epi = EPI_DSILU;
        g.aux = Zprev;
        g.out_f = outp;
        g.ldo = MLP_H;
        e = gemm<float, float>(g, 1, st);
    };
    wgrad(m->dY, MLP_OUT, m->H3, MLP_H, 3);
    dgrad(m->dY, MLP_OUT, 3, m->Z3, m->dZa);
    wgrad(m->dZa, MLP_H, m->H2, MLP_H, 2);
    dgrad(m->dZa, MLP_H, 2, m->Z2, m->dZb);
    wgrad(m->dZb, MLP_H, m->H1, MLP_H, 1);
    dgrad(m->dZb, MLP_H, 1, m->Z1, m->dZa);
    wgrad(m->dZa, MLP_H, m->Xb, MLP_IN, 0);
    if (e != hipSuccess) return mlp_fail(m, MD_E_HIP, hip_msg("md_mlp_backward", e));
    m->last_B = B;
    m->have_bwd = true;
    return MD_OK;
}

md_status md_mlp_get_grads(const md_mlp *m, float *h_grads) {
    if (!m || !h_grads) return MD_E_INVALID_ARG;
    (void)hipDeviceSynchronize();
    return hipMemcpy(h_grads, m->grads, sizeof(float) * md::MLP_NPARAMS, hipMemcpyDeviceToHost) == hipSuccess
               ? MD_OK
               : MD_E_HIP;
}

md_status md_mlp_loss(const md_mlp *m, double *out) {
    if (!m || !out) return MD_E_INVALID_ARG;
    if (!m->have_bwd) return MD_E_INVALID_ARG;
    (void)hipDeviceSynchronize();
    const int nblk = (m->last_B * md::MLP_OUT + 255) / 256;
    std::vector<float> h(nblk);
    if (hipMemcpy(h.data(), m->loss_part, sizeof(float) * nblk, hipMemcpyDeviceToHost) != hipSuccess) return MD_E_HIP;
    double s = 0.0;
    for (float v : h) s += v;
    *out = s / ((double)m->last_B * md::MLP_OUT);
    return MD_OK;
}

md_status md_mlp_adam(md_mlp *m, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!m || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return MD_E_INVALID_ARG;
    if (!m->have_bwd) return mlp_fail(m, MD_E_INVALID_ARG, "adam needs gradients (call md_mlp_backward)");
    m->t += 1;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)m->t));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)m->t));
    hipLaunchKernelGGL(md::adam_kernel, dim3((md::MLP_NPARAMS + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       m->params, m->grads, m->m1, m->m2, md::MLP_NPARAMS, lr, beta1, beta2, eps, bc1, bc2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MD_OK : mlp_fail(m, MD_E_HIP, md::hip_msg("md_mlp_adam", e));
}

}  // extern "C"

namespace md {

__global__ void destd_kernel(const float *Y, const float *ymean_std, float *out, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * MLP_OUT) return;
    const int o = i % MLP_OUT;
    out[i] = Y[i] * ymean_std[MLP_OUT + o] + ymean_std[o];
}

hipError_t mlp_destandardize(const float *Y, const float *ymean_std, float *out, int B, hipStream_t st) {
    hipLaunchKernelGGL(destd_kernel, dim3((B * MLP_OUT + 255) / 256), dim3(256), 0, st, Y, ymean_std, out, B);
    return hipGetLastError();
}

const float *mlp_device_params(const md_mlp *m) { return m->params; }
const float *mlp_device_norm(const md_mlp *m) { return m->norm; }

}  // namespace md
