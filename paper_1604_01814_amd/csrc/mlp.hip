// mlp.hip -- learned warm start for the force solve: a per-marker MLP
// (nin -> nh -> nh -> nout, tanh), BF16 weights and GEMM operands with FP32
// accumulation on the matrix cores, FP32 master weights trained with Adam by
// hand-written forward / backward kernels.
//
// The warm start is x0_i = 2 f_{k-1,i} - f_{k-2,i} + MLP(features_i) for the
// force solve of step k (the network corrects the linear extrapolation of
// the force history); the CG iteration it starts still decides convergence
// (ib_force_solve rejects a warm start whose residual exceeds ||b||).
//
// GEMM: C[m][n] = sum_k A(m, k) B(k, n) with arbitrary element strides, so one
// kernel serves X W^T, dY W and dY^T X.  A workgroup of four wavefronts owns a
// 64 x 64 tile of C; operands are staged in LDS as bf16 16-deep K slices and
// each wavefront issues 2 x 2 v_mfma_f32_16x16x16_bf16 per slice.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace lgfib {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even FP32 -> BF16 bits
__host__ __device__ inline unsigned short f2bf(float f) {
    unsigned int u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    const unsigned int r = 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)((u + r) >> 16);
}

constexpr int kTM = 64, kTN = 64, kTK = 16;

// C = alpha * A B (+ C if beta), A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]
__global__ __launch_bounds__(256) void k_gemm_bf16(const float *__restrict__ A, long sam, long sak,
                                                   const float *__restrict__ Bm, long sbk, long sbn,
                                                   float *__restrict__ C, long scm, int M, int N, int K, float alpha,
                                                   int accumulate) {
    __shared__ unsigned short As[kTM][kTK + 2];   // [m][k]
    __shared__ unsigned short Bs[kTN][kTK + 2];   // [n][k]
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;   // wave's 32x32 sub-tile
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kTK) {
        // stage A (64 x 16) and B (16 x 64): 1024 values each, 4 per thread
        for (int e = tid; e < kTM * kTK; e += 256) {
            const int mm = e / kTK, kk = e % kTK;
            const int m = m0 + mm, k = k0 + kk;
            As[mm][kk] = (m < M && k < K) ? f2bf(A[(long)m * sam + (long)k * sak]) : (unsigned short)0;
        }
        for (int e = tid; e < kTN * kTK; e += 256) {
            const int nn = e / kTK, kk = e % kTK;
            const int n = n0 + nn, k = k0 + kk;
            Bs[nn][kk] = (n < N && k < K) ? f2bf(Bm[(long)k * sbk + (long)n * sbn]) : (unsigned short)0;
        }
        __syncthreads();
        // operand layout of v_mfma_f32_16x16x16_bf16: lane l holds
        //   A[row l%16][k 4(l/16)..+3], B[k 4(l/16)..+3][col l%16]
        const int r = lane % 16, kq = 4 * (lane / 16);
        bf16x4 a[2], b[2];
        for (int i = 0; i < 2; ++i)
            for (int q = 0; q < 4; ++q) a[i][q] = (short)As[wm + 16 * i + r][kq + q];
        for (int j = 0; j < 2; ++j)
            for (int q = 0; q < 4; ++q) b[j][q] = (short)Bs[wn + 16 * j + r][kq + q];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // result layout: lane l holds D[row 4(l/16)+q][col l%16]
    const int c = lane % 16, rq = 4 * (lane / 16);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + 16 * i + rq + q, n = n0 + wn + 16 * j + c;
                if (m < M && n < N) {
                    float v = alpha * acc[i][j][q];
                    if (accumulate) v += C[(long)m * scm + n];
                    C[(long)m * scm + n] = v;
                }
            }
}

// Z[m][n] += b[n]; H = tanh(Z) (apply_tanh) in place
__global__ void k_bias_act(float *__restrict__ Z, const float *__restrict__ b, int M, int N, int apply_tanh) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)M * N) return;
    const float v = Z[t] + b[t % N];
    Z[t] = apply_tanh ? tanhf(v) : v;
}

// normalised input xhat = (x - shift) / scale
__global__ void k_normalize(const float *__restrict__ x, const float *__restrict__ shift,
                            const float *__restrict__ scale, float *__restrict__ y, int M, int N) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)M * N) return;
    const int n = (int)(t % N);
    y[t] = (x[t] - shift[n]) / scale[n];
}

// y = shift + scale * x (outputs back to physical units)
__global__ void k_denormalize(const float *__restrict__ x, const float *__restrict__ shift,
                              const float *__restrict__ scale, float *__restrict__ y, int M, int N) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)M * N) return;
    const int n = (int)(t % N);
    y[t] = shift[n] + scale[n] * x[t];
}

// dO = (O - T) / M and per-row squared error (for the loss)
__global__ void k_mse_grad(const float *__restrict__ O, const float *__restrict__ T, float *__restrict__ dO,
                           float *__restrict__ err, int M, int N) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    float e = 0.f;
    for (int n = 0; n < N; ++n) {
        const float d = O[(long)m * N + n] - T[(long)m * N + n];
        dO[(long)m * N + n] = d / (float)M;
        e += d * d;
    }
    err[m] = e;
}

// dZ = dH * (1 - H^2)
__global__ void k_tanh_back(float *__restrict__ dH, const float *__restrict__ H, long n) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dH[t] *= 1.f - H[t] * H[t];
}

// column sums: out[n] = sum_m X[m][n] (fixed order per column)
__global__ void k_colsum(const float *__restrict__ X, float *__restrict__ out, int M, int N) {
    const int n = blockIdx.x;
    __shared__ float sh[256];
    float s = 0.f;
    for (int m = threadIdx.x; m < M; m += 256) s += X[(long)m * N + n];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = sh[0];
}

__global__ void k_sum(const float *__restrict__ x, int n, double *__restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += x[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gi = g[t];
    const float a = b1 * m1[t] + (1.f - b1) * gi;
    const float v = b2 * m2[t] + (1.f - b2) * gi * gi;
    m1[t] = a;
    m2[t] = v;
    p[t] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// features of marker i for the force solve of step k:
//   [n_i (3), U_{k+1} - U_k, U_k - U_{k-1}, U_{k-1} - U_{k-2},
//    f_{k-1,i} (3), f_{k-1,i} - f_{k-2,i} (3)]
__global__ void k_features(const double *__restrict__ normals, double d0, double d1, double d2,
                           const double *__restrict__ f1, const double *__restrict__ f2, float *__restrict__ out,
                           int NL) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NL) return;
    float *o = out + (long)i * 12;
    for (int a = 0; a < 3; ++a) o[a] = (float)normals[3 * i + a];
    o[3] = (float)d0;
    o[4] = (float)d1;
    o[5] = (float)d2;
    for (int a = 0; a < 3; ++a) {
        o[6 + a] = (float)f1[3 * i + a];
        o[9 + a] = (float)(f1[3 * i + a] - f2[3 * i + a]);
    }
}

// x0 = 2 f_{k-1} - f_{k-2} + (shift + scale * o): the network corrects the
// linear extrapolation of the force history
__global__ void k_warm(const double *__restrict__ f1, const double *__restrict__ f2, const float *__restrict__ o,
                       const float *__restrict__ shift, const float *__restrict__ scale, double *__restrict__ x0,
                       int NL) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * NL) return;
    const int a = t % 3;
    x0[t] = (2.0 * f1[t] - f2[t]) + (double)(shift[a] + scale[a] * o[t]);
}

// out[r][:] = in[idx[r]][:]
__global__ void k_gather_rows(const float *__restrict__ in, const int *__restrict__ idx, float *__restrict__ out,
                              int rows, int width) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)rows * width) return;
    const int r = (int)(t / width), c = (int)(t % width);
    out[t] = in[(long)idx[r] * width + c];
}

static unsigned nb(long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace lgfib

using namespace lgfib;

struct ib_mlp {
    lgfib_ctx *ctx = nullptr;
    int nin = 0, nh = 0, nout = 0;
    long nparam = 0;
    long oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
    DevBuf p, g, m1, m2;                  // params, grads, Adam moments (FP32)
    DevBuf in_shift, in_scale, out_shift, out_scale;
    DevBuf xh, h1, h2, o, dO, d1, d2, err, loss;   // activations (grown on demand)
    int cap = 0;
    long step = 0;
};

static int mlp_reserve(ib_mlp *m, int M) {
    if (M <= m->cap) return LGFIB_OK;
    int rc;
    const size_t f = sizeof(float);
    if ((rc = m->xh.reserve((size_t)M * m->nin * f)) || (rc = m->h1.reserve((size_t)M * m->nh * f)) ||
        (rc = m->h2.reserve((size_t)M * m->nh * f)) || (rc = m->o.reserve((size_t)M * m->nout * f)) ||
        (rc = m->dO.reserve((size_t)M * m->nout * f)) ||
        (rc = m->d1.reserve((size_t)M * std::max(m->nh, m->nout) * f)) ||
        (rc = m->d2.reserve((size_t)M * m->nh * f)) || (rc = m->err.reserve((size_t)M * f)))
        return rc;
    m->cap = M;
    return LGFIB_OK;
}

static int gemm(hipStream_t st, const float *A, long sam, long sak, const float *B, long sbk, long sbn, float *C,
                long scm, int M, int N, int K) {
    dim3 grid((N + kTN - 1) / kTN, (M + kTM - 1) / kTM);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, C, scm, M, N, K, 1.f, 0);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// forward: xh = normalised inputs (M x nin) -> h1, h2, o (normalised outputs)
static int mlp_fwd(ib_mlp *m, const float *x, int M, hipStream_t st) {
    const float *P = m->p.as<float>();
    float *xh = m->xh.as<float>(), *h1 = m->h1.as<float>(), *h2 = m->h2.as<float>(), *o = m->o.as<float>();
    int rc;
    hipLaunchKernelGGL(k_normalize, dim3(nb((long)M * m->nin)), dim3(256), 0, st, x, m->in_shift.as<float>(),
                       m->in_scale.as<float>(), xh, M, m->nin);
    // h1 = tanh(xh W1^T + b1):  A(m,k) = xh[m][k], B(k,n) = W1[n][k]
    if ((rc = gemm(st, xh, m->nin, 1, P + m->oW1, 1, m->nin, h1, m->nh, M, m->nh, m->nin))) return rc;
    hipLaunchKernelGGL(k_bias_act, dim3(nb((long)M * m->nh)), dim3(256), 0, st, h1, P + m->ob1, M, m->nh, 1);
    if ((rc = gemm(st, h1, m->nh, 1, P + m->oW2, 1, m->nh, h2, m->nh, M, m->nh, m->nh))) return rc;
    hipLaunchKernelGGL(k_bias_act, dim3(nb((long)M * m->nh)), dim3(256), 0, st, h2, P + m->ob2, M, m->nh, 1);
    if ((rc = gemm(st, h2, m->nh, 1, P + m->oW3, 1, m->nh, o, m->nout, M, m->nout, m->nh))) return rc;
    hipLaunchKernelGGL(k_bias_act, dim3(nb((long)M * m->nout)), dim3(256), 0, st, o, P + m->ob3, M, m->nout, 0);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// gradient of  0.5/M sum_m ||o_m - that_m||^2  (that = normalised targets) into g
static int mlp_bwd(ib_mlp *m, const float *t, int M, hipStream_t st) {
    const float *P = m->p.as<float>();
    float *G = m->g.as<float>();
    float *xh = m->xh.as<float>(), *h1 = m->h1.as<float>(), *h2 = m->h2.as<float>();
    float *dO = m->dO.as<float>(), *d1 = m->d1.as<float>(), *d2 = m->d2.as<float>();
    const int nh = m->nh, nout = m->nout, nin = m->nin;
    int rc;
    // normalised targets: d1 (sized M x max(nh, nout)) is free until dZ1
    hipLaunchKernelGGL(k_normalize, dim3(nb((long)M * nout)), dim3(256), 0, st, t, m->out_shift.as<float>(),
                       m->out_scale.as<float>(), d1, M, nout);
    hipLaunchKernelGGL(k_mse_grad, dim3(nb(M)), dim3(256), 0, st, m->o.as<float>(), d1, dO, m->err.as<float>(), M,
                       nout);
    // dW3[n][k] = sum_m dO[m][n] h2[m][k];  db3 = colsum dO
    if ((rc = gemm(st, dO, 1, nout, h2, nh, 1, G + m->oW3, nh, nout, nh, M))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3(nout), dim3(256), 0, st, dO, G + m->ob3, M, nout);
    // dZ2 = (dO W3) (1 - h2^2)
    if ((rc = gemm(st, dO, nout, 1, P + m->oW3, nh, 1, d2, nh, M, nh, nout))) return rc;
    hipLaunchKernelGGL(k_tanh_back, dim3(nb((long)M * nh)), dim3(256), 0, st, d2, h2, (long)M * nh);
    if ((rc = gemm(st, d2, 1, nh, h1, nh, 1, G + m->oW2, nh, nh, nh, M))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3(nh), dim3(256), 0, st, d2, G + m->ob2, M, nh);
    // dZ1 = (dZ2 W2) (1 - h1^2)
    if ((rc = gemm(st, d2, nh, 1, P + m->oW2, nh, 1, d1, nh, M, nh, nh))) return rc;
    hipLaunchKernelGGL(k_tanh_back, dim3(nb((long)M * nh)), dim3(256), 0, st, d1, h1, (long)M * nh);
    if ((rc = gemm(st, d1, 1, nh, xh, nin, 1, G + m->oW1, nin, nh, nin, M))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3(nh), dim3(256), 0, st, d1, G + m->ob1, M, nh);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, m->err.as<float>(), M, m->loss.as<double>());
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

extern "C" int ib_mlp_create(lgfib_ctx *ctx, int nin, int nh, int nout, const float *params, const float *in_shift,
                             const float *in_scale, const float *out_shift, const float *out_scale, ib_mlp **out) {
    if (!out) return fail(LGFIB_EINVAL, "ib_mlp_create: null output");
    *out = nullptr;
    if (!ctx || !params || !in_shift || !in_scale || !out_shift || !out_scale)
        return fail(LGFIB_EINVAL, "ib_mlp_create: null argument");
    if (nin < 1 || nin > 4096 || nh < 1 || nh > 4096 || nout < 1 || nout > 4096)
        return fail(LGFIB_EINVAL, "ib_mlp_create: layer widths must lie in [1, 4096]");
    for (int i = 0; i < nin; ++i)
        if (!(in_scale[i] != 0.f)) return fail(LGFIB_EINVAL, "ib_mlp_create: zero input scale");
    for (int i = 0; i < nout; ++i)
        if (!(out_scale[i] != 0.f)) return fail(LGFIB_EINVAL, "ib_mlp_create: zero output scale");
    LGF_HIP(hipSetDevice(ctx->device));
    auto m = std::make_unique<ib_mlp>();
    m->ctx = ctx;
    m->nin = nin;
    m->nh = nh;
    m->nout = nout;
    m->oW1 = 0;
    m->ob1 = m->oW1 + (long)nh * nin;
    m->oW2 = m->ob1 + nh;
    m->ob2 = m->oW2 + (long)nh * nh;
    m->oW3 = m->ob2 + nh;
    m->ob3 = m->oW3 + (long)nout * nh;
    m->nparam = m->ob3 + nout;
    const size_t pb = (size_t)m->nparam * sizeof(float);
    int rc;
    if ((rc = m->p.reserve(pb)) || (rc = m->g.reserve(pb)) || (rc = m->m1.reserve(pb)) || (rc = m->m2.reserve(pb)) ||
        (rc = m->in_shift.reserve(nin * 4)) || (rc = m->in_scale.reserve(nin * 4)) ||
        (rc = m->out_shift.reserve(nout * 4)) || (rc = m->out_scale.reserve(nout * 4)) || (rc = m->loss.reserve(8)))
        return rc;
    LGF_HIP(hipMemcpy(m->p.p, params, pb, hipMemcpyHostToDevice));
    LGF_HIP(hipMemset(m->m1.p, 0, pb));
    LGF_HIP(hipMemset(m->m2.p, 0, pb));
    LGF_HIP(hipMemcpy(m->in_shift.p, in_shift, nin * 4, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(m->in_scale.p, in_scale, nin * 4, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(m->out_shift.p, out_shift, nout * 4, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(m->out_scale.p, out_scale, nout * 4, hipMemcpyHostToDevice));
    *out = m.release();
    return LGFIB_OK;
}

extern "C" void ib_mlp_destroy(ib_mlp *m) {
    if (!m) return;
    (void)hipSetDevice(m->ctx->device);
    (void)hipDeviceSynchronize();
    delete m;
}

extern "C" int ib_mlp_get_params(ib_mlp *m, float *host, int64_t n) {
    if (!m || !host) return fail(LGFIB_EINVAL, "ib_mlp_get_params: null argument");
    if (n != m->nparam) return fail(LGFIB_EINVAL, "ib_mlp_get_params: count must be " + std::to_string(m->nparam));
    LGF_HIP(hipSetDevice(m->ctx->device));
    LGF_HIP(hipMemcpy(host, m->p.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    return LGFIB_OK;
}

extern "C" int ib_mlp_forward(lgfib_ctx *ctx, ib_mlp *m, const float *x, int M, float *y, lgfib_stream_t stream) {
    if (!ctx || !m || m->ctx != ctx || !x || !y || M < 0) return fail(LGFIB_EINVAL, "ib_mlp_forward: bad argument");
    if (M == 0) return LGFIB_OK;
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = mlp_reserve(m, M)) || (rc = mlp_fwd(m, x, M, st))) return rc;
    hipLaunchKernelGGL(k_denormalize, dim3(nb((long)M * m->nout)), dim3(256), 0, st, m->o.as<float>(),
                       m->out_shift.as<float>(), m->out_scale.as<float>(), y, M, m->nout);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

extern "C" int ib_mlp_grad(lgfib_ctx *ctx, ib_mlp *m, const float *x, const float *t, int M, float *grad_host,
                           double *loss) {
    if (!ctx || !m || m->ctx != ctx || !x || !t || M < 1) return fail(LGFIB_EINVAL, "ib_mlp_grad: bad argument");
    LGF_HIP(hipSetDevice(ctx->device));
    int rc;
    if ((rc = mlp_reserve(m, M)) || (rc = mlp_fwd(m, x, M, nullptr)) || (rc = mlp_bwd(m, t, M, nullptr))) return rc;
    LGF_HIP(hipDeviceSynchronize());
    if (grad_host) LGF_HIP(hipMemcpy(grad_host, m->g.p, (size_t)m->nparam * 4, hipMemcpyDeviceToHost));
    if (loss) {
        double e = 0.0;
        LGF_HIP(hipMemcpy(&e, m->loss.p, 8, hipMemcpyDeviceToHost));
        *loss = 0.5 * e / M;
    }
    return LGFIB_OK;
}

extern "C" int ib_mlp_train_step(lgfib_ctx *ctx, ib_mlp *m, const float *x, const float *t, int M, float lr,
                                 lgfib_stream_t stream) {
    if (!ctx || !m || m->ctx != ctx || !x || !t || M < 1 || !(lr > 0.f))
        return fail(LGFIB_EINVAL, "ib_mlp_train_step: bad argument");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = mlp_reserve(m, M)) || (rc = mlp_fwd(m, x, M, st)) || (rc = mlp_bwd(m, t, M, st))) return rc;
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)m->step), c2 = 1.f - powf(b2, (float)m->step);
    hipLaunchKernelGGL(k_adam, dim3(nb(m->nparam)), dim3(256), 0, st, m->p.as<float>(), m->g.as<float>(),
                       m->m1.as<float>(), m->m2.as<float>(), m->nparam, lr, b1, b2, eps, c1, c2);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

extern "C" int ib_mlp_last_loss(ib_mlp *m, int M, double *loss) {
    if (!m || !loss || M < 1) return fail(LGFIB_EINVAL, "ib_mlp_last_loss: bad argument");
    LGF_HIP(hipSetDevice(m->ctx->device));
    double e = 0.0;
    LGF_HIP(hipMemcpy(&e, m->loss.p, 8, hipMemcpyDeviceToHost));
    *loss = 0.5 * e / M;
    return LGFIB_OK;
}

extern "C" int ib_mlp_features(lgfib_ctx *ctx, const double *normals, const double *ustate, const double *f1,
                               const double *f2, int NL, float *feats, lgfib_stream_t stream) {
    if (!ctx || !normals || !ustate || !f1 || !f2 || !feats || NL < 0)
        return fail(LGFIB_EINVAL, "ib_mlp_features: bad argument");
    if (NL == 0) return LGFIB_OK;
    LGF_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_features, dim3(nb(NL)), dim3(256), 0, (hipStream_t)stream, normals, ustate[0] - ustate[1],
                       ustate[1] - ustate[2], ustate[2] - ustate[3], f1, f2, feats, NL);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

extern "C" int ib_mlp_warmstart(lgfib_ctx *ctx, ib_mlp *m, const float *feats, const double *f1, const double *f2,
                                int NL, double *x0, lgfib_stream_t stream) {
    if (!ctx || !m || m->ctx != ctx || !feats || !f1 || !f2 || !x0 || NL < 0)
        return fail(LGFIB_EINVAL, "ib_mlp_warmstart: bad argument");
    if (m->nout != 3 || m->nin != 12) return fail(LGFIB_EINVAL, "ib_mlp_warmstart: network must map 12 -> 3");
    if (NL == 0) return LGFIB_OK;
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = mlp_reserve(m, NL)) || (rc = mlp_fwd(m, feats, NL, st))) return rc;
    hipLaunchKernelGGL(k_warm, dim3(nb(3L * NL)), dim3(256), 0, st, f1, f2, m->o.as<float>(),
                       m->out_shift.as<float>(), m->out_scale.as<float>(), x0, NL);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// splitmix64: a counter-based generator for the epoch permutations
static uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

extern "C" int ib_mlp_train(lgfib_ctx *ctx, ib_mlp *m, const float *x, const float *t, int M, int epochs, int batch,
                            float lr, uint64_t seed, double *final_loss) {
    if (!ctx || !m || m->ctx != ctx || !x || !t || M < 1 || epochs < 0 || batch < 1 || !(lr > 0.f))
        return fail(LGFIB_EINVAL, "ib_mlp_train: bad argument");
    LGF_HIP(hipSetDevice(ctx->device));
    batch = std::min(batch, M);
    DevBuf bx, bt, bidx;
    int rc;
    if ((rc = bx.reserve((size_t)batch * m->nin * 4)) || (rc = bt.reserve((size_t)batch * m->nout * 4)) ||
        (rc = bidx.reserve((size_t)M * 4)))
        return rc;
    std::vector<int> perm(M);
    uint64_t st = seed;
    double last = 0.0;
    for (int e = 0; e < epochs; ++e) {
        for (int i = 0; i < M; ++i) perm[i] = i;
        for (int i = M - 1; i > 0; --i) std::swap(perm[i], perm[splitmix64(st) % (uint64_t)(i + 1)]);
        LGF_HIP(hipMemcpy(bidx.p, perm.data(), (size_t)M * 4, hipMemcpyHostToDevice));
        for (int b0 = 0; b0 + batch <= M; b0 += batch) {
            const int *ix = bidx.as<int>() + b0;
            hipLaunchKernelGGL(k_gather_rows, dim3(nb((long)batch * m->nin)), dim3(256), 0, nullptr, x, ix,
                               bx.as<float>(), batch, m->nin);
            hipLaunchKernelGGL(k_gather_rows, dim3(nb((long)batch * m->nout)), dim3(256), 0, nullptr, t, ix,
                               bt.as<float>(), batch, m->nout);
            if ((rc = ib_mlp_train_step(ctx, m, bx.as<float>(), bt.as<float>(), batch, lr, nullptr))) return rc;
        }
        if ((rc = ib_mlp_last_loss(m, batch, &last))) return rc;
    }
    LGF_HIP(hipDeviceSynchronize());
    if (final_loss) *final_loss = last;
    return LGFIB_OK;
}
