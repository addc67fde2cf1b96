// pair.hip -- the block-pair form of the LGF convolution (Sec. 2.2,
// Eq. dpoisson_conv summed block pair by block pair), for blocks of 8^3.
//
// u_t = sum_s G_{t-s} * f_s, where G_d is the kernel restricted to the
// offsets of block pair distance d: (G_d)(j) = G(8 d + j), j in [-7, 7]^3.
// Placed circularly in a 16^3 box (j < 0 at 16 + j, slot 8 unused) the
// circular convolution of length 16 with f_s (nonzero on [0, 8)^3) is exact
// on the kept outputs [0, 8)^3, so
//   U_t(k) = sum_s Ghat_{t-s}(k) Fhat_s(k),  u_t = IDFT_16(U_t) on [0, 8)^3,
// with every spectrum Hermitian (real data): only kx in [0, 8] is kept,
// 16 x 16 x 9 complex values per block.
//
// Per-block transforms (three axes of 16-point DFTs) come in two variants:
//   LGF_DFT_FFT32: each 16-point DFT in registers by one thread, FP32;
//   LGF_DFT_BF16X3: each axis as a complex 16 x 16 matrix product on the
//     matrix cores, both operands split into three BF16 terms
//     (x = hi + mid + lo) and the six products down to relative size 2^-16
//     accumulated in FP32 (v_mfma_f32_16x16x16_bf16).
// The kernel spectra Ghat_d (every offset d of the target/source span) are
// transformed once in FP64 and kept as FP32; the multiply-accumulate over
// source blocks is FP32 complex.  The cost grows with the number of block
// pairs, so this form suits small or sparse sets; the box FFT (conv.hip)
// suits large dense ones.
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "conv_common.h"
#include "fft_static.h"

namespace lgfib {

constexpr int kPB = 8, kPN = 16, kPH = 9, kPS = kPN * kPN * kPH;   // 2304 complex per block spectrum

using F2 = float2;
using D2 = double2;

// ---------------------------------------------------------------- FP32 DFTs

// forward spectrum of one source block: f [8^3] real (z, y, x) -> [kz][ky][kx<9]
__global__ __launch_bounds__(256) void k_pair_fwd(const float *__restrict__ f, int nsrc, F2 *__restrict__ Fh) {
    __shared__ F2 T[kPB * kPB * kPH];   // [z<8][y<8][kx<9]
    __shared__ F2 U[kPB * kPN * kPH];   // [z<8][ky<16][kx<9]
    const int s = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    const float *fs = f + ((size_t)c * nsrc + s) * 512;
    if (tid < 64) {   // x rows (z, y)
        F2 v[16];
#pragma unroll
        for (int x = 0; x < 16; ++x) v[x] = F2{x < 8 ? fs[tid * 8 + x] : 0.f, 0.f};
        Dft<F2, 16, false>::run(v);
#pragma unroll
        for (int k = 0; k < kPH; ++k) T[tid * kPH + k] = v[k];
    }
    __syncthreads();
    if (tid < kPB * kPH) {   // y columns (z, kx)
        const int z = tid / kPH, kx = tid % kPH;
        F2 v[16];
#pragma unroll
        for (int y = 0; y < 16; ++y) v[y] = y < 8 ? T[(z * kPB + y) * kPH + kx] : F2{0.f, 0.f};
        Dft<F2, 16, false>::run(v);
#pragma unroll
        for (int k = 0; k < 16; ++k) U[(z * kPN + k) * kPH + kx] = v[k];
    }
    __syncthreads();
    if (tid < kPN * kPH) {   // z columns (ky, kx)
        const int ky = tid / kPH, kx = tid % kPH;
        F2 v[16];
#pragma unroll
        for (int z = 0; z < 16; ++z) v[z] = z < 8 ? U[(z * kPN + ky) * kPH + kx] : F2{0.f, 0.f};
        Dft<F2, 16, false>::run(v);
        F2 *o = Fh + ((size_t)c * nsrc + s) * kPS;
#pragma unroll
        for (int k = 0; k < 16; ++k) o[(k * kPN + ky) * kPH + kx] = v[k];
    }
}

// inverse of one target spectrum, kept on [0, 8)^3 and scaled
__global__ __launch_bounds__(256) void k_pair_inv(const F2 *__restrict__ Uh, int ntgt, float scale,
                                                  float *__restrict__ u) {
    __shared__ F2 V[kPB * kPN * kPH];   // [z<8][ky][kx]
    __shared__ F2 W[kPB * kPB * kPH];   // [z<8][y<8][kx]
    const int t = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    const F2 *in = Uh + ((size_t)c * ntgt + t) * kPS;
    if (tid < kPN * kPH) {   // z columns
        const int ky = tid / kPH, kx = tid % kPH;
        F2 v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = in[(k * kPN + ky) * kPH + kx];
        Dft<F2, 16, true>::run(v);
#pragma unroll
        for (int z = 0; z < 8; ++z) V[(z * kPN + ky) * kPH + kx] = v[z];
    }
    __syncthreads();
    if (tid < kPB * kPH) {   // y columns
        const int z = tid / kPH, kx = tid % kPH;
        F2 v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = V[(z * kPN + k) * kPH + kx];
        Dft<F2, 16, true>::run(v);
#pragma unroll
        for (int y = 0; y < 8; ++y) W[(z * kPB + y) * kPH + kx] = v[y];
    }
    __syncthreads();
    if (tid < 64) {   // x rows: Hermitian completion, real part
        F2 v[16];
#pragma unroll
        for (int k = 0; k < kPH; ++k) v[k] = W[tid * kPH + k];
#pragma unroll
        for (int k = kPH; k < 16; ++k) {
            const F2 h = W[tid * kPH + (16 - k)];
            v[k] = F2{h.x, -h.y};
        }
        Dft<F2, 16, true>::run(v);
        float *o = u + ((size_t)c * ntgt + t) * 512 + tid * 8;
#pragma unroll
        for (int x = 0; x < 8; ++x) o[x] = v[x].x * scale;
    }
}

// --------------------------------------------- split-BF16 matrix-core DFTs

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
// x = hi + mid + lo: hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid).
// Each remainder is exact in FP32, so the three terms hold 24 significant bits
// and |x - hi - mid - lo| <= 2^-24 |x|.
__device__ __forceinline__ void split3_bf16(float x, short &hi, short &mid, short &lo) {
    const unsigned short h = bf16_rne(x);
    const float r1 = x - bf16_to_f(h);
    const unsigned short m = bf16_rne(r1);
    hi = (short)h;
    mid = (short)m;
    lo = (short)bf16_rne(r1 - bf16_to_f(m));
}

// One complex 16-point DFT stage on the matrix cores for the 16 columns held
// by a wavefront: Y = W X with W the 16 x 16 DFT matrix (forward or
// inverse), X given column-wise through `get(k, col)` and Y delivered through
// `put(row, col, value)`.  Operand layout of v_mfma_f32_16x16x16_bf16: lane l
// holds A[row l%16][k 4(l/16)+q] and B[k 4(l/16)+q][col l%16]; the result
// D[row 4(l/16)+q][col l%16].
//
// Both operands are split three ways (split3_bf16).  Of the nine products of
// the parts, the six of relative size 1, 2^-8 and 2^-16 are kept: hh; hm, mh;
// hl, lh, mm.  The three dropped ones (ml, lm, ll) are at most 2^-23 of
// |w||x| together, below the FP32 accumulation's own rounding.  The products
// go into the FP32 accumulator smallest first.
template <bool INV, typename Get, typename Put>
__device__ __forceinline__ void mfma_dft16(Get get, Put put) {
    const int lane = threadIdx.x % 64;
    const int r = lane % 16, kq = 4 * (lane / 16);
    // [part]: 0 hi, 1 mid, 2 lo
    bf16x4 wr[3], wi[3], win[3], xr[3], xi[3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = kq + q;
        // W[r][k] = exp(-+ 2 pi i r k / 16), exact angle reduction mod 16
        const int m = (r * k) & 15;
        const float cs = cospif((float)m * 0.125f), sn = sinpif((float)m * 0.125f);
        short p0, p1, p2;
        split3_bf16(cs, p0, p1, p2);
        wr[0][q] = p0;
        wr[1][q] = p1;
        wr[2][q] = p2;
        split3_bf16(INV ? sn : -sn, p0, p1, p2);
        wi[0][q] = p0;
        wi[1][q] = p1;
        wi[2][q] = p2;
        win[0][q] = (short)(p0 ^ (short)0x8000);
        win[1][q] = (short)(p1 ^ (short)0x8000);
        win[2][q] = (short)(p2 ^ (short)0x8000);
        const F2 x = get(k, r);   // B[k][col = r]
        split3_bf16(x.x, p0, p1, p2);
        xr[0][q] = p0;
        xr[1][q] = p1;
        xr[2][q] = p2;
        split3_bf16(x.y, p0, p1, p2);
        xi[0][q] = p0;
        xi[1][q] = p1;
        xi[2][q] = p2;
    }
    // (w part, x part), smallest first
    constexpr int kTerms = 6;
    constexpr int pw[kTerms] = {1, 2, 0, 1, 0, 0};
    constexpr int px[kTerms] = {1, 0, 2, 0, 1, 0};
    f32x4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
    // yr = Wr Xr - Wi Xi ; yi = Wr Xi + Wi Xr
#pragma unroll
    for (int t = 0; t < kTerms; ++t) {
        yr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wr[pw[t]], xr[px[t]], yr, 0, 0, 0);
        yr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(win[pw[t]], xi[px[t]], yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wr[pw[t]], xi[px[t]], yi, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wi[pw[t]], xr[px[t]], yi, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) put(kq + q, r, F2{yr[q], yi[q]});
}

// forward spectrum, matrix-core DFTs: 4 wavefronts, each a 16-column slab
__global__ __launch_bounds__(256) void k_pair_fwd_mfma(const float *__restrict__ f, int nsrc, F2 *__restrict__ Fh) {
    __shared__ F2 A[kPN * kPN * kPN];   // [z][y][kx]: 32 KiB, kx < 16 holds the full x spectrum
    const int s = blockIdx.x, c = blockIdx.y, tid = threadIdx.x, wave = tid / 64;
    const float *fs = f + ((size_t)c * nsrc + s) * 512;
    // x: columns are the 64 rows (z<8, y<8); K = x (8 nonzero of 16)
    for (int g = wave; g < 4; g += 4) {
        const int row0 = 16 * g;
        mfma_dft16<false>(
            [&](int k, int col) {
                const int row = row0 + col;
                return F2{k < 8 ? fs[row * 8 + k] : 0.f, 0.f};
            },
            [&](int kx, int col, F2 v) {
                const int row = row0 + col;   // row = z * 8 + y
                A[((row / 8) * kPN + row % 8) * kPN + kx] = v;
            });
    }
    __syncthreads();
    // y: columns (z<8, kx<16): 128 columns, 8 groups of 16; K = y (8 nonzero)
    for (int g = wave; g < 8; g += 4) {
        const int z = g;   // group g: z = g, all 16 kx (the wave reads its slab before writing it)
        mfma_dft16<false>(
            [&](int k, int col) { return k < 8 ? A[(z * kPN + k) * kPN + col] : F2{0.f, 0.f}; },
            [&](int ky, int col, F2 v) { A[(z * kPN + ky) * kPN + col] = v; });
    }
    __syncthreads();
    // z: columns (ky<16, kx<9): 16 groups (one per ky), kx = col (only < 9 kept)
    F2 *o = Fh + ((size_t)c * nsrc + s) * kPS;
    for (int g = wave; g < 16; g += 4) {
        const int ky = g;
        mfma_dft16<false>(
            [&](int k, int col) { return k < 8 ? A[(k * kPN + ky) * kPN + col] : F2{0.f, 0.f}; },
            [&](int kz, int col, F2 v) {
                if (col < kPH) o[(kz * kPN + ky) * kPH + col] = v;
            });
    }
}

// inverse, matrix-core DFTs
__global__ __launch_bounds__(256) void k_pair_inv_mfma(const F2 *__restrict__ Uh, int ntgt, float scale,
                                                       float *__restrict__ u) {
    __shared__ F2 A[kPN * kPN * kPN];   // [z][y][kx<16]
    const int t = blockIdx.x, c = blockIdx.y, tid = threadIdx.x, wave = tid / 64;
    const F2 *in = Uh + ((size_t)c * ntgt + t) * kPS;
    // Hermitian completion of kx in [9, 16) while staging: X(kx) = conj(X(-k))
    for (int i = tid; i < kPN * kPN * kPN; i += 256) {
        const int kx = i % kPN, ky = (i / kPN) % kPN, kz = i / (kPN * kPN);
        F2 v;
        if (kx < kPH) {
            v = in[(kz * kPN + ky) * kPH + kx];
        } else {
            const F2 h = in[(((16 - kz) & 15) * kPN + ((16 - ky) & 15)) * kPH + (16 - kx)];
            v = F2{h.x, -h.y};
        }
        A[i] = v;
    }
    __syncthreads();
    // z: columns (ky, kx) -- 256 columns, 16 groups of 16 (one ky each);
    // every group reads its whole column before any group writes, so the
    // results go through registers
    F2 zres[4][4];
    for (int g = wave, n = 0; g < 16; g += 4, ++n) {
        const int ky = g;
        mfma_dft16<true>([&](int k, int col) { return A[(k * kPN + ky) * kPN + col]; },
                         [&](int z, int col, F2 v) { zres[n][z % 4] = v; });
    }
    __syncthreads();
    for (int g = wave, n = 0; g < 16; g += 4, ++n) {
        const int lane = tid % 64, r = lane % 16, kq = 4 * (lane / 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) A[((kq + q) * kPN + g) * kPN + r] = zres[n][q];
    }
    __syncthreads();
    // y: columns (z<8, kx) -- 8 groups
    for (int g = wave; g < 8; g += 4) {
        const int z = g;
        mfma_dft16<true>([&](int k, int col) { return A[(z * kPN + k) * kPN + col]; },
                         [&](int y, int col, F2 v) { zres[0][y % 4] = v; });
        // the slab z belongs to this wave alone and was read before the writes
        const int lane = tid % 64, r = lane % 16, kq = 4 * (lane / 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) A[(z * kPN + kq + q) * kPN + r] = zres[0][q];
    }
    __syncthreads();
    // x: columns are rows (z<8, y<8), 64 of them, 4 groups; output x < 8 real
    float *ob = u + ((size_t)c * ntgt + t) * 512;
    for (int g = wave; g < 4; g += 4) {
        const int row0 = 16 * g;
        mfma_dft16<true>(
            [&](int k, int col) {
                const int row = row0 + col;
                return A[((row / 8) * kPN + row % 8) * kPN + k];
            },
            [&](int x, int col, F2 v) {
                if (x < 8) ob[(row0 + col) * 8 + x] = v.x * scale;
            });
    }
}

// ------------------------------------------------------------ kernel spectra

// Ghat_d for every block offset d of the span (FP64 transform, stored FP32):
// window (G_d)(j) = G(8 d + j), j in [-7, 7]^3, circular in 16^3
__global__ __launch_bounds__(256) void k_pair_ghat(const double *__restrict__ g, int e1, int e2, int e3, int S0,
                                                   int S1, int S2, F2 *__restrict__ Gh) {
    __shared__ D2 A[kPN * kPN * kPH];   // [z][y][kx<9], 36 KiB
    const int o = blockIdx.x, tid = threadIdx.x;
    const int W0 = 2 * S0 + 1, W1 = 2 * S1 + 1;
    const int dx = o % W0 - S0, dy = (o / W0) % W1 - S1, dz = o / (W0 * W1) - S2;
    // x rows (z, y): 256 rows
    {
        const int z = tid / 16, y = tid % 16;
        const int jz = z < 8 ? z : z - 16, jy = y < 8 ? y : y - 16;
        D2 v[16];
#pragma unroll
        for (int x = 0; x < 16; ++x) {
            const int jx = x < 8 ? x : x - 16;
            double val = 0.0;
            if (x != 8 && y != 8 && z != 8) {
                const int nx = abs(8 * dx + jx), ny = abs(8 * dy + jy), nz = abs(8 * dz + jz);
                val = g[((size_t)nz * (e2 + 1) + ny) * (e1 + 1) + nx];
            }
            v[x] = D2{val, 0.0};
        }
        Dft<D2, 16, false>::run(v);
#pragma unroll
        for (int k = 0; k < kPH; ++k) A[tid * kPH + k] = v[k];
    }
    __syncthreads();
    // y columns (z, kx): 144, in place through registers
    D2 v[16];
    const bool ycol = tid < kPN * kPH;
    const int z = tid / kPH, kx = tid % kPH;
    if (ycol) {
#pragma unroll
        for (int y = 0; y < 16; ++y) v[y] = A[(z * kPN + y) * kPH + kx];
        Dft<D2, 16, false>::run(v);
    }
    __syncthreads();
    if (ycol) {
#pragma unroll
        for (int k = 0; k < 16; ++k) A[(z * kPN + k) * kPH + kx] = v[k];
    }
    __syncthreads();
    if (ycol) {   // z columns (ky, kx)
        const int ky = tid / kPH;
#pragma unroll
        for (int zz = 0; zz < 16; ++zz) v[zz] = A[(zz * kPN + ky) * kPH + kx];
        Dft<D2, 16, false>::run(v);
        F2 *out = Gh + (size_t)o * kPS;
#pragma unroll
        for (int k = 0; k < 16; ++k) out[(k * kPN + ky) * kPH + kx] = F2{(float)v[k].x, (float)v[k].y};
    }
}

// u = 0 (a fill kernel: no memset node where a caller captures the work)
__global__ void k_zero_f32(float *__restrict__ u, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) u[i] = 0.f;
}

// ------------------------------------------------------ pair multiply-accumulate

// U_t(k) = sum_s Ghat_{t-s}(k) Fhat_s(k): a thread per (target, frequency),
// sources in list order (FP32 complex sums)
// U_t(k) = sum_s Ghat_{t-s}(k) F_s(k) for one frequency k per thread, TT
// targets and NC components at once: each loaded kernel value serves NC
// components and each loaded source value TT targets.  The offset index of
// pair (t, s) is tofs[t] - sofs[s] (flat positions in the offset box,
// precomputed on the host); tofs[t] < 0 marks a padding target.
template <int NC, int TT>
__global__ __launch_bounds__(256) void k_pair_mac(const F2 *__restrict__ Gh, const F2 *__restrict__ Fh,
                                                  const int *__restrict__ tofs, const int *__restrict__ sofs, int ntgt,
                                                  int nsrc, F2 *__restrict__ Uh) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int t0 = blockIdx.y * TT, c0 = blockIdx.z * NC;
    if (k >= kPS) return;
    int ot[TT];
#pragma unroll
    for (int j = 0; j < TT; ++j) ot[j] = t0 + j < ntgt ? tofs[t0 + j] : -1;
    float ar[TT][NC], ai[TT][NC];
#pragma unroll
    for (int j = 0; j < TT; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) ar[j][c] = ai[j][c] = 0.f;
    const F2 *fk = Fh + (size_t)c0 * nsrc * kPS + k;
    const F2 *gk = Gh + k;
    for (int s = 0; s < nsrc; ++s) {
        const int os = sofs[s];
        F2 fv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) fv[c] = fk[((size_t)c * nsrc + s) * kPS];
#pragma unroll
        for (int j = 0; j < TT; ++j) {
            if (ot[j] < 0) continue;   // uniform over the workgroup
            const F2 g = gk[(size_t)(ot[j] - os) * kPS];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                ar[j][c] += g.x * fv[c].x - g.y * fv[c].y;
                ai[j][c] += g.x * fv[c].y + g.y * fv[c].x;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < TT; ++j) {
        if (ot[j] < 0) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c) Uh[((size_t)(c0 + c) * ntgt + t0 + j) * kPS + k] = F2{ar[j][c], ai[j][c]};
    }
}

// The same sum for groups of four targets, walking the sources in ascending
// offset-box position.  When a group's targets are consecutive in x
// (tofs[t_j] = tofs[t_0] + j) and the next source is the x neighbour of the
// last one, the four kernel values needed are the previous four shifted by
// one place, so only one new value is loaded per source instead of four.
template <int NC>
__global__ __launch_bounds__(256) void k_pair_mac_runs(const F2 *__restrict__ Gh, const F2 *__restrict__ Fh,
                                                       const int *__restrict__ tofs, const int *__restrict__ sorder,
                                                       const int *__restrict__ ssorted, const int *__restrict__ groups,
                                                       const int *__restrict__ gconsec, int ntgt, int nsrc, int ngrp,
                                                       F2 *__restrict__ Uh) {
    // frequency chunk major, spread so that each XCD works on one or two
    // chunks: the source spectra of a chunk then stay in that XCD's L2
    const int nchunk = (kPS + 255) / 256;
    const int w = xcd_remap(blockIdx.x, nchunk * ngrp);
    const int k = (w / ngrp) * 256 + threadIdx.x;
    const int grp = w % ngrp, c0 = blockIdx.z * NC;
    if (k >= kPS) return;
    int tj[4], to[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        tj[j] = groups[4 * grp + j];
        to[j] = tj[j] >= 0 ? tofs[tj[j]] : 0;
    }
    const bool consec = gconsec[grp] != 0;   // uniform over the workgroup
    float ar[4][NC], ai[4][NC];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) ar[j][c] = ai[j][c] = 0.f;
    const F2 *fk = Fh + (size_t)c0 * nsrc * kPS + k;
    const F2 *gk = Gh + k;
    F2 g[4] = {F2{0.f, 0.f}, F2{0.f, 0.f}, F2{0.f, 0.f}, F2{0.f, 0.f}};
    int prev = -(1 << 30);
    for (int q = 0; q < nsrc; ++q) {
        const int s = sorder[q], os = ssorted[q];
        F2 fv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) fv[c] = fk[((size_t)c * nsrc + s) * kPS];
        if (consec && os == prev + 1) {
            g[3] = g[2];
            g[2] = g[1];
            g[1] = g[0];
            g[0] = gk[(size_t)(to[0] - os) * kPS];
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) g[j] = tj[j] >= 0 ? gk[(size_t)(to[j] - os) * kPS] : F2{0.f, 0.f};
        }
        prev = os;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                ar[j][c] += g[j].x * fv[c].x - g[j].y * fv[c].y;
                ai[j][c] += g[j].x * fv[c].y + g[j].y * fv[c].x;
            }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (tj[j] < 0) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c) Uh[((size_t)(c0 + c) * ntgt + tj[j]) * kPS + k] = F2{ar[j][c], ai[j][c]};
    }
}

template <int NC>
static void launch_pair_mac(const F2 *Gh, const F2 *Fh, const int *tofs, const int *sofs, int ntgt, int nsrc,
                            int ngrp, F2 *Uh, hipStream_t st) {
    // four targets per thread once there are enough threads to fill the chip
    if (ntgt >= 128)
        hipLaunchKernelGGL((k_pair_mac<NC, 4>), dim3((kPS + 255) / 256, (ntgt + 3) / 4, ngrp), dim3(256), 0, st, Gh, Fh,
                           tofs, sofs, ntgt, nsrc, Uh);
    else
        hipLaunchKernelGGL((k_pair_mac<NC, 1>), dim3((kPS + 255) / 256, ntgt, ngrp), dim3(256), 0, st, Gh, Fh, tofs,
                           sofs, ntgt, nsrc, Uh);
}

}  // namespace lgfib

using namespace lgfib;

namespace lgfib {

// The host-side lists of a source/target pair set: the span D of the block
// offsets, and (int32) source positions, target positions, the sources in
// ascending position with those positions, and the target groups of four.
struct PairLists {
    int D[3] = {0, 0, 0};
    int ngrp = 0;
    long noff = 0;
    std::vector<int> v;
};

static int pair_lists(const Table &tb, const int32_t *src, int nsrc, const int32_t *tgt, int ntgt, PairLists &pl) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = 1 << 30;
        hi[a] = -(1 << 30);
        for (int i = 0; i < nsrc; ++i) {
            lo[a] = std::min(lo[a], (int)src[3 * i + a]);
            hi[a] = std::max(hi[a], (int)src[3 * i + a]);
        }
        for (int i = 0; i < ntgt; ++i) {
            lo[a] = std::min(lo[a], (int)tgt[3 * i + a]);
            hi[a] = std::max(hi[a], (int)tgt[3 * i + a]);
        }
    }
    if (ntgt > 65535) return fail(LGFIB_ERANGE, "block-pair form: more than 65535 target blocks");
    for (int a = 0; a < 3; ++a) {
        pl.D[a] = hi[a] - lo[a];
        if (tb.ext[a] < (pl.D[a] + 1) * kPB - 1) return fail(LGFIB_ERANGE, "block-pair form: table extent too small");
    }
    pl.noff = (long)(2 * pl.D[0] + 1) * (2 * pl.D[1] + 1) * (2 * pl.D[2] + 1);
    if (pl.noff > (1l << 20)) return fail(LGFIB_ERANGE, "block-pair form: block span too large");
    // flat offset-box positions: pair (t, s) uses kernel spectrum tofs[t] - sofs[s]
    const int W0 = 2 * pl.D[0] + 1, W1 = 2 * pl.D[1] + 1;
    const int centre = (pl.D[2] * W1 + pl.D[1]) * W0 + pl.D[0];
    std::vector<int> &ofs = pl.v;
    ofs.assign((size_t)nsrc + ntgt, 0);
    auto flat = [&](const int32_t *b) { return ((b[2] - lo[2]) * W1 + (b[1] - lo[1])) * W0 + (b[0] - lo[0]); };
    for (int i = 0; i < nsrc; ++i) ofs[i] = flat(src + 3 * i);
    for (int i = 0; i < ntgt; ++i) ofs[(size_t)nsrc + i] = flat(tgt + 3 * i) + centre;
    // sources in ascending position; targets in groups of four (consecutive
    // in x where possible) for the run form of the multiply-accumulate
    std::vector<int> sord(nsrc), tord(ntgt);
    for (int i = 0; i < nsrc; ++i) sord[i] = i;
    for (int i = 0; i < ntgt; ++i) tord[i] = i;
    std::sort(sord.begin(), sord.end(), [&](int a, int b) { return ofs[a] < ofs[b]; });
    std::sort(tord.begin(), tord.end(), [&](int a, int b) { return ofs[nsrc + a] < ofs[nsrc + b]; });
    std::vector<int> groups, gcon;
    for (int i = 0; i < ntgt;) {
        int n = 1;
        while (n < 4 && i + n < ntgt && ofs[nsrc + tord[i + n]] == ofs[nsrc + tord[i + n - 1]] + 1) ++n;
        for (int j = 0; j < 4; ++j) groups.push_back(j < n ? tord[i + j] : -1);
        gcon.push_back(n == 4 ? 1 : 0);
        i += n;
    }
    pl.ngrp = (int)gcon.size();
    if (pl.ngrp > 65535) return fail(LGFIB_ERANGE, "block-pair form: too many target groups");
    std::vector<int> ssort(nsrc);
    for (int i = 0; i < nsrc; ++i) ssort[i] = ofs[sord[i]];
    ofs.insert(ofs.end(), sord.begin(), sord.end());
    ofs.insert(ofs.end(), ssort.begin(), ssort.end());
    ofs.insert(ofs.end(), groups.begin(), groups.end());
    ofs.insert(ofs.end(), gcon.begin(), gcon.end());
    return LGFIB_OK;
}

static void launch_pair_ghat(const Table &tb, const int D[3], long noff, F2 *Gh, hipStream_t st) {
    hipLaunchKernelGGL(k_pair_ghat, dim3((unsigned)noff), dim3(256), 0, st, tb.g.as<double>(), tb.ext[0], tb.ext[1],
                       tb.ext[2], D[0], D[1], D[2], Gh);
}

int pair_prepare(lgfib_ctx *ctx, lgf_table_t tbl, const int32_t *src, int nsrc, const int32_t *tgt, int ntgt,
                 PairExec &px, hipStream_t st) {
    int rc;
    const Table &tb = *ctx->tables[tbl];
    PairLists pl;
    if ((rc = pair_lists(tb, src, nsrc, tgt, ntgt, pl))) return rc;
    for (int a = 0; a < 3; ++a) px.D[a] = pl.D[a];
    // kernel spectra of every offset of the span, cached in the context
    auto key = std::make_tuple((int)tbl, px.D[0], px.D[1], px.D[2]);
    auto it = ctx->pair_ghat.find(key);
    if (it == ctx->pair_ghat.end()) {
        auto p = std::make_shared<DevBuf>();
        if ((rc = p->reserve((size_t)pl.noff * kPS * sizeof(F2)))) return rc;
        launch_pair_ghat(tb, px.D, pl.noff, p->as<F2>(), st);
        LGF_HIP(hipGetLastError());
        px.ghat = p;
        const size_t gb = p->bytes;
        ctx->pair_ghat[key] = CacheEnt<DevBuf>{std::move(p), ++ctx->cache_tick, gb};
        cache_trim_all(ctx, 1);
    } else {
        it->second.tick = ++ctx->cache_tick;
        px.ghat = it->second.v;
    }
    px.nsrc = nsrc;
    px.ntgt = ntgt;
    px.ngrp = pl.ngrp;
    if ((rc = px.lists.reserve(sizeof(int) * pl.v.size()))) return rc;
    LGF_HIP(hipMemcpyAsync(px.lists.p, pl.v.data(), sizeof(int) * pl.v.size(), hipMemcpyHostToDevice, st));
    LGF_HIP(hipStreamSynchronize(st));   // the host lists go away on return
    return LGFIB_OK;
}

size_t pair_work_bytes(int n, int ncomp) { return (size_t)ncomp * n * kPS * sizeof(F2); }

// The three launches of one pair-form apply on resolved device lists and
// kernel spectra; wf and wu hold the source and target spectra.
static int pair_launch(lgfib_ctx *ctx, const F2 *Gh, const int *lists, int nsrc, int ntgt, int ngrp, int ncomp, int dft,
                       double dx, const float *f, float *u, void *wf, void *wu, hipStream_t st, bool prof) {
    lgfib_ctx *pctx = prof ? ctx : nullptr;   // no timing events when profiling is not wanted
    const int *sofs = lists, *tofs = sofs + nsrc;
    F2 *Fh = (F2 *)wf, *Uh = (F2 *)wu;
    {
        ProfScope ps(pctx, "k_pair_fwd", st);
        if (dft == LGF_DFT_FFT32)
            hipLaunchKernelGGL(k_pair_fwd, dim3(nsrc, ncomp), dim3(256), 0, st, f, nsrc, Fh);
        else
            hipLaunchKernelGGL(k_pair_fwd_mfma, dim3(nsrc, ncomp), dim3(256), 0, st, f, nsrc, Fh);
        LGF_HIP(hipGetLastError());
    }
    {
        ProfScope ps(pctx, "k_pair_mac", st);
        const int *sorder = tofs + ntgt, *ssorted = sorder + nsrc, *groups = ssorted + nsrc, *gcon = groups + 4 * ngrp;
        const dim3 rg((unsigned)(((kPS + 255) / 256) * ngrp), 1, 1);
        if (ntgt >= 128 && ncomp == 3)
            hipLaunchKernelGGL(k_pair_mac_runs<3>, rg, dim3(256), 0, st, Gh, Fh, tofs, sorder, ssorted, groups, gcon,
                               ntgt, nsrc, ngrp, Uh);
        else if (ntgt >= 128 && ncomp == 1)
            hipLaunchKernelGGL(k_pair_mac_runs<1>, rg, dim3(256), 0, st, Gh, Fh, tofs, sorder, ssorted, groups, gcon,
                               ntgt, nsrc, ngrp, Uh);
        else if (ncomp == 3)
            launch_pair_mac<3>(Gh, Fh, tofs, sofs, ntgt, nsrc, 1, Uh, st);
        else if (ncomp == 2)
            launch_pair_mac<2>(Gh, Fh, tofs, sofs, ntgt, nsrc, 1, Uh, st);
        else if (ncomp == 4)
            launch_pair_mac<4>(Gh, Fh, tofs, sofs, ntgt, nsrc, 1, Uh, st);
        else
            launch_pair_mac<1>(Gh, Fh, tofs, sofs, ntgt, nsrc, ncomp, Uh, st);
        LGF_HIP(hipGetLastError());
    }
    {
        ProfScope ps(pctx, "k_pair_inv", st);
        const float scale = (float)(dx * dx / 4096.0);
        if (dft == LGF_DFT_FFT32)
            hipLaunchKernelGGL(k_pair_inv, dim3(ntgt, ncomp), dim3(256), 0, st, Uh, ntgt, scale, u);
        else
            hipLaunchKernelGGL(k_pair_inv_mfma, dim3(ntgt, ncomp), dim3(256), 0, st, Uh, ntgt, scale, u);
        LGF_HIP(hipGetLastError());
    }
    return LGFIB_OK;
}

int pair_enqueue(lgfib_ctx *ctx, const PairExec &px, int ncomp, int dft, double dx, const float *f, float *u,
                 void *wf, void *wu, hipStream_t st) {
    return pair_launch(ctx, px.ghat->as<F2>(), px.lists.as<int>(), px.nsrc, px.ntgt, px.ngrp, ncomp, dft, dx, f, u, wf,
                       wu, st, true);
}

// ------------------------------------------------ allocation-free variant

// Static device scratch of the allocation-free entry point: the pair lists,
// the kernel spectra of the span, and the source and target spectra.  Each
// device that loads the library holds its own copy until the process ends.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_dev[kMaxDevices];   // scratch's device address, per device
static std::mutex g_scratch_mu;

// Resolve the scratch array's address on the current device (once per device).
int pair_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(LGFIB_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return LGFIB_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(LGFIB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[device] = ptr;
    return LGFIB_OK;
}

static void *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < kMaxDevices ? g_scratch_dev[device] : nullptr;
}

}  // namespace lgfib

using namespace lgfib;

extern "C" int lgf_pair_apply_noalloc(lgfib_ctx *ctx, lgf_table_t tbl, int B, const int32_t *src_blocks, int nsrc,
                                      const int32_t *tgt_blocks, int ntgt, int ncomp, int dft, double dx,
                                      const float *f, float *u, lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgf_pair_apply_noalloc: null context");
    if (tbl < 0 || (size_t)tbl >= ctx->tables.size())
        return fail(LGFIB_ENOTBUILT, "lgf_pair_apply_noalloc: unknown table");
    if (B != kPB) return fail(LGFIB_EINVAL, "lgf_pair_apply_noalloc: blocks must be 8^3");
    if (ncomp < 1 || ncomp > 8) return fail(LGFIB_EINVAL, "lgf_pair_apply_noalloc: ncomp must lie in [1, 8]");
    if (dft != LGF_DFT_FFT32 && dft != LGF_DFT_BF16X3) return fail(LGFIB_EINVAL, "lgf_pair_apply_noalloc: unknown dft");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LGFIB_EINVAL, "lgf_pair_apply_noalloc: dx must be positive");
    if (nsrc < 0 || ntgt < 0) return fail(LGFIB_EINVAL, "lgf_pair_apply_noalloc: negative block count");
    if ((nsrc > 0 && (!src_blocks || !f)) || (ntgt > 0 && (!tgt_blocks || !u)))
        return fail(LGFIB_EINVAL, "lgf_pair_apply_noalloc: null pointer");
    int rc;
    if ((rc = validate_blocks(src_blocks, nsrc, "source blocks")) || (rc = validate_blocks(tgt_blocks, ntgt, "target blocks")))
        return rc;
    if (ntgt == 0) return LGFIB_OK;
    const Table &tb = *ctx->tables[tbl];
    PairLists pl;
    if (nsrc > 0 && (rc = pair_lists(tb, src_blocks, nsrc, tgt_blocks, ntgt, pl))) return rc;
    // scratch layout: lists | kernel spectra | source spectra | target spectra
    auto up = [](size_t n) { return (n + 255) / 256 * 256; };
    const size_t b_lists = up(sizeof(int) * pl.v.size()), b_ghat = up((size_t)pl.noff * kPS * sizeof(F2));
    const size_t b_f = up(pair_work_bytes(nsrc, ncomp)), b_u = up(pair_work_bytes(ntgt, ncomp));
    const size_t need = b_lists + b_ghat + b_f + b_u;
    if (nsrc > 0 && need > kNoAllocBytes)
        return fail(LGFIB_ERANGE, "lgf_pair_apply_noalloc: this apply needs " + std::to_string(need) +
                                      " bytes of scratch; the static scratch holds " + std::to_string(kNoAllocBytes));
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (nsrc == 0) {
        hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)std::min<size_t>(((size_t)ncomp * ntgt * 512 + 255) / 256, 65535)),
                           dim3(256), 0, st, u, (size_t)ncomp * ntgt * 512);
        LGF_HIP(hipGetLastError());
        return LGFIB_OK;
    }
    unsigned char *base = (unsigned char *)scratch_of(ctx->device);
    if (!base) return fail(LGFIB_ENOTBUILT, "lgf_pair_apply_noalloc: scratch not resolved on this device");
    int *lists = (int *)base;
    F2 *Gh = (F2 *)(base + b_lists);
    void *wf = base + b_lists + b_ghat, *wu = base + b_lists + b_ghat + b_f;
    LGF_HIP(hipMemcpyAsync(lists, pl.v.data(), sizeof(int) * pl.v.size(), hipMemcpyHostToDevice, st));
    launch_pair_ghat(tb, pl.D, pl.noff, Gh, st);
    LGF_HIP(hipGetLastError());
    rc = pair_launch(ctx, Gh, lists, nsrc, ntgt, pl.ngrp, ncomp, dft, dx, f, u, wf, wu, st, false);
    LGF_HIP(hipStreamSynchronize(st));   // the host lists go away on return
    return rc;
}

extern "C" int lgf_pair_apply(lgfib_ctx *ctx, lgf_table_t tbl, int B, const int32_t *src_blocks, int nsrc,
                              const int32_t *tgt_blocks, int ntgt, int ncomp, int dft, double dx, const float *f,
                              float *u, lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgf_pair_apply: null context");
    if (tbl < 0 || (size_t)tbl >= ctx->tables.size()) return fail(LGFIB_ENOTBUILT, "lgf_pair_apply: unknown table");
    if (B != kPB) return fail(LGFIB_EINVAL, "lgf_pair_apply: blocks must be 8^3");
    if (ncomp < 1 || ncomp > 8) return fail(LGFIB_EINVAL, "lgf_pair_apply: ncomp must lie in [1, 8]");
    if (dft != LGF_DFT_FFT32 && dft != LGF_DFT_BF16X3) return fail(LGFIB_EINVAL, "lgf_pair_apply: unknown dft");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LGFIB_EINVAL, "lgf_pair_apply: dx must be positive");
    if (nsrc < 0 || ntgt < 0) return fail(LGFIB_EINVAL, "lgf_pair_apply: negative block count");
    if ((nsrc > 0 && (!src_blocks || !f)) || (ntgt > 0 && (!tgt_blocks || !u)))
        return fail(LGFIB_EINVAL, "lgf_pair_apply: null pointer");
    int rc;
    if ((rc = validate_blocks(src_blocks, nsrc, "source blocks")) || (rc = validate_blocks(tgt_blocks, ntgt, "target blocks")))
        return rc;
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (ntgt == 0) return LGFIB_OK;
    if (nsrc == 0) {
        LGF_HIP(hipMemsetAsync(u, 0, (size_t)ncomp * ntgt * 512 * 4, st));
        return LGFIB_OK;
    }
    PairExec px;
    if ((rc = pair_prepare(ctx, tbl, src_blocks, nsrc, tgt_blocks, ntgt, px, st))) return rc;
    if ((rc = ctx->work1.reserve(pair_work_bytes(nsrc, ncomp))) || (rc = ctx->work2.reserve(pair_work_bytes(ntgt, ncomp))))
        return rc;
    rc = pair_enqueue(ctx, px, ncomp, dft, dx, f, u, ctx->work1.p, ctx->work2.p, st);
    LGF_HIP(hipStreamSynchronize(st));   // px (its block lists) is released on return
    return rc;
}
