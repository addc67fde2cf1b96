// if_apply.hip -- the integrating factor u = E(a) f on a block set.
//
// E(a) = exp(aL) has the LGF prod_q e^{-2a} I_{n_q}(2a) (App. A,
// Eq. lgf_intfac): a separable, even, rapidly decaying stencil, truncated
// where the 1D weight falls below 1e-14 in FP64 and 2^-28 in FP32 (half-width r).  One workgroup owns
// one target block and one component; thread (x, y) owns the output column
// (x, y, 0..B-1).  The (B+2r)^2 halo of each input z-plane is staged in LDS
// (neighbour source blocks looked up once per call in a host-built table),
// filtered along x, then along y, and the filtered plane is accumulated into
// the B z-outputs of every column with the z weights.  HBM sees each source
// value once per neighbouring target block (mostly L2 hits) and each output
// once.
//
// Small blocks (B <= 8) have too little work per plane for that streaming
// scheme to hide its latency, so when the whole (B+2r)^3 halo fits in LDS a
// 512-thread workgroup loads all of it at once (every load in flight
// together) and filters x, y, z in three LDS passes.
#include <cmath>

#include "conv_common.h"

namespace lgfib {

template <typename Real, int B>
__global__ __launch_bounds__(B * B) void k_if_apply(const Real *__restrict__ f, Real *__restrict__ u,
                                                    const int *__restrict__ nbr, const double *__restrict__ wts,
                                                    int r, int rb, int nsrc, int ntgt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int H = B + 2 * r;
    Real *w = reinterpret_cast<Real *>(smem_raw);   // 2r+1 weights, index d + r
    Real *Pl = w + (2 * r + 1);                     // H x H input plane
    Real *Q = Pl + H * H;                           // H x B x-filtered plane
    int *slots = reinterpret_cast<int *>(Q + H * B);   // (2rb+1)^3 neighbour slots
    const int t = blockIdx.x, c = blockIdx.y;
    const int tid = threadIdx.x;
    const int W = 2 * rb + 1, W3 = W * W * W;
    constexpr int B2 = B * B, B3 = B2 * B;
    for (int i = tid; i <= 2 * r; i += B2) w[i] = (Real)wts[abs(i - r)];
    for (int i = tid; i < W3; i += B2) slots[i] = nbr[(size_t)t * W3 + i];
    __syncthreads();
    const int tx = tid % B, ty = tid / B;
    Real acc[B];
#pragma unroll
    for (int z = 0; z < B; ++z) acc[z] = 0;
    const Real *fc = f + (size_t)c * nsrc * B3;
    for (int zi = -r; zi < B + r; ++zi) {
        const int bz = (zi + rb * B) / B - rb;   // floor(zi / B)
        const int lz = zi - bz * B;
        // skip planes whose neighbour row of blocks is entirely absent
        bool any = false;
        for (int i = 0; i < W * W; ++i) any |= slots[((bz + rb) * W) * W + i] >= 0;
        if (!any) continue;
        for (int i = tid; i < H * H; i += B2) {
            const int xx = i % H - r, yy = i / H - r;
            const int bx = (xx + rb * B) / B - rb, by = (yy + rb * B) / B - rb;
            const int slot = slots[((bz + rb) * W + (by + rb)) * W + (bx + rb)];
            Real v = 0;
            if (slot >= 0) v = fc[(size_t)slot * B3 + lz * B2 + (yy - by * B) * B + (xx - bx * B)];
            Pl[i] = v;
        }
        __syncthreads();
        for (int i = tid; i < H * B; i += B2) {
            const int x = i % B, yy = i / B;
            const Real *row = Pl + yy * H + x;   // input x + d sits at row[d + r]
            Real s = 0;
            for (int d = 0; d <= 2 * r; ++d) s += w[d] * row[d];
            Q[i] = s;
        }
        __syncthreads();
        Real v = 0;
        for (int d = 0; d <= 2 * r; ++d) v += w[d] * Q[(ty + d) * B + tx];
#pragma unroll
        for (int z = 0; z < B; ++z) {
            const int dz = z - zi;
            if (dz >= -r && dz <= r) acc[z] += w[dz + r] * v;
        }
        __syncthreads();
    }
    Real *uc = u + ((size_t)c * ntgt + t) * B3;
#pragma unroll
    for (int z = 0; z < B; ++z) uc[z * B2 + ty * B + tx] = acc[z];
}

constexpr int kHaloThreads = 512;

// LDS: A [H^3] halo (reused for the y-filtered H x B x B), Q [H][H][B]
// x-filtered, w [2r+1], slots [(2rb+1)^3]
template <typename Real, int B>
__global__ __launch_bounds__(kHaloThreads) void k_if_halo(const Real *__restrict__ f, Real *__restrict__ u,
                                                          const int *__restrict__ nbr, const double *__restrict__ wts,
                                                          int r, int rb, int nsrc, int ntgt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int H = B + 2 * r, H3 = H * H * H;
    const int W = 2 * rb + 1, W3 = W * W * W;
    constexpr int B2 = B * B, B3 = B2 * B;
    Real *A = reinterpret_cast<Real *>(smem_raw);
    Real *Q = A + H3;
    Real *w = Q + H * H * B;
    int *slots = reinterpret_cast<int *>(w + 2 * r + 1);
    const int t = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    for (int i = tid; i <= 2 * r; i += kHaloThreads) w[i] = (Real)wts[abs(i - r)];
    for (int i = tid; i < W3; i += kHaloThreads) slots[i] = nbr[(size_t)t * W3 + i];
    __syncthreads();
    const Real *fc = f + (size_t)c * nsrc * B3;
    // halo rows (z, y) are walked 16 at a time by 32 lanes each (H <= 32 on
    // this path), keeping (y, z) incrementally: no runtime divisions
    {
        const int x = tid & 31;
        const int gx = x - r;
        const int bx = (gx + rb * B) / B - rb, lx = gx - bx * B;
        int y = tid >> 5, z = 0;
        for (int row = tid >> 5; row < H * H; row += kHaloThreads / 32) {
            while (y >= H) {
                y -= H;
                ++z;
            }
            if (x < H) {
                const int gy = y - r, gz = z - r;
                const int by = (gy + rb * B) / B - rb, bz = (gz + rb * B) / B - rb;
                const int slot = slots[((bz + rb) * W + (by + rb)) * W + (bx + rb)];
                Real v = 0;
                if (slot >= 0) v = fc[(size_t)slot * B3 + ((gz - bz * B) * B + (gy - by * B)) * B + lx];
                A[row * H + x] = v;
            }
            y += kHaloThreads / 32;
        }
    }
    __syncthreads();
    // x: Q[z][y][xo] = sum_d w[d] A[z][y][xo + d]
    for (int i = tid; i < H * H * B; i += kHaloThreads) {
        const int xo = i % B, row = i / B;
        const Real *a = A + row * H + xo;
        Real s = 0;
        for (int d = 0; d <= 2 * r; ++d) s += w[d] * a[d];
        Q[i] = s;
    }
    __syncthreads();
    // y: A[z][yo][xo] = sum_d w[d] Q[z][yo + d][xo]
    for (int i = tid; i < H * B2; i += kHaloThreads) {
        const int xo = i % B, yo = (i / B) % B, z = i / B2;
        const Real *q = Q + (z * H + yo) * B + xo;
        Real s = 0;
        for (int d = 0; d <= 2 * r; ++d) s += w[d] * q[d * B];
        A[i] = s;
    }
    __syncthreads();
    // z: u[zo][yo][xo] = sum_d w[d] A[zo + d][yo][xo]
    Real *uc = u + ((size_t)c * ntgt + t) * B3;
    for (int i = tid; i < B3; i += kHaloThreads) {
        const Real *a = A + i;
        Real s = 0;
        for (int d = 0; d <= 2 * r; ++d) s += w[d] * a[d * B2];
        uc[i] = s;
    }
}

// The same halo scheme with the radius a template constant: the taps unroll
// (weights in registers, all loads of an output in flight together) and the
// x pass keeps a whole halo row in registers, producing its B outputs from
// one read of the row.  The halo's row stride is padded to an odd length
// against LDS bank conflicts.
template <typename Real, int B, int R>
__global__ __launch_bounds__(kHaloThreads) void k_if_halo_r(const Real *__restrict__ f, Real *__restrict__ u,
                                                            const int *__restrict__ nbr,
                                                            const double *__restrict__ wts, int rb, int nsrc,
                                                            int ntgt) {
    constexpr int H = B + 2 * R, HP = H | 1, T = 2 * R + 1;
    constexpr int B2 = B * B, B3 = B2 * B;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Real *A = reinterpret_cast<Real *>(smem_raw);   // [H][H][HP] halo, later [H][B][B] y-filtered
    Real *Q = A + H * H * HP;                       // [H][H][B] x-filtered
    int *slots = reinterpret_cast<int *>(Q + H * H * B);
    const int W = 2 * rb + 1, W3 = W * W * W;
    const int t = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    Real w[T];
#pragma unroll
    for (int d = 0; d < T; ++d) w[d] = (Real)wts[d < R ? R - d : d - R];
    for (int i = tid; i < W3; i += kHaloThreads) slots[i] = nbr[(size_t)t * W3 + i];
    __syncthreads();
    const Real *fc = f + (size_t)c * nsrc * B3;
    {
        // 32 lanes per halo row, 16 rows per pass: every load of the thread
        // is issued before the first LDS store waits on one
        constexpr int NR = (H * H + 15) / 16;
        const int x = tid & 31;
        const int gx = x - R;
        const int bx = (gx + rb * B) / B - rb, lx = gx - bx * B;
        Real v[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int row = (tid >> 5) + 16 * k;
            v[k] = 0;
            if (x < H && row < H * H) {
                const int y = row % H, z = row / H;
                const int gy = y - R, gz = z - R;
                const int by = (gy + rb * B) / B - rb, bz = (gz + rb * B) / B - rb;
                const int slot = slots[((bz + rb) * W + (by + rb)) * W + (bx + rb)];
                if (slot >= 0) v[k] = fc[(size_t)slot * B3 + ((gz - bz * B) * B + (gy - by * B)) * B + lx];
            }
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int row = (tid >> 5) + 16 * k;
            if (x < H && row < H * H) A[row * HP + x] = v[k];
        }
    }
    __syncthreads();
    // x: a thread per halo row
    for (int row = tid; row < H * H; row += kHaloThreads) {
        Real v[H];
#pragma unroll
        for (int i = 0; i < H; ++i) v[i] = A[row * HP + i];
#pragma unroll
        for (int xo = 0; xo < B; ++xo) {
            Real s = 0;
#pragma unroll
            for (int d = 0; d < T; ++d) s += w[d] * v[xo + d];
            Q[row * B + xo] = s;
        }
    }
    __syncthreads();
    // y: A[z][yo][xo] = sum_d w[d] Q[z][yo + d][xo]
    for (int i = tid; i < H * B2; i += kHaloThreads) {
        const int xo = i % B, yo = (i / B) % B, z = i / B2;
        const Real *q = Q + (z * H + yo) * B + xo;
        Real s = 0;
#pragma unroll
        for (int d = 0; d < T; ++d) s += w[d] * q[d * B];
        A[i] = s;
    }
    __syncthreads();
    Real *uc = u + ((size_t)c * ntgt + t) * B3;
    for (int i = tid; i < B3; i += kHaloThreads) {
        const Real *a = A + i;
        Real s = 0;
#pragma unroll
        for (int d = 0; d < T; ++d) s += w[d] * a[d * B2];
        uc[i] = s;
    }
}

// Blocks of 16^3 (and 8^3) with a one-block halo (H = B + 2R <= 32 for
// B = 16): one workgroup per target block and component (thread count
// below).  A thread per halo row reads its H values from the three source
// blocks along x and keeps the B x-filtered outputs in LDS (z planes of
// [H][B+1]); then a thread per (z, x) column filters along y in place
// through registers, and a thread per (y, x) column filters along z and
// writes the B^3 outputs to HBM.  Workgroups are ordered XCD-aware:
// consecutive ids go round-robin to the 8 XCDs, so each XCD is handed a
// contiguous run of targets and the halos that neighbouring targets share
// meet in its L2.
constexpr int kCubeThreads = 1024;
// threads of the row kernel: on 8^3 blocks one per halo row (H^2 rounded up
// to whole wavefronts); on 16^3 blocks the same up to radius 5, then 512 up
// to radius 8, the rows beyond wrapping to a second pass (one thread per row
// measured slower there); 1024 elsewhere
constexpr int if_rows_threads(int B, int R) {
    const int H = B + 2 * R;
    if (B == 8) return (H * H + 63) / 64 * 64;   // H <= 24: at most 576 threads
    if (B != 16) return kCubeThreads;
    if (H * H <= 704) return (H * H + 63) / 64 * 64;
    return H * B <= 512 ? 512 : kCubeThreads;
}
// LDS stride of one z plane of the x-filtered halo ([H][BP] values, BP = B + 1):
// the smallest at or above H (B + 1) that is an odd multiple of B, so the y
// pass's lanes (64 / B planes of B columns each) fall on distinct banks --
// unless the padding would leave room for fewer workgroups per CU
// (160 KiB of LDS)
constexpr int if_rows_plane(int B, int R, int es) {
    const int H = B + 2 * R, base = H * (B + 1);
    int ps = base;
    while (ps % (2 * B) != B) ++ps;
    const long bytes_base = (long)es * H * base + 4 * 27, bytes_pad = (long)es * H * ps + 4 * 27;
    return 163840 / bytes_pad >= 163840 / bytes_base ? ps : base;
}


// 16-byte vectors of the element type
template <typename Real> struct Vec16;
template <> struct Vec16<float> {
    using T = float4;
    static constexpr int n = 4;
    __device__ __forceinline__ static T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <> struct Vec16<double> {
    using T = double2;
    static constexpr int n = 2;
    __device__ __forceinline__ static T zero() { return make_double2(0.0, 0.0); }
};
__device__ __forceinline__ float vlane(const float4 &v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
__device__ __forceinline__ double vlane(const double2 &v, int i) { return i == 0 ? v.x : v.y; }

// Row loads are 16-byte vectors (float4 / double2).
template <typename Real, int B, int R>
__global__ __launch_bounds__(if_rows_threads(B, R)) void k_if_rows(const Real *__restrict__ f, Real *__restrict__ u,
                                                          const int *__restrict__ nbr, const double *__restrict__ wts,
                                                          int nsrc, int ntgt, int ncomp) {
    constexpr int H = B + 2 * R, BP = B + 1, PS = if_rows_plane(B, R, sizeof(Real)), T = 2 * R + 1;
    constexpr int B2 = B * B, B3 = B2 * B;
    constexpr int W = 3, W3 = 27;
    using V = typename Vec16<Real>::T;
    constexpr int VW = Vec16<Real>::n, RQ = (R + VW - 1) / VW;   // vectors per side halo
    constexpr int NT = if_rows_threads(B, R);
    static_assert(H * B <= NT && B * B <= NT && R <= B, "a thread per (z, x) column");
    static_assert(B % VW == 0 && VW * RQ <= B, "side halos in whole vectors of one block");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Real *Q = reinterpret_cast<Real *>(smem_raw);   // [H][PS] planes of [H][BP], x-filtered
    int *slots = reinterpret_cast<int *>(Q + H * PS);
    const int item = xcd_remap(blockIdx.x, ntgt * ncomp);
    const int c = item / ntgt, t = item % ntgt, tid = threadIdx.x;
    Real w[T];
#pragma unroll
    for (int d = 0; d < T; ++d) w[d] = (Real)wts[d < R ? R - d : d - R];
    if (tid < W3) slots[tid] = nbr[(size_t)t * W3 + tid];
    __syncthreads();
    const Real *fc = f + (size_t)c * nsrc * B3;
    Real o[B];
    for (int row = tid; row < H * H; row += NT) {
        const int gy = row % H - R, gz = row / H - R;
        const int by = gy < 0 ? -1 : (gy >= B ? 1 : 0), bz = gz < 0 ? -1 : (gz >= B ? 1 : 0);
        const int rowoff = ((gz - bz * B) * B + (gy - by * B)) * B;
        const int *sl = slots + ((bz + 1) * W + (by + 1)) * W;
        Real r[H];
        // x in [-R, 0) from block -1, [0, B) from block 0, [B, B + R) from block +1
        const int s0 = sl[0], s1 = sl[1], s2 = sl[2];
        // the side halos come in aligned 16-byte vectors covering the R cells
        // next to the block (the unused lanes of the left vectors are dropped)
        const Real *p0 = fc + (size_t)s0 * B3 + rowoff + B - VW * RQ, *p1 = fc + (size_t)s1 * B3 + rowoff,
                   *p2 = fc + (size_t)s2 * B3 + rowoff;
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            const V v = s0 >= 0 ? reinterpret_cast<const V *>(p0)[q] : Vec16<Real>::zero();
#pragma unroll
            for (int i = 0; i < VW; ++i) {
                const int e = VW * q + i - (VW * RQ - R);   // halo index of lane i
                if (e >= 0) r[e] = vlane(v, i);
            }
        }
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            const V v = s2 >= 0 ? reinterpret_cast<const V *>(p2)[q] : Vec16<Real>::zero();
#pragma unroll
            for (int i = 0; i < VW; ++i)
                if (VW * q + i < R) r[R + B + VW * q + i] = vlane(v, i);
        }
        if constexpr (sizeof(Real) == 4) {
#pragma unroll
            for (int q = 0; q < B / 4; ++q) {
                const float4 v = s1 >= 0 ? reinterpret_cast<const float4 *>(p1)[q] : make_float4(0.f, 0.f, 0.f, 0.f);
                r[R + 4 * q] = v.x, r[R + 4 * q + 1] = v.y, r[R + 4 * q + 2] = v.z, r[R + 4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < B / 2; ++q) {
                const double2 v = s1 >= 0 ? reinterpret_cast<const double2 *>(p1)[q] : make_double2(0.0, 0.0);
                r[R + 2 * q] = v.x, r[R + 2 * q + 1] = v.y;
            }
        }
#pragma unroll
        for (int xo = 0; xo < B; ++xo) {
            Real sum = 0;
#pragma unroll
            for (int d = 0; d < T; ++d) sum += w[d] * r[xo + d];
            Q[(row / H) * PS + (row % H) * BP + xo] = sum;
        }
    }
    __syncthreads();
    // y: thread per (z, x) column, in place
    const int zc = tid / B, xc = tid % B;
    if (tid < H * B) {
        Real r[H];
#pragma unroll
        for (int y = 0; y < H; ++y) r[y] = Q[zc * PS + y * BP + xc];
#pragma unroll
        for (int yo = 0; yo < B; ++yo) {
            Real s = 0;
#pragma unroll
            for (int d = 0; d < T; ++d) s += w[d] * r[yo + d];
            o[yo] = s;
        }
    }
    __syncthreads();
    if (tid < H * B) {
#pragma unroll
        for (int yo = 0; yo < B; ++yo) Q[zc * PS + yo * BP + xc] = o[yo];
    }
    __syncthreads();
    if (tid < B2) {
        const int yo = tid / B, xo = tid % B;
        Real r[H];
#pragma unroll
        for (int z = 0; z < H; ++z) r[z] = Q[z * PS + yo * BP + xo];
        Real *uc = u + ((size_t)c * ntgt + t) * B3 + yo * B + xo;
#pragma unroll
        for (int zo = 0; zo < B; ++zo) {
            Real s = 0;
#pragma unroll
            for (int d = 0; d < T; ++d) s += w[d] * r[zo + d];
            uc[zo * B2] = s;
        }
    }
}

static size_t rows_lds_bytes(int B, int r, size_t es = 4) {
    const size_t H = (size_t)B + 2 * r;
    return es * H * (size_t)if_rows_plane(B, r, (int)es) + 4 * 27;
}

template <typename Real, int B, int R>
static int launch_cube(size_t sm, int ntgt, int ncomp, hipStream_t st, const Real *f, Real *u, const int *nbr,
                       const double *w, int nsrc);

static size_t halo_r_lds_bytes(int B, int r, int rb, size_t es) {
    const size_t H = (size_t)B + 2 * r, HP = H | 1, W = 2 * (size_t)rb + 1;
    return es * (H * H * HP + H * H * B) + 4 * W * W * W;
}

static size_t halo_lds_bytes(int B, int r, int rb, size_t es) {
    const size_t H = (size_t)B + 2 * r, W = 2 * (size_t)rb + 1;
    return es * (H * H * H + H * H * B + 2 * r + 1) + 4 * W * W * W;
}

static int max_lds_per_block(int device) {
    static int cached[64] = {0};
    if (device < 0 || device >= 64) return 65536;
    if (!cached[device]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || v <= 0)
            v = 65536;
        cached[device] = v;
    }
    return cached[device];
}

template <typename Real, int B>
static int launch_halo(size_t sm, dim3 grid, hipStream_t st, const Real *f, Real *u, const int *nbr, const double *w,
                       int r, int rb, int nsrc, int ntgt) {
    // raise the kernel's dynamic LDS limit once, to the device maximum (kept
    // out of the launch path so that launches can be captured into graphs)
    static bool raised = false;
    if (!raised) {
        LGF_HIP(hipFuncSetAttribute((const void *)k_if_halo<Real, B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    max_lds_per_block(0)));
        raised = true;
    }
    hipLaunchKernelGGL((k_if_halo<Real, B>), grid, dim3(kHaloThreads), sm, st, f, u, nbr, w, r, rb, nsrc, ntgt);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename Real, int B, int R>
static int launch_halo_r(size_t sm, dim3 grid, hipStream_t st, const Real *f, Real *u, const int *nbr,
                         const double *w, int rb, int nsrc, int ntgt) {
    static bool raised = false;
    if (!raised) {
        LGF_HIP(hipFuncSetAttribute((const void *)k_if_halo_r<Real, B, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    max_lds_per_block(0)));
        raised = true;
    }
    hipLaunchKernelGGL((k_if_halo_r<Real, B, R>), grid, dim3(kHaloThreads), sm, st, f, u, nbr, w, rb, nsrc, ntgt);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename Real, int B, int R>
static int launch_cube(size_t sm, int ntgt, int ncomp, hipStream_t st, const Real *f, Real *u, const int *nbr,
                       const double *w, int nsrc) {
    static bool raised = false;
    if (!raised) {
        LGF_HIP(hipFuncSetAttribute((const void *)k_if_rows<Real, B, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    max_lds_per_block(0)));
        raised = true;
    }
    hipLaunchKernelGGL((k_if_rows<Real, B, R>), dim3(ntgt * ncomp), dim3(if_rows_threads(B, R)), sm, st, f, u, nbr, w, nsrc,
                       ntgt, ncomp);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename Real>
static int launch_if(lgfib_ctx *ctx, int B, int r, int rb, int ntgt, int ncomp, int nsrc, const Real *f, Real *u, const int *nbr,
                     const double *w, hipStream_t st) {
    if constexpr (sizeof(Real) == 4) {
        if (B == 16 && rb == 1 && ((r >= 3 && r <= 8) || r == 12) &&
            rows_lds_bytes(B, r) <= (size_t)max_lds_per_block(ctx->device) && (long)ntgt * ncomp < (1l << 31)) {
            ProfScope ps(ctx, "k_if_apply", st);
            const size_t sm = rows_lds_bytes(B, r);
            switch (r) {
            case 3: return launch_cube<float, 16, 3>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
            case 4: return launch_cube<float, 16, 4>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
            case 5: return launch_cube<float, 16, 5>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
            case 6: return launch_cube<float, 16, 6>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
            case 7: return launch_cube<float, 16, 7>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
            case 8: return launch_cube<float, 16, 8>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
            default: return launch_cube<float, 16, 12>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
            }
        }
    }
    // blocks of 8^3 too (the force solve's E(a), the drivers' FP64 E(a)):
    // faster than staging the whole halo in LDS first
    if (B == 8 && rb == 1 && r >= 3 && r <= 8 &&
        rows_lds_bytes(B, r, sizeof(Real)) <= (size_t)max_lds_per_block(ctx->device) &&
        (long)ntgt * ncomp < (1l << 31)) {
        ProfScope ps(ctx, "k_if_apply", st);
        const size_t sm = rows_lds_bytes(B, r, sizeof(Real));
        switch (r) {
        case 3: return launch_cube<Real, 8, 3>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
        case 4: return launch_cube<Real, 8, 4>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
        case 5: return launch_cube<Real, 8, 5>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
        case 6: return launch_cube<Real, 8, 6>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
        case 7: return launch_cube<Real, 8, 7>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
        default: return launch_cube<Real, 8, 8>(sm, ntgt, ncomp, st, f, u, nbr, w, nsrc);
        }
    }
    if (B == 8 && (r == 6 || r == 7 || r == 8 || r == 12)) {
        const size_t hs = halo_r_lds_bytes(B, r, rb, sizeof(Real));
        if (hs <= (size_t)max_lds_per_block(ctx->device)) {
            ProfScope ps(ctx, "k_if_apply", st);
            dim3 grid(ntgt, ncomp);
            switch (r) {
            case 6: return launch_halo_r<Real, 8, 6>(hs, grid, st, f, u, nbr, w, rb, nsrc, ntgt);
            case 7: return launch_halo_r<Real, 8, 7>(hs, grid, st, f, u, nbr, w, rb, nsrc, ntgt);
            case 8: return launch_halo_r<Real, 8, 8>(hs, grid, st, f, u, nbr, w, rb, nsrc, ntgt);
            default: return launch_halo_r<Real, 8, 12>(hs, grid, st, f, u, nbr, w, rb, nsrc, ntgt);
            }
        }
    }
    if (B <= 8 && B + 2 * r <= 32) {
        const size_t hs = halo_lds_bytes(B, r, rb, sizeof(Real));
        if (hs <= (size_t)max_lds_per_block(ctx->device)) {
            ProfScope ps(ctx, "k_if_apply", st);
            dim3 grid(ntgt, ncomp);
            if (B == 4) return launch_halo<Real, 4>(hs, grid, st, f, u, nbr, w, r, rb, nsrc, ntgt);
            return launch_halo<Real, 8>(hs, grid, st, f, u, nbr, w, r, rb, nsrc, ntgt);
        }
    }
    const int H = B + 2 * r, W = 2 * rb + 1;
    const size_t sm = sizeof(Real) * (size_t)(2 * r + 1 + H * H + H * B) + sizeof(int) * (size_t)W * W * W;
    if (sm > 160 * 1024) return fail(LGFIB_ERANGE, "lgf_if_apply: stencil too wide for LDS");
    dim3 grid(ntgt, ncomp);
    ProfScope ps(ctx, "k_if_apply", st);
    switch (B) {
    case 4: hipLaunchKernelGGL((k_if_apply<Real, 4>), grid, dim3(16), sm, st, f, u, nbr, w, r, rb, nsrc, ntgt); break;
    case 8: hipLaunchKernelGGL((k_if_apply<Real, 8>), grid, dim3(64), sm, st, f, u, nbr, w, r, rb, nsrc, ntgt); break;
    case 16:
        hipLaunchKernelGGL((k_if_apply<Real, 16>), grid, dim3(256), sm, st, f, u, nbr, w, r, rb, nsrc, ntgt);
        break;
    default:
        hipLaunchKernelGGL((k_if_apply<Real, 32>), grid, dim3(1024), sm, st, f, u, nbr, w, r, rb, nsrc, ntgt);
        break;
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// Truncation of the 1D factor by the precision of the apply.  FP64 drops
// the weights below 1e-14.  FP32 drops those below 2^-28: the factors fall
// off faster than geometrically (w_{j+1} / w_j < a / (j + 1)), so the
// neglected tail along an axis is about twice the first dropped weight and,
// over the three axes, stays below FP32's unit roundoff 2^-24 relative to
// the largest source value.
constexpr double kIfCutoff64 = LGF_IF_CUTOFF_F64;
constexpr double kIfCutoff32 = LGF_IF_CUTOFF_F32;

// 1D weights e^{-2a} I_j(2a), j = 0..r, cached per (a, precision) on the device.
int get_if_weights(lgfib_ctx *ctx, double a, int prec, int *radius, const double **dev) {
    const auto key = std::make_pair(a, prec == LGF_F32 ? (int)LGF_F32 : (int)LGF_F64);
    auto it = ctx->if_weights.find(key);
    if (it != ctx->if_weights.end()) {
        *radius = it->second.first;
        *dev = it->second.second->as<double>();
        return LGFIB_OK;
    }
    int r = 0;
    std::vector<double> w(4097);
    int rc = lgf_if_weights(ctx, a, key.second == LGF_F32 ? kIfCutoff32 : kIfCutoff64, w.data(), (int)w.size(), &r);
    if (rc) return rc;
    auto buf = std::make_unique<DevBuf>();
    if ((rc = buf->reserve(sizeof(double) * (r + 1)))) return rc;
    LGF_HIP(hipMemcpy(buf->p, w.data(), sizeof(double) * (r + 1), hipMemcpyHostToDevice));
    *radius = r;
    *dev = buf->as<double>();
    ctx->if_weights[key] = std::make_pair(r, std::move(buf));
    return LGFIB_OK;
}

}  // namespace lgfib

using namespace lgfib;

extern "C" int lgf_if_apply(lgfib_ctx *ctx, double a, int B, const int32_t *src_blocks, int nsrc,
                            const int32_t *tgt_blocks, int ntgt, int ncomp, int prec, const void *f, void *u,
                            lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgf_if_apply: null context");
    if (B != 4 && B != 8 && B != 16 && B != 32) return fail(LGFIB_EINVAL, "lgf_if_apply: B must be 4, 8, 16 or 32");
    if (ncomp < 1 || ncomp > 8) return fail(LGFIB_EINVAL, "lgf_if_apply: ncomp must lie in [1, 8]");
    if (prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, "lgf_if_apply: prec must be LGF_F32 or LGF_F64");
    if (!(a >= 0.0) || a > 64.0) return fail(LGFIB_EINVAL, "lgf_if_apply: a must lie in [0, 64]");
    if (nsrc < 0 || ntgt < 0) return fail(LGFIB_EINVAL, "lgf_if_apply: negative block count");
    const size_t es = prec == LGF_F64 ? 8 : 4, B3 = (size_t)B * B * B;
    const size_t fbytes = (size_t)ncomp * nsrc * B3 * es, ubytes = (size_t)ncomp * ntgt * B3 * es;
    if ((nsrc > 0 && !f) || (ntgt > 0 && !u)) return fail(LGFIB_EINVAL, "lgf_if_apply: null field pointer");
    if (nsrc > 0 && ntgt > 0) {
        const char *pf = (const char *)f, *pu = (const char *)u;
        if (pf < pu + ubytes && pu < pf + fbytes) return fail(LGFIB_EINVAL, "lgf_if_apply: f and u overlap");
    }
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    // block lists are validated when their plan is built (a cached plan
    // matched the same lists before)
    if ((nsrc > 0 && !src_blocks) || (ntgt > 0 && !tgt_blocks)) return fail(LGFIB_EINVAL, "null block list");
    int rc = LGFIB_OK;
    if (ntgt == 0) return LGFIB_OK;
    if (nsrc == 0) {
        LGF_HIP(hipMemsetAsync(u, 0, ubytes, st));
        return LGFIB_OK;
    }
    int r = 0;
    const double *w = nullptr;
    if ((rc = get_if_weights(ctx, a, prec, &r, &w))) return rc;
    std::shared_ptr<IfPlan> plan;
    if ((rc = get_if_plan(ctx, B, r, src_blocks, nsrc, tgt_blocks, ntgt, plan))) return rc;
    const int rb = plan->rb;
    if (prec == LGF_F64)
        return launch_if<double>(ctx, B, r, rb, ntgt, ncomp, nsrc, (const double *)f, (double *)u, plan->nbr.as<int>(), w,
                                 st);
    return launch_if<float>(ctx, B, r, rb, ntgt, ncomp, nsrc, (const float *)f, (float *)u, plan->nbr.as<int>(), w, st);
}
