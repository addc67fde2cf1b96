// if_apply.hip -- the integrating factor u = E(a) f on a block set.
//
// E(a) = exp(aL) has the LGF prod_q e^{-2a} I_{n_q}(2a) (App. A,
// Eq. lgf_intfac): a separable, even, rapidly decaying stencil, truncated
// where the 1D weight falls below 1e-14 (half-width r).  One workgroup owns
// one target block and one component; thread (x, y) owns the output column
// (x, y, 0..B-1).  The (B+2r)^2 halo of each input z-plane is staged in LDS
// (neighbour source blocks looked up once per call in a host-built table),
// filtered along x, then along y, and the filtered plane is accumulated into
// the B z-outputs of every column with the z weights.  HBM sees each source
// value once per neighbouring target block (mostly L2 hits) and each output
// once.
#include <cmath>

#include "internal.h"

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

template <typename Real>
static int launch_if(lgfib_ctx *ctx, int B, int r, int rb, int ntgt, int ncomp, int nsrc, const Real *f, Real *u, const int *nbr,
                     const double *w, hipStream_t st) {
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

// 1D weights e^{-2a} I_j(2a), j = 0..r, cached per a on the device.
int get_if_weights(lgfib_ctx *ctx, double a, int *radius, const double **dev) {
    auto it = ctx->if_weights.find(a);
    if (it != ctx->if_weights.end()) {
        *radius = it->second.first;
        *dev = it->second.second->as<double>();
        return LGFIB_OK;
    }
    int r = 0;
    std::vector<double> w(4097);
    int rc = lgf_if_weights(ctx, a, 1e-14, w.data(), (int)w.size(), &r);
    if (rc) return rc;
    auto buf = std::make_unique<DevBuf>();
    if ((rc = buf->reserve(sizeof(double) * (r + 1)))) return rc;
    LGF_HIP(hipMemcpy(buf->p, w.data(), sizeof(double) * (r + 1), hipMemcpyHostToDevice));
    *radius = r;
    *dev = buf->as<double>();
    ctx->if_weights[a] = std::make_pair(r, std::move(buf));
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
    int rc = validate_blocks(src_blocks, nsrc, "source blocks");
    if (rc) return rc;
    if ((rc = validate_blocks(tgt_blocks, ntgt, "target blocks"))) return rc;
    if (ntgt == 0) return LGFIB_OK;
    if (nsrc == 0) {
        LGF_HIP(hipMemsetAsync(u, 0, ubytes, st));
        return LGFIB_OK;
    }
    int r = 0;
    const double *w = nullptr;
    if ((rc = get_if_weights(ctx, a, &r, &w))) return rc;
    IfPlan *plan = nullptr;
    if ((rc = get_if_plan(ctx, B, r, src_blocks, nsrc, tgt_blocks, ntgt, &plan))) return rc;
    const int rb = plan->rb;
    if (prec == LGF_F64)
        return launch_if<double>(ctx, B, r, rb, ntgt, ncomp, nsrc, (const double *)f, (double *)u, plan->nbr.as<int>(), w,
                                 st);
    return launch_if<float>(ctx, B, r, rb, ntgt, ncomp, nsrc, (const float *)f, (float *)u, plan->nbr.as<int>(), w, st);
}
