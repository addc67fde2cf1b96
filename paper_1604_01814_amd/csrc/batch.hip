// batch.hip -- many independent FP32 LGF Poisson applies (u_i = dx^2 G * f_i
// on block set S_i, targets = sources; Sec. 2.2, Eq. dpoisson_conv) in one
// HIP-graph launch.
//
// Each instance is a box-FFT convolution (conv.hip) or, for small sets, the
// block-pair form on 8^3 blocks (pair.hip).  At creation an autotuner times,
// per instance, the block size the box is built from (the caller's B, B/2 --
// each block split exactly into 8 -- or 2B, covering blocks zero-padded), the
// tiles per workgroup of the x and y passes, and the block-pair form, and
// keeps the fastest.  Instances are then bin-packed by their measured time
// onto a few branch streams, each with its own FFT workspace, and the whole
// batch (re-blocking gathers, five passes, scatters) is captured once into a
// graph whose branches run concurrently.  Running the batch is one
// hipGraphLaunch.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "conv_common.h"

namespace lgfib {

struct RMap {   // block box map on the device
    int lo0, lo1, lo2, nb0, nb1, nb2, B;
    const int *map;   // [nb2][nb1][nb0] -> slot or -1
    __device__ int slot_of_cell(int x, int y, int z) const {
        const int bx = (x >= 0 ? x / B : -((-x + B - 1) / B)) - lo0;
        const int by = (y >= 0 ? y / B : -((-y + B - 1) / B)) - lo1;
        const int bz = (z >= 0 ? z / B : -((-z + B - 1) / B)) - lo2;
        if (bx < 0 || by < 0 || bz < 0 || bx >= nb0 || by >= nb1 || bz >= nb2) return -1;
        return map[((size_t)bz * nb1 + by) * nb0 + bx];
    }
};

// dst[d][cell] = src value of the same lattice cell (0 where no source block):
// re-lays a field between two block sizes
__device__ __forceinline__ void reblock_cell(const float *__restrict__ src, const RMap &sm, float *__restrict__ dst,
                                             const int *__restrict__ dblocks, int Bd, int ndst, size_t t) {
    const size_t B3 = (size_t)Bd * Bd * Bd;
    if (t >= (size_t)ndst * B3) return;
    const int d = (int)(t / B3), cell = (int)(t % B3);
    const int x = dblocks[3 * d] * Bd + cell % Bd, y = dblocks[3 * d + 1] * Bd + (cell / Bd) % Bd,
              z = dblocks[3 * d + 2] * Bd + cell / (Bd * Bd);
    const int s = sm.slot_of_cell(x, y, z);
    float v = 0.f;
    if (s >= 0) {
        const int Bs = sm.B;
        const int lx = x - (x >= 0 ? x / Bs : -((-x + Bs - 1) / Bs)) * Bs;
        const int ly = y - (y >= 0 ? y / Bs : -((-y + Bs - 1) / Bs)) * Bs;
        const int lz = z - (z >= 0 ? z / Bs : -((-z + Bs - 1) / Bs)) * Bs;
        v = src[(size_t)s * Bs * Bs * Bs + ((size_t)lz * Bs + ly) * Bs + lx];
    }
    dst[t] = v;
}

__global__ void k_reblock(const float *__restrict__ src, RMap sm, float *__restrict__ dst,
                          const int *__restrict__ dblocks, int Bd, int ndst) {
    reblock_cell(src, sm, dst, dblocks, Bd, ndst, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// many re-blockings in one launch: workgroup w belongs to job owner[w]
struct ReblockJob {
    const float *src;
    RMap sm;
    float *dst;
    const int *dblocks;
    int Bd, ndst, w0;   // w0: the job's first workgroup
};
__global__ void k_reblock_batched(const ReblockJob *__restrict__ jobs, const int *__restrict__ owner) {
    const ReblockJob &J = jobs[__builtin_amdgcn_readfirstlane(owner[blockIdx.x])];
    reblock_cell(J.src, J.sm, J.dst, J.dblocks, J.Bd, J.ndst, (size_t)(blockIdx.x - J.w0) * blockDim.x + threadIdx.x);
}

struct HostMap {
    int lo[3] = {0, 0, 0}, nb[3] = {1, 1, 1}, B = 0;
    DevBuf map;
    DevBuf blocks;
    int n = 0;
    RMap dev() const {
        return RMap{lo[0], lo[1], lo[2], nb[0], nb[1], nb[2], B, map.as<int>()};
    }
};

static int build_map(HostMap &m, const std::vector<int32_t> &bl, int B) {
    m.B = B;
    m.n = (int)(bl.size() / 3);
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    for (int i = 0; i < m.n; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], bl[3 * i + a]);
            hi[a] = std::max(hi[a], bl[3 * i + a]);
        }
    size_t sz = 1;
    for (int a = 0; a < 3; ++a) {
        m.lo[a] = lo[a];
        m.nb[a] = hi[a] - lo[a] + 1;
        sz *= (size_t)m.nb[a];
    }
    if (sz > (size_t)1 << 26) return fail(LGFIB_ERANGE, "batch: instance spans too large a box");
    std::vector<int32_t> map(sz, -1);
    for (int i = 0; i < m.n; ++i)
        map[((size_t)(bl[3 * i + 2] - lo[2]) * m.nb[1] + (bl[3 * i + 1] - lo[1])) * m.nb[0] + (bl[3 * i] - lo[0])] = i;
    int rc;
    if ((rc = m.map.reserve(map.size() * 4)) || (rc = m.blocks.reserve(bl.size() * 4))) return rc;
    LGF_HIP(hipMemcpy(m.map.p, map.data(), map.size() * 4, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(m.blocks.p, bl.data(), bl.size() * 4, hipMemcpyHostToDevice));
    return LGFIB_OK;
}

// blocks of size Bd covering the cells of blocks of size Bs (sorted z, y, x)
static std::vector<int32_t> reblock_list(const int32_t *bl, int n, int Bs, int Bd) {
    std::vector<std::array<int32_t, 3>> v;
    auto fd = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    if (Bd <= Bs) {
        const int k = Bs / Bd;
        for (int i = 0; i < n; ++i)
            for (int dz = 0; dz < k; ++dz)
                for (int dy = 0; dy < k; ++dy)
                    for (int dx = 0; dx < k; ++dx)
                        v.push_back({bl[3 * i] * k + dx, bl[3 * i + 1] * k + dy, bl[3 * i + 2] * k + dz});
    } else {
        for (int i = 0; i < n; ++i)
            v.push_back({fd(bl[3 * i] * Bs, Bd), fd(bl[3 * i + 1] * Bs, Bd), fd(bl[3 * i + 2] * Bs, Bd)});
    }
    std::sort(v.begin(), v.end(), [](const std::array<int32_t, 3> &a, const std::array<int32_t, 3> &b) {
        if (a[2] != b[2]) return a[2] < b[2];
        if (a[1] != b[1]) return a[1] < b[1];
        return a[0] < b[0];
    });
    v.erase(std::unique(v.begin(), v.end()), v.end());
    std::vector<int32_t> out;
    for (auto &b : v) out.insert(out.end(), b.begin(), b.end());
    return out;
}

struct Candidate {
    int B = 0, tpx = 0, tpy = 0;
    int path = 0;   // 0: box FFT, 1: block pairs (8^3 blocks, FP32 DFTs)
};

// the block-pair form is tried for sets up to this many 8^3 blocks
constexpr int kPairMaxBlocks = 400;

static unsigned nblk256(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace lgfib

using namespace lgfib;

struct BatchInst {
    int nblk = 0;
    std::vector<int32_t> blocks;
    const float *f = nullptr;
    float *u = nullptr;
    // chosen execution
    Candidate pick;
    double ms = 0.0;
    std::vector<int32_t> eblocks;
    std::shared_ptr<BoxPlan> plan;     // held: pins the cached plan while the batch lives
    std::shared_ptr<Spectrum> spec;
    PairExec pair;
    HostMap refmap, exmap;
    DevBuf fe, ue;   // re-blocked fields (when pick.B differs from the caller's)
    size_t w1 = 0, w2 = 0;
    int branch = 0;
    bool fast = false;   // runs in the batched passes
};

// One persistent launch of the batched passes: every instance of one FFT
// length for one pass.
struct PassGroup {
    int pass = 0, P = 0;
    std::vector<FastJob> jobs;
    std::vector<int> start;   // work-item offsets, start[njobs] = total
    size_t sm = 0;            // LDS bytes (largest over the instances)
    DevBuf djobs, dstart, downer;   // jobs, item offsets, owner instance of every item
    int queue = 0;            // index of its counter
};

struct lgf_batch {
    lgfib_ctx *ctx = nullptr;
    lgf_table_t tbl = -1;
    int B = 0;
    double dx = 1.0;
    std::vector<std::unique_ptr<BatchInst>> inst;
    // instances whose box convolution runs in the batched passes
    std::vector<int> fast;
    std::vector<std::unique_ptr<PassGroup>> groups;   // ordered by pass
    DevBuf arena;                    // their FFT workspaces
    DevBuf queues;                   // one work counter per group
    // re-blocking of the batched instances whose block size was changed:
    // gathers before the passes [0] and scatters after them [1]
    DevBuf rjobs[2], rowner[2];
    int rgroups[2] = {0, 0};
    // in the captured graph the groups of one pass (one per FFT length) run
    // side by side on these streams, forked from and joined to the capture
    // stream around each pass: pev[pass] forks, pev[kNumPasses + pass *
    // pstreams.size() + k] joins stream k
    std::vector<hipStream_t> pstreams;
    std::vector<hipEvent_t> pev;

    int nbranch = 1;
    std::vector<std::unique_ptr<DevBuf>> w1, w2;   // per branch
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace lgfib {

// set up instance execution for candidate c (plans, spectrum, maps, buffers)
static int prepare(lgf_batch *b, BatchInst &I, const Candidate &c, hipStream_t st) {
    lgfib_ctx *ctx = b->ctx;
    I.pick = c;
    I.plan.reset();   // release the previous candidate's cached objects
    I.spec.reset();
    I.pair.ghat.reset();
    I.eblocks = c.B == b->B ? I.blocks : reblock_list(I.blocks.data(), I.nblk, b->B, c.B);
    const int ne = (int)(I.eblocks.size() / 3);
    int rc;
    if (c.path == 1) {
        if ((rc = pair_prepare(ctx, b->tbl, I.eblocks.data(), ne, I.eblocks.data(), ne, I.pair, st))) return rc;
        I.w1 = I.w2 = pair_work_bytes(ne, 1);
    } else {
        if ((rc = get_box_plan(ctx, c.B, I.eblocks.data(), ne, I.eblocks.data(), ne, I.plan))) return rc;
        const Table &tb = *ctx->tables[b->tbl];
        for (int a = 0; a < 3; ++a) {
            int lo = 1 << 30, hi = -(1 << 30);
            for (int i = 0; i < ne; ++i) {
                lo = std::min(lo, I.eblocks[3 * i + a]);
                hi = std::max(hi, I.eblocks[3 * i + a]);
            }
            if (tb.ext[a] < (hi - lo + 1) * c.B - 1) return fail(LGFIB_ERANGE, "batch: table extent too small");
        }
        if ((rc = get_spectrum(ctx, b->tbl, *I.plan, LGF_F32, st, I.spec))) return rc;
        box_work_bytes(*I.plan, 1, LGF_F32, &I.w1, &I.w2);
    }
    if (c.B != b->B) {
        const size_t ncell = (size_t)ne * c.B * c.B * c.B;
        if ((rc = build_map(I.refmap, I.blocks, b->B)) || (rc = build_map(I.exmap, I.eblocks, c.B))) return rc;
        if ((rc = I.fe.reserve(ncell * 4)) || (rc = I.ue.reserve(ncell * 4))) return rc;
    }
    return LGFIB_OK;
}

// enqueue one instance on st with workspace (w1, w2)
static int enqueue(lgf_batch *b, BatchInst &I, hipStream_t st, void *w1, size_t w1b, void *w2, size_t w2b) {
    ConvOverrides &ov = conv_overrides();
    ov.tpw_x = I.pick.tpx;
    ov.tpw_y = I.pick.tpy;
    ov.w1 = w1;
    ov.w2 = w2;
    ov.w1_bytes = w1b;
    ov.w2_bytes = w2b;
    int rc;
    const int Be = I.pick.B;
    auto run = [&](const float *fi, float *uo) {
        if (I.pick.path == 1) return pair_enqueue(b->ctx, I.pair, 1, LGF_DFT_FFT32, b->dx, fi, uo, w1, w2, st);
        return box_conv_f32(b->ctx, *I.plan, *I.spec, 1, b->dx, fi, uo, 0, st);
    };
    if (Be == b->B) {
        rc = run(I.f, I.u);
    } else {
        const int ne = I.exmap.n;
        const size_t ncell = (size_t)ne * Be * Be * Be;
        hipLaunchKernelGGL(k_reblock, dim3(nblk256(ncell)), dim3(256), 0, st, I.f, I.refmap.dev(), I.fe.as<float>(),
                           I.exmap.blocks.as<int>(), Be, ne);
        rc = run(I.fe.as<float>(), I.ue.as<float>());
        if (!rc) {
            const size_t nref = (size_t)I.nblk * b->B * b->B * b->B;
            hipLaunchKernelGGL(k_reblock, dim3(nblk256(nref)), dim3(256), 0, st, (const float *)I.ue.as<float>(),
                               I.exmap.dev(), I.u, I.refmap.blocks.as<int>(), b->B, I.nblk);
        }
    }
    ov = ConvOverrides{};
    LGF_HIP(hipGetLastError());
    return rc;
}

__global__ void k_zero_ints(int *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// the batched instances on st: counters cleared by a fill kernel (no memset
// node in a captured graph), gathers, the five passes in pass order, scatters.
// With fork set (graph capture) the groups of one pass run on the pass
// streams side by side; otherwise group after group on st.
static int run_fast(lgf_batch *b, hipStream_t st, bool fork) {
    if (b->fast.empty()) return LGFIB_OK;
    const int nq = (int)b->groups.size();
    hipLaunchKernelGGL(k_zero_ints, dim3((nq + 255) / 256), dim3(256), 0, st, b->queues.as<int>(), nq);
    if (b->rgroups[0])
        hipLaunchKernelGGL(k_reblock_batched, dim3(b->rgroups[0]), dim3(256), 0, st, b->rjobs[0].as<ReblockJob>(),
                           b->rowner[0].as<int>());
    int rc;
    const int ns = (int)b->pstreams.size();
    for (int g0 = 0; g0 < nq;) {
        const int pass = b->groups[g0]->pass;
        int g1 = g0;
        while (g1 < nq && b->groups[g1]->pass == pass) ++g1;   // groups are ordered by pass
        const bool side = fork && ns > 1 && g1 - g0 > 1;
        if (side) {
            LGF_HIP(hipEventRecord(b->pev[pass], st));
            for (int k = 0; k < std::min(ns, g1 - g0); ++k) LGF_HIP(hipStreamWaitEvent(b->pstreams[k], b->pev[pass], 0));
        }
        for (int gi = g0; gi < g1; ++gi) {
            const PassGroup &G = *b->groups[gi];
            hipStream_t s = side ? b->pstreams[(gi - g0) % ns] : st;
            ProfScope ps(b->ctx, "k_batch_pass", s);
            if ((rc = launch_fast_batched(G.pass, G.P, G.djobs.as<FastJob>(), G.dstart.as<int>(), G.downer.as<int>(),
                                          (int)G.jobs.size(), G.start.back(), b->queues.as<int>() + G.queue, G.sm,
                                          b->ctx->num_cu, s)))
                return rc;
        }
        if (side)
            for (int k = 0; k < std::min(ns, g1 - g0); ++k) {
                hipEvent_t e = b->pev[kNumPasses + pass * ns + k];
                LGF_HIP(hipEventRecord(e, b->pstreams[k]));
                LGF_HIP(hipStreamWaitEvent(st, e, 0));
            }
        g0 = g1;
    }
    if (b->rgroups[1])
        hipLaunchKernelGGL(k_reblock_batched, dim3(b->rgroups[1]), dim3(256), 0, st, b->rjobs[1].as<ReblockJob>(),
                           b->rowner[1].as<int>());
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// Set up the batched passes for the instances whose picked box plan has
// specialised FFT lengths on every axis: workspaces, jobs, groups.
static int build_fast(lgf_batch *b) {
    lgfib_ctx *ctx = b->ctx;
    std::vector<BoxGeo> geo(b->inst.size());
    size_t need = 0;
    for (size_t i = 0; i < b->inst.size(); ++i) {
        BatchInst &I = *b->inst[i];
        I.fast = false;
        if (I.pick.path != 0) continue;
        make_box_geo(*I.plan, 1, geo[i]);
        const BoxGeo &g = geo[i];
        if (!(fast_x_ok(g) && fast_size(g.P1) && fast_size(g.P2))) continue;
        I.fast = true;
        b->fast.push_back((int)i);
        need += (I.w1 + 255) / 256 * 256 + (I.w2 + 255) / 256 * 256;
    }
    if (b->fast.empty()) return LGFIB_OK;
    int rc;
    if ((rc = b->arena.reserve(need))) return rc;
    std::map<std::pair<int, int>, std::unique_ptr<PassGroup>> by;   // (pass, P)
    size_t off = 0;
    for (int i : b->fast) {
        BatchInst &I = *b->inst[i];
        const BoxGeo &g = geo[i];
        float2 *X1 = (float2 *)((char *)b->arena.p + off);
        off += (I.w1 + 255) / 256 * 256;
        float2 *X2 = (float2 *)((char *)b->arena.p + off);
        off += (I.w2 + 255) / 256 * 256;
        const void *tw[3];
        for (int a = 0; a < 3; ++a)
            if ((rc = get_twiddles(ctx, a == 0 ? g.P0 : a == 1 ? g.P1 : g.P2, LGF_F32, &tw[a]))) return rc;
        const float2 *twc[3] = {(const float2 *)tw[0], (const float2 *)tw[1], (const float2 *)tw[2]};
        const bool rb = I.pick.B != b->B;
        const float *fin = rb ? I.fe.as<float>() : I.f;
        float *uout = rb ? I.ue.as<float>() : I.u;
        const float scale = (float)(b->dx * b->dx / ((double)g.P0 * g.P1 * g.P2));
        FastJob jobs[kNumPasses];
        int items[kNumPasses], P[kNumPasses];
        size_t sm[kNumPasses];
        if ((rc = fast_jobs(g, fin, uout, X1, X2, I.spec->ghat.as<float>(), scale, twc, I.pick.tpx, I.pick.tpy, jobs,
                            items, sm, P)))
            return rc;
        for (int pass = 0; pass < kNumPasses; ++pass) {
            auto &Gp = by[std::make_pair(pass, P[pass])];
            if (!Gp) Gp = std::make_unique<PassGroup>();
            PassGroup &G = *Gp;
            G.pass = pass;
            G.P = P[pass];
            if (G.start.empty()) G.start.push_back(0);
            G.jobs.push_back(jobs[pass]);
            G.start.push_back(G.start.back() + items[pass]);
            G.sm = std::max(G.sm, sm[pass]);
        }
    }
    // re-blocking jobs, one workgroup per 256 cells
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<ReblockJob> rj;
        std::vector<int> own;
        for (int i : b->fast) {
            BatchInst &I = *b->inst[i];
            if (I.pick.B == b->B) continue;
            ReblockJob J;
            if (dir == 0) {
                J = ReblockJob{I.f, I.refmap.dev(), I.fe.as<float>(), I.exmap.blocks.as<int>(), I.pick.B, I.exmap.n, 0};
            } else {
                J = ReblockJob{I.ue.as<float>(), I.exmap.dev(), I.u, I.refmap.blocks.as<int>(), b->B, I.nblk, 0};
            }
            const size_t ncell = (size_t)J.ndst * J.Bd * J.Bd * J.Bd;
            J.w0 = (int)own.size();
            own.insert(own.end(), nblk256(ncell), (int)rj.size());
            rj.push_back(J);
        }
        b->rgroups[dir] = (int)own.size();
        if (own.empty()) continue;
        if ((rc = b->rjobs[dir].reserve(sizeof(ReblockJob) * rj.size())) ||
            (rc = b->rowner[dir].reserve(sizeof(int) * own.size())))
            return rc;
        LGF_HIP(hipMemcpy(b->rjobs[dir].p, rj.data(), sizeof(ReblockJob) * rj.size(), hipMemcpyHostToDevice));
        LGF_HIP(hipMemcpy(b->rowner[dir].p, own.data(), sizeof(int) * own.size(), hipMemcpyHostToDevice));
    }
    for (auto &kv : by) {   // std::map order: by pass, then length
        b->groups.push_back(std::move(kv.second));
        PassGroup &G = *b->groups.back();
        G.queue = (int)b->groups.size() - 1;
        std::vector<int> owner(std::max(G.start.back(), 1), 0);
        for (size_t k = 0; k + 1 < G.start.size(); ++k)
            for (int it = G.start[k]; it < G.start[k + 1]; ++it) owner[it] = (int)k;
        if ((rc = G.djobs.reserve(sizeof(FastJob) * G.jobs.size())) ||
            (rc = G.dstart.reserve(sizeof(int) * G.start.size())) || (rc = G.downer.reserve(sizeof(int) * owner.size())))
            return rc;
        LGF_HIP(hipMemcpy(G.djobs.p, G.jobs.data(), sizeof(FastJob) * G.jobs.size(), hipMemcpyHostToDevice));
        LGF_HIP(hipMemcpy(G.dstart.p, G.start.data(), sizeof(int) * G.start.size(), hipMemcpyHostToDevice));
        LGF_HIP(hipMemcpy(G.downer.p, owner.data(), sizeof(int) * owner.size(), hipMemcpyHostToDevice));
    }
    if ((rc = b->queues.reserve(sizeof(int) * std::max<size_t>(b->groups.size(), 1)))) return rc;
    return LGFIB_OK;
}

static std::vector<Candidate> candidates(int B, int nblk, bool tune) {
    std::vector<Candidate> v;
    if (!tune) {
        v.push_back({B, 0, 0, 0});
        return v;
    }
    for (int Be : {B / 2, B, 2 * B}) {
        if (Be != 8 && Be != 16 && Be != 32) continue;
        for (int tx : {1, 2})
            for (int ty : {1, 2, 4}) v.push_back({Be, tx, ty, 0});
    }
    const long n8 = (long)nblk * (B / 8) * (B / 8) * (B / 8);
    if ((B == 8 || B == 16) && n8 <= kPairMaxBlocks) v.push_back({8, 0, 0, 1});
    return v;
}

}  // namespace lgfib

extern "C" int lgf_batch_create(lgfib_ctx *ctx, lgf_table_t tbl, int B, int ninst, const lgf_instance_t *insts,
                                double dx, int flags, int nbranch, lgf_batch_t **out) {
    if (!out) return fail(LGFIB_EINVAL, "lgf_batch_create: null output");
    *out = nullptr;
    if (!ctx || !insts || ninst < 1) return fail(LGFIB_EINVAL, "lgf_batch_create: bad argument");
    if (flags & ~(LGF_BATCH_AUTOTUNE | LGF_BATCH_PASSES)) return fail(LGFIB_EINVAL, "lgf_batch_create: unknown flags");
    const int autotune = flags & LGF_BATCH_AUTOTUNE;
    if (tbl < 0 || (size_t)tbl >= ctx->tables.size()) return fail(LGFIB_ENOTBUILT, "lgf_batch_create: unknown table");
    if (B != 8 && B != 16 && B != 32) return fail(LGFIB_EINVAL, "lgf_batch_create: B must be 8, 16 or 32");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LGFIB_EINVAL, "lgf_batch_create: dx must be positive");
    if (nbranch < 1 || nbranch > 16) return fail(LGFIB_EINVAL, "lgf_batch_create: nbranch must lie in [1, 16]");
    LGF_HIP(hipSetDevice(ctx->device));
    auto b = std::make_unique<lgf_batch>();
    b->ctx = ctx;
    b->tbl = tbl;
    b->B = B;
    b->dx = dx;
    for (int i = 0; i < ninst; ++i) b->inst.push_back(std::make_unique<BatchInst>());
    int rc;
    for (int i = 0; i < ninst; ++i) {
        const lgf_instance_t &s = insts[i];
        if (s.nblk < 1 || !s.blocks || !s.f || !s.u) return fail(LGFIB_EINVAL, "lgf_batch_create: bad instance");
        if ((rc = validate_blocks(s.blocks, s.nblk, "instance blocks"))) return rc;
        BatchInst &I = *b->inst[i];
        I.nblk = s.nblk;
        I.blocks.assign(s.blocks, s.blocks + 3 * (size_t)s.nblk);
        I.f = s.f;
        I.u = s.u;
    }
    hipStream_t st = nullptr;
    hipEvent_t e0, e1;
    LGF_HIP(hipEventCreate(&e0));
    LGF_HIP(hipEventCreate(&e1));
    // autotune (or the default) per instance, timed eagerly with the
    // context's workspaces
    for (auto &Ip : b->inst) {
        BatchInst &I = *Ip;
        double best = 1e30;
        Candidate bestc;
        for (const Candidate &c : candidates(B, I.nblk, autotune != 0)) {
            if ((rc = prepare(b.get(), I, c, st))) {
                if (rc == LGFIB_ERANGE) continue;   // this block size needs a larger table
                return rc;
            }
            if ((rc = ctx->work1.reserve(I.w1)) || (rc = ctx->work2.reserve(I.w2))) return rc;
            double ms = 0.0;
            if (autotune) {
                const int reps = 3;
                if ((rc = enqueue(b.get(), I, st, ctx->work1.p, ctx->work1.bytes, ctx->work2.p, ctx->work2.bytes)))
                    return rc;
                LGF_HIP(hipEventRecord(e0, st));
                for (int r = 0; r < reps; ++r)
                    if ((rc = enqueue(b.get(), I, st, ctx->work1.p, ctx->work1.bytes, ctx->work2.p, ctx->work2.bytes)))
                        return rc;
                LGF_HIP(hipEventRecord(e1, st));
                LGF_HIP(hipEventSynchronize(e1));
                float t = 0.f;
                LGF_HIP(hipEventElapsedTime(&t, e0, e1));
                ms = t / reps;
            }
            if (ms < best) {
                best = ms;
                bestc = c;
            }
        }
        if (best > 1e29) return fail(LGFIB_ERANGE, "lgf_batch_create: no block size fits the table");
        if ((rc = prepare(b.get(), I, bestc, st))) return rc;
        I.ms = best;
        // one eager run of the choice creates everything the capture will
        // reference (twiddle tables, spectra) outside the capture
        if ((rc = ctx->work1.reserve(I.w1)) || (rc = ctx->work2.reserve(I.w2))) return rc;
        if ((rc = enqueue(b.get(), I, st, ctx->work1.p, ctx->work1.bytes, ctx->work2.p, ctx->work2.bytes))) return rc;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if ((flags & LGF_BATCH_PASSES) && (rc = build_fast(b.get()))) return rc;
    // the other instances (block-pair form, or box lengths without
    // specialised passes) are bin-packed by measured time onto branch streams
    // beside the batched passes, each branch with its own FFT workspace
    std::vector<int> order;
    for (int i = 0; i < ninst; ++i)
        if (!b->inst[i]->fast) order.push_back(i);
    b->nbranch = std::max(1, std::min(nbranch, (int)order.size()));
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->inst[x]->ms > b->inst[y]->ms; });
    std::vector<double> load(b->nbranch, 0.0);
    std::vector<size_t> need1(b->nbranch, 0), need2(b->nbranch, 0);
    for (int i : order) {
        const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        auto &I = *b->inst[i];
        I.branch = br;
        load[br] += std::max(I.ms, 1e-3);
        need1[br] = std::max(need1[br], I.w1);
        need2[br] = std::max(need2[br], I.w2);
    }
    for (int br = 0; br < b->nbranch; ++br) {
        b->w1.push_back(std::make_unique<DevBuf>());
        b->w2.push_back(std::make_unique<DevBuf>());
        if ((rc = b->w1[br]->reserve(std::max<size_t>(need1[br], 256))) ||
            (rc = b->w2[br]->reserve(std::max<size_t>(need2[br], 256))))
            return rc;
    }
    // capture: the batched passes on the capture stream, the other instances
    // forked onto the branch streams and joined at the end
    LGF_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    b->streams.resize(b->nbranch);
    b->joins.resize(b->nbranch);
    for (int br = 0; br < b->nbranch; ++br) {
        LGF_HIP(hipStreamCreateWithFlags(&b->streams[br], hipStreamNonBlocking));
        LGF_HIP(hipEventCreateWithFlags(&b->joins[br], hipEventDisableTiming));
    }
    LGF_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    {   // streams and events for the side-by-side groups of each batched pass
        int most = 0;
        for (size_t g0 = 0; g0 < b->groups.size();) {
            size_t g1 = g0;
            while (g1 < b->groups.size() && b->groups[g1]->pass == b->groups[g0]->pass) ++g1;
            most = std::max(most, (int)(g1 - g0));
            g0 = g1;
        }
        const int ns = std::min(most, 8);
        if (ns > 1) {
            b->pstreams.resize(ns);
            b->pev.resize(kNumPasses * (1 + ns));
            for (auto &s : b->pstreams) LGF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            for (auto &e : b->pev) LGF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
    }
    LGF_HIP(hipDeviceSynchronize());
    if (ctx->profiling) return fail(LGFIB_EINVAL, "lgf_batch_create: disable profiling while a batch is captured");
    hipGraph_t g = nullptr;
    LGF_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int crc = LGFIB_OK;
    const bool others = !order.empty();
    if (others && hipEventRecord(b->fork, b->cap) != hipSuccess) crc = fail(LGFIB_EHIP, "batch capture: fork");
    for (int br = 0; others && !crc && br < b->nbranch; ++br)
        if (hipStreamWaitEvent(b->streams[br], b->fork, 0) != hipSuccess) crc = fail(LGFIB_EHIP, "batch capture: wait");
    for (int i : order) {
        if (crc) break;
        BatchInst &I = *b->inst[i];
        crc = enqueue(b.get(), I, b->streams[I.branch], b->w1[I.branch]->p, b->w1[I.branch]->bytes,
                      b->w2[I.branch]->p, b->w2[I.branch]->bytes);
    }
    if (!crc) crc = run_fast(b.get(), b->cap, true);
    for (int br = 0; others && !crc && br < b->nbranch; ++br) {
        if (hipEventRecord(b->joins[br], b->streams[br]) != hipSuccess ||
            hipStreamWaitEvent(b->cap, b->joins[br], 0) != hipSuccess)
            crc = fail(LGFIB_EHIP, "batch capture: join");
    }
    const hipError_t ee = hipStreamEndCapture(b->cap, &g);
    if (crc) {
        if (g) (void)hipGraphDestroy(g);
        return crc;
    }
    if (ee != hipSuccess || !g) return fail(LGFIB_EHIP, std::string("batch capture: ") + hipGetErrorString(ee));
    const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(LGFIB_EHIP, std::string("batch graph instantiate: ") + hipGetErrorString(ei));
    *out = b.release();
    return LGFIB_OK;
}

extern "C" int lgf_batch_run(lgfib_ctx *ctx, lgf_batch_t *b, int eager, lgfib_stream_t stream) {
    if (!ctx || !b || b->ctx != ctx) return fail(LGFIB_EINVAL, "lgf_batch_run: bad argument");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (!eager) {
        LGF_HIP(hipGraphLaunch(b->exec, st));
        return LGFIB_OK;
    }
    // the same work, one launch after another on one stream, in the
    // context's workspaces
    int rc;
    size_t n1 = 0, n2 = 0;
    for (auto &I : b->inst) {
        if (I->fast) continue;
        n1 = std::max(n1, I->w1);
        n2 = std::max(n2, I->w2);
    }
    if ((rc = ctx->work1.reserve(std::max<size_t>(n1, 256))) || (rc = ctx->work2.reserve(std::max<size_t>(n2, 256))))
        return rc;
    for (auto &I : b->inst)
        if (!I->fast && (rc = enqueue(b, *I, st, ctx->work1.p, ctx->work1.bytes, ctx->work2.p, ctx->work2.bytes)))
            return rc;
    return run_fast(b, st, false);
}

extern "C" int lgf_batch_info(lgf_batch_t *b, int i, int *block, int *tiles_x, int *tiles_y, int *branch,
                              double *tuned_ms, int *path) {
    if (!b || i < 0 || i >= (int)b->inst.size()) return fail(LGFIB_EINVAL, "lgf_batch_info: bad argument");
    const BatchInst &I = *b->inst[i];
    if (block) *block = I.pick.B;
    if (tiles_x) *tiles_x = I.pick.tpx;
    if (tiles_y) *tiles_y = I.pick.tpy;
    if (branch) *branch = I.branch;
    if (tuned_ms) *tuned_ms = I.ms;
    if (path) *path = I.pick.path;
    return LGFIB_OK;
}

extern "C" void lgf_batch_destroy(lgf_batch_t *b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    for (auto s : b->streams) (void)hipStreamDestroy(s);

    for (auto e : b->joins) (void)hipEventDestroy(e);
    for (auto s : b->pstreams) (void)hipStreamDestroy(s);
    for (auto e : b->pev) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

extern "C" int lgf_poisson_apply_batched(lgfib_ctx *ctx, lgf_table_t tbl, int B, int ninst, const lgf_instance_t *inst,
                                         double dx, lgfib_stream_t stream) {
    lgf_batch_t *b = nullptr;
    int rc = lgf_batch_create(ctx, tbl, B, ninst, inst, dx, 0, 4, &b);
    if (rc) return rc;
    rc = lgf_batch_run(ctx, b, 0, stream);
    if (!rc && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = fail(LGFIB_EHIP, "lgf_poisson_apply_batched: stream");
    lgf_batch_destroy(b);
    return rc;
}
