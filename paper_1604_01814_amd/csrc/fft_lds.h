// fft_lds.h -- mixed-radix (2, 3, 4, 5, 8) Stockham FFT of many pencils held in
// LDS by one 256-thread workgroup.
//
// A workgroup keeps NP pencils of length P in LDS; element j of pencil p sits
// at s[p * sp + j * sj].  Each stage of radix R reads the R inputs of every
// butterfly into registers, twiddles them, applies the R-point DFT, and after
// a barrier writes them to their auto-sorted positions (Stockham), so a
// single LDS buffer suffices and no bit reversal is needed.  Twiddles come
// from a per-length table tw[m] = exp(-2 pi i m / P) (conjugated for the
// inverse).  Threads walk pencils fastest when pencils are adjacent in LDS
// (column passes) and elements fastest otherwise (row passes), which keeps
// the LDS accesses of a wavefront on distinct banks.
#pragma once

#include <hip/hip_runtime.h>

namespace lgfib {

template <typename Real> struct CplxOf;
template <> struct CplxOf<float> { using T = float2; };
template <> struct CplxOf<double> { using T = double2; };

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i (forward) or +i (inverse)
template <typename C, bool INV> __device__ __forceinline__ C mul_mi(C a) {
    return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

constexpr int kFftThreads = 256;
constexpr int kMaxStages = 12;

struct FftPlan1D {
    int P;
    int nst;
    int rad[kMaxStages];
};

// Radix DFTs (forward uses exp(-2 pi i k n / R)).
template <typename C, int R, bool INV> struct Dft;

template <typename C, bool INV> struct Dft<C, 2, INV> {
    __device__ __forceinline__ static void run(C *v) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename C, bool INV> struct Dft<C, 4, INV> {
    __device__ __forceinline__ static void run(C *v) {
        C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        C t2 = cadd(v[1], v[3]), t3 = mul_mi<C, INV>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <typename C, bool INV> struct Dft<C, 3, INV> {
    __device__ __forceinline__ static void run(C *v) {
        using R = decltype(v[0].x);
        const R h = (R)0.8660254037844386467637231707529362;   // sin(2 pi / 3)
        C s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        C m = C{v[0].x - (R)0.5 * s.x, v[0].y - (R)0.5 * s.y};
        // forward: -i h d ; inverse: +i h d
        C r = mul_mi<C, INV>(C{h * d.x, h * d.y});
        v[0] = cadd(v[0], s);
        v[1] = cadd(m, r);
        v[2] = csub(m, r);
    }
};

template <typename C, bool INV> struct Dft<C, 5, INV> {
    __device__ __forceinline__ static void run(C *v) {
        using R = decltype(v[0].x);
        const R c1 = (R)0.3090169943749474241022934171828191;    // cos(2 pi / 5)
        const R c2 = (R)-0.8090169943749474241022934171828191;   // cos(4 pi / 5)
        const R s1 = (R)0.9510565162951535721164393333793821;    // sin(2 pi / 5)
        const R s2 = (R)0.5877852522924731291687059546390728;    // sin(4 pi / 5)
        C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        C x0 = v[0];
        C p1 = C{x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
        C p2 = C{x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
        C q1 = mul_mi<C, INV>(C{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
        C q2 = mul_mi<C, INV>(C{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
        v[0] = C{x0.x + a1.x + a2.x, x0.y + a1.y + a2.y};
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    }
};

template <typename C, bool INV> struct Dft<C, 8, INV> {
    __device__ __forceinline__ static void run(C *v) {
        using R = decltype(v[0].x);
        const R r = (R)0.7071067811865475244008443621048490;
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        Dft<C, 4, INV>::run(e);
        Dft<C, 4, INV>::run(o);
        // o[k] *= W8^k, W8 = exp(-+ 2 pi i / 8)
        C o1 = o[1], o3 = o[3];
        if (!INV) {
            o[1] = C{r * (o1.x + o1.y), r * (o1.y - o1.x)};
            o[3] = C{r * (o3.y - o3.x), -r * (o3.x + o3.y)};
        } else {
            o[1] = C{r * (o1.x - o1.y), r * (o1.y + o1.x)};
            o[3] = C{-r * (o3.x + o3.y), r * (o3.x - o3.y)};
        }
        o[2] = mul_mi<C, INV>(o[2]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
};

// One Stockham stage of radix R over NP pencils.  MAXV bounds the complex
// values a thread holds (ceil(P * NP / 256)).
template <typename C, int R, int MAXV, bool INV, bool PFAST>
__device__ __forceinline__ void fft_stage(C *s, int P, int NP, int sp, int sj, int Ns, const C *__restrict__ tw) {
    constexpr int MAXB = (MAXV + R - 1) / R;
    const int nb = P / R;
    const int total = nb * NP;
    const int tstep = P / (Ns * R);
    C v[MAXB][R];
    int obase[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int idx = threadIdx.x + i * kFftThreads;
        if (idx < total) {
            int p, j;
            if (PFAST) {
                p = idx % NP;
                j = idx / NP;
            } else {
                j = idx % nb;
                p = idx / nb;
            }
            const C *src = s + p * sp;
            const int k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src[(j + r * nb) * sj];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tw[k * r * tstep];
                    if (INV) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            Dft<C, R, INV>::run(v[i]);
            obase[i] = p * sp + ((j - k) * R + k) * sj;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int idx = threadIdx.x + i * kFftThreads;
        if (idx < total) {
#pragma unroll
            for (int r = 0; r < R; ++r) s[obase[i] + r * Ns * sj] = v[i][r];
        }
    }
    __syncthreads();
}

// Full transform of NP pencils in LDS; the caller synchronises before.
template <typename C, int MAXV, bool INV, bool PFAST>
__device__ void fft_lds(C *s, const FftPlan1D &pl, int NP, int sp, int sj, const C *__restrict__ tw) {
    int Ns = 1;
    for (int st = 0; st < pl.nst; ++st) {
        const int R = pl.rad[st];
        switch (R) {
        case 2: fft_stage<C, 2, MAXV, INV, PFAST>(s, pl.P, NP, sp, sj, Ns, tw); break;
        case 3: fft_stage<C, 3, MAXV, INV, PFAST>(s, pl.P, NP, sp, sj, Ns, tw); break;
        case 4: fft_stage<C, 4, MAXV, INV, PFAST>(s, pl.P, NP, sp, sj, Ns, tw); break;
        case 5: fft_stage<C, 5, MAXV, INV, PFAST>(s, pl.P, NP, sp, sj, Ns, tw); break;
        default: fft_stage<C, 8, MAXV, INV, PFAST>(s, pl.P, NP, sp, sj, Ns, tw); break;
        }
        Ns *= R;
    }
}

}  // namespace lgfib
