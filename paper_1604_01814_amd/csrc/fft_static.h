// fft_static.h -- compile-time specialised Stockham FFT of NP pencils of length
// P held in LDS by one 256-thread workgroup (the hot-path version of the
// runtime engine in fft_lds.h).
//
// Everything that decides an address is a template constant (P, NP, the LDS
// strides, the radix of every stage and its Ns), so index arithmetic folds to
// shifts and multiplies.  Stages use radices up to 16 (three LDS round trips
// for the 384- and 640-point transforms of the benchmark box).  Twiddles come
// from a P/2-entry table in LDS (the other half by symmetry): a butterfly reads
// the exact powers w^1, w^2, w^4, w^8 and forms the others with at most two
// complex products.
#pragma once

#include <utility>

#include "fft_lds.h"

namespace lgfib {

template <typename C, bool INV> struct Dft<C, 16, INV> {
    __device__ __forceinline__ static void run(C *v) {
        using R = decltype(v[0].x);
        const R c1 = (R)0.9238795325112867561281831893967883;   // cos(pi/8)
        const R s1 = (R)0.3826834323650897717284599840303989;   // sin(pi/8)
        const R h = (R)0.7071067811865475244008443621048490;
        C a[4][4];
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) {
            C t[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
            Dft<C, 4, INV>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) a[n1][k2] = t[k2];
        }
        // a[n1][k2] *= W16^(n1 k2), W16 = exp(-+ 2 pi i / 16)
        const R sg = INV ? (R)1 : (R)-1;   // sign of the imaginary part of W16^1
        auto tw = [&](C x, R c, R s) { return C{x.x * c - x.y * s, x.x * s + x.y * c}; };
        // exponents: (1,1)=1 (1,2)=2 (1,3)=3 (2,1)=2 (2,2)=4 (2,3)=6 (3,1)=3 (3,2)=6 (3,3)=9
        a[1][1] = tw(a[1][1], c1, sg * s1);
        a[1][2] = tw(a[1][2], h, sg * h);
        a[1][3] = tw(a[1][3], s1, sg * c1);
        a[2][1] = tw(a[2][1], h, sg * h);
        a[2][2] = mul_mi<C, INV>(a[2][2]);
        a[2][3] = tw(a[2][3], -h, sg * h);
        a[3][1] = tw(a[3][1], s1, sg * c1);
        a[3][2] = tw(a[3][2], -h, sg * h);
        a[3][3] = tw(a[3][3], -c1, -sg * s1);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            C t[4] = {a[0][k2], a[1][k2], a[2][k2], a[3][k2]};
            Dft<C, 4, INV>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) v[k2 + 4 * k1] = t[k1];
        }
    }
};

// Composite radices in registers, R = R1 x R2 (Cooley-Tukey, n = R2 n1 + n2,
// k = k1 + R1 k2): R1-point DFTs over n1, twiddles W_R^(n2 k1), R2-point
// DFTs over n2.  They let long transforms run in fewer LDS stages (384 as
// 24 x 16: 0.50 -> 0.44 ms for the plate z pass; 640 as 40 x 16 was slower,
// its 80-register butterflies cost occupancy).  TwiddleTable<R> holds cos / sin (2 pi m / R)
// for m = 0 .. (R1 - 1)(R2 - 1), rounded to double.
template <int R> struct TwiddleTable;
template <> struct TwiddleTable<20> {
    static constexpr int N = 13;
    static constexpr double c[13] = {
        1, 0.95105651629515353, 0.80901699437494745, 0.58778525229247314, 0.30901699437494745, 0,
        -0.30901699437494734, -0.58778525229247303, -0.80901699437494734, -0.95105651629515353, -1,
        -0.95105651629515375, -0.80901699437494756};
    static constexpr double s[13] = {
        0, 0.3090169943749474, 0.58778525229247314, 0.80901699437494745, 0.95105651629515353, 1,
        0.95105651629515364, 0.80901699437494745, 0.58778525229247325, 0.30901699437494751, 0,
        -0.3090169943749469, -0.58778525229247303};
};
template <> struct TwiddleTable<24> {
    static constexpr int N = 15;
    static constexpr double c[15] = {
        1, 0.96592582628906831, 0.86602540378443871, 0.70710678118654757, 0.50000000000000011,
        0.25881904510252074, 0, -0.25881904510252063, -0.49999999999999978, -0.70710678118654746,
        -0.86602540378443871, -0.9659258262890682, -1, -0.96592582628906831, -0.86602540378443882};
    static constexpr double s[15] = {
        0, 0.25881904510252074, 0.49999999999999994, 0.70710678118654746, 0.8660254037844386,
        0.96592582628906831, 1, 0.96592582628906831, 0.86602540378443871, 0.70710678118654757,
        0.49999999999999994, 0.25881904510252102, 0, -0.25881904510252079, -0.49999999999999972};
};
template <> struct TwiddleTable<40> {
    static constexpr int N = 29;
    static constexpr double c[29] = {
        1, 0.98768834059513777, 0.95105651629515353, 0.8910065241883679, 0.80901699437494745,
        0.70710678118654757, 0.58778525229247314, 0.4539904997395468, 0.30901699437494745,
        0.15643446504023092, 0, -0.15643446504023059, -0.30901699437494734, -0.45399049973954669,
        -0.58778525229247303, -0.70710678118654746, -0.80901699437494734, -0.89100652418836779,
        -0.95105651629515353, -0.98768834059513766, -1, -0.98768834059513777, -0.95105651629515375,
        -0.8910065241883679, -0.80901699437494756, -0.70710678118654768, -0.58778525229247325,
        -0.45399049973954692, -0.30901699437494756};
    static constexpr double s[29] = {
        0, 0.15643446504023087, 0.3090169943749474, 0.45399049973954675, 0.58778525229247314,
        0.70710678118654746, 0.80901699437494745, 0.89100652418836779, 0.95105651629515353,
        0.98768834059513777, 1, 0.98768834059513777, 0.95105651629515364, 0.8910065241883679,
        0.80901699437494745, 0.70710678118654757, 0.58778525229247325, 0.45399049973954686,
        0.30901699437494751, 0.15643446504023098, 0, -0.15643446504023073, -0.3090169943749469,
        -0.45399049973954669, -0.58778525229247303, -0.70710678118654746, -0.80901699437494734,
        -0.89100652418836779, -0.95105651629515353};
};

template <typename C, bool INV, int R1, int R2> struct DftComposite {
    __device__ __forceinline__ static void run(C *v) {
        using Re = decltype(v[0].x);
        using TT = TwiddleTable<R1 * R2>;
        C a[R1][R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            C t[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[n2 + R2 * n1];
            Dft<C, R1, INV>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                const int m = n2 * k1;
                if (m == 0) {
                    a[k1][n2] = t[k1];
                } else {
                    const Re c = (Re)TT::c[m], sg = INV ? (Re)TT::s[m] : (Re)-TT::s[m];
                    a[k1][n2] = C{t[k1].x * c - t[k1].y * sg, t[k1].x * sg + t[k1].y * c};
                }
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            Dft<C, R2, INV>::run(a[k1]);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = a[k1][k2];
        }
    }
};
template <typename C, bool INV> struct Dft<C, 20, INV> : DftComposite<C, INV, 5, 4> {};
template <typename C, bool INV> struct Dft<C, 24, INV> : DftComposite<C, INV, 3, 8> {};
template <typename C, bool INV> struct Dft<C, 40, INV> : DftComposite<C, INV, 5, 8> {};

// twiddle power w^r from the exact powers w1, w2, w4, w8
template <typename C, int r>
__device__ __forceinline__ C tw_pow(const C &w1, const C &w2, const C &w4, const C &w8) {
    if constexpr (r == 1) return w1;
    else if constexpr (r == 2) return w2;
    else if constexpr (r == 4) return w4;
    else if constexpr (r == 8) return w8;
    else if constexpr (r == 3) return cmul(w2, w1);
    else if constexpr (r == 5) return cmul(w4, w1);
    else if constexpr (r == 6) return cmul(w4, w2);
    else if constexpr (r == 7) return cmul(w4, cmul(w2, w1));
    else if constexpr (r == 9) return cmul(w8, w1);
    else if constexpr (r == 10) return cmul(w8, w2);
    else if constexpr (r == 11) return cmul(w8, cmul(w2, w1));
    else if constexpr (r == 12) return cmul(w8, w4);
    else if constexpr (r == 13) return cmul(cmul(w8, w4), w1);
    else if constexpr (r == 14) return cmul(cmul(w8, w4), w2);
    else return cmul(cmul(w8, w4), cmul(w2, w1));
}

// Workgroup barrier that orders LDS accesses only: global loads issued before
// it stay in flight (a full __syncthreads() would wait for them too), which
// lets a pass prefetch its next tile into registers while it transforms the
// current one in LDS.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// w^m = exp(-2 pi i m / P) from a half table t[0..P/2): w^(m + P/2) = -w^m
template <typename C, int P> __device__ __forceinline__ C tw_half(const C *__restrict__ t, int m) {
    if (m < P / 2) return t[m];
    const C w = t[m - P / 2];
    return C{-w.x, -w.y};
}

// Post-operation of the last stage (identity by default): called with the
// pencil, the output element index and its value before the value is stored.
struct NoPost {
    template <typename C> __device__ __forceinline__ C operator()(int, int, C v) const { return v; }
};

// One stage: radix R, Ns = product of the earlier radices.  Element j of
// pencil p at s[p * SP + j * SJ].  PFAST: consecutive threads walk pencils.
// Pruning: ZIN > 0 declares elements ZIN..P-1 of the input zero (the first
// stage then neither reads them nor spends arithmetic on them); ZOUT > 0
// declares only outputs 0..ZOUT-1 needed (the last stage stores only those,
// and the arithmetic that feeds nothing else is dropped); post is applied to
// every value the last stage stores.
template <typename C, int P, int NP, int SP, int SJ, bool PFAST, bool INV, int ZIN, int ZOUT, class Post, bool TT,
          int Ns, int R>
__device__ __forceinline__ void sfft_stage(C *s, const C *__restrict__ tw, const Post &post, const C *__restrict__ twt) {
    static_assert(R <= 16 || Ns == 1, "twiddle powers above 15 are not formed: a radix above 16 must come first");
    constexpr int nb = P / R;
    constexpr int total = nb * NP;
    constexpr int NB = (total + kFftThreads - 1) / kFftThreads;
    constexpr int tstep = P / (Ns * R);
    constexpr bool first = Ns == 1, last = Ns * R == P;
    // input r of a first-stage butterfly is element j + r nb (j < nb): zero for
    // r >= RIN, checked at run time for r == RIN - 1 when ZIN is not a
    // multiple of nb; output r of a last-stage butterfly is element j + r Ns
    constexpr int ZI = (first && ZIN > 0) ? ZIN : P, ZO = (last && ZOUT > 0) ? ZOUT : P;
    constexpr int RIN = first ? (ZI + nb - 1) / nb : R, ROUT = last ? (ZO + Ns - 1) / Ns : R;
    static_assert(RIN <= R && ROUT <= R, "pruning bounds");
    C v[NB][R];
    int ob[NB], op[NB], oe[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int idx = threadIdx.x + i * kFftThreads;
        if (total % kFftThreads == 0 || idx < total) {
            int p, j;
            if constexpr (PFAST) {
                p = idx % NP;
                j = idx / NP;
            } else {
                j = idx % nb;
                p = idx / nb;
            }
            const C *src = s + p * SP;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r < RIN && ((r + 1) * nb <= ZI || j + r * nb < ZI))
                    v[i][r] = src[(j + r * nb) * SJ];
                else
                    v[i][r] = C{};
            }
            const int k = (Ns == 1) ? 0 : j % Ns;
            if constexpr (Ns > 1 && TT && last) {
                // all powers w^(k r), r = 1..R-1, from the last stage's table
                const C *t = twt + k * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = t[r - 1];
                    if (INV) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            } else if constexpr (Ns > 1) {
                const int m = k * tstep;
                C w1 = tw_half<C, P>(tw, m);
                C w2 = R > 2 ? tw_half<C, P>(tw, (2 * m) % P) : w1;
                C w4 = R > 4 ? tw_half<C, P>(tw, (4 * m) % P) : w1;
                C w8 = R > 8 ? tw_half<C, P>(tw, (8 * m) % P) : w1;
                if (INV) {
                    w1.y = -w1.y;
                    w2.y = -w2.y;
                    w4.y = -w4.y;
                    w8.y = -w8.y;
                }
                [&]<int... rs>(std::integer_sequence<int, rs...>) {
                    ((v[i][rs + 1] = cmul(v[i][rs + 1], tw_pow<C, rs + 1>(w1, w2, w4, w8))), ...);
                }(std::make_integer_sequence<int, R - 1>{});
            }
            Dft<C, R, INV>::run(v[i]);
            op[i] = p;
            oe[i] = (j - k) * R + k;
            ob[i] = p * SP + oe[i] * SJ;
        }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int idx = threadIdx.x + i * kFftThreads;
        if (total % kFftThreads == 0 || idx < total) {
#pragma unroll
            for (int r = 0; r < ROUT; ++r) {
                if constexpr (last) {
                    if ((r + 1) * Ns <= ZO || oe[i] + r * Ns < ZO)
                        s[ob[i] + r * Ns * SJ] = post(op[i], oe[i] + r * Ns, v[i][r]);
                } else {
                    s[ob[i] + r * Ns * SJ] = v[i][r];
                }
            }
        }
    }
    lds_barrier();
}

template <typename C, int P, int NP, int SP, int SJ, bool PFAST, bool INV, int ZIN, int ZOUT, class Post, bool TT,
          int Ns, int... Rs>
struct SStages;
template <typename C, int P, int NP, int SP, int SJ, bool PFAST, bool INV, int ZIN, int ZOUT, class Post, bool TT,
          int Ns>
struct SStages<C, P, NP, SP, SJ, PFAST, INV, ZIN, ZOUT, Post, TT, Ns> {
    __device__ __forceinline__ static void run(C *, const C *, const Post &, const C *) {}
};
template <typename C, int P, int NP, int SP, int SJ, bool PFAST, bool INV, int ZIN, int ZOUT, class Post, bool TT,
          int Ns, int R, int... Rest>
struct SStages<C, P, NP, SP, SJ, PFAST, INV, ZIN, ZOUT, Post, TT, Ns, R, Rest...> {
    __device__ __forceinline__ static void run(C *s, const C *tw, const Post &post, const C *twt) {
        sfft_stage<C, P, NP, SP, SJ, PFAST, INV, ZIN, ZOUT, Post, TT, Ns, R>(s, tw, post, twt);
        SStages<C, P, NP, SP, SJ, PFAST, INV, ZIN, ZOUT, Post, TT, Ns * R, Rest...>::run(s, tw, post, twt);
    }
};

// Radix lists of the specialised lengths (product = P, at most four stages).
// A radix above 16 may only come first (its stage needs no twiddles).
template <int P> struct RadixOf;
template <int... Rs> struct LastOf;
template <int R> struct LastOf<R> { static constexpr int value = R; };
template <int R, int... Rest> struct LastOf<R, Rest...> {
    static constexpr int value = sizeof...(Rest) ? LastOf<Rest...>::value : R;
};
#define LGF_RADICES(P_, ...)                                                                        \
    template <> struct RadixOf<P_> {                                                                \
        template <typename C, int NP, int SP, int SJ, bool PFAST, bool INV, int ZIN, int ZOUT, class Post, bool TT> \
        using Run = SStages<C, P_, NP, SP, SJ, PFAST, INV, ZIN, ZOUT, Post, TT, 1, __VA_ARGS__>;    \
        static constexpr int last = LastOf<__VA_ARGS__>::value;                                     \
    };
LGF_RADICES(16, 16)
LGF_RADICES(32, 2, 16)
LGF_RADICES(48, 3, 16)
LGF_RADICES(64, 4, 16)
LGF_RADICES(80, 5, 16)
LGF_RADICES(96, 24, 4)
LGF_RADICES(128, 8, 16)
LGF_RADICES(144, 3, 3, 16)
LGF_RADICES(160, 40, 4)
LGF_RADICES(192, 24, 8)
LGF_RADICES(240, 3, 5, 16)
LGF_RADICES(256, 16, 16)
LGF_RADICES(288, 24, 3, 4)
LGF_RADICES(320, 20, 16)
LGF_RADICES(384, 24, 16)
LGF_RADICES(480, 3, 5, 2, 16)
LGF_RADICES(512, 2, 16, 16)
LGF_RADICES(576, 24, 3, 8)
LGF_RADICES(640, 5, 8, 16)
LGF_RADICES(768, 3, 16, 16)
LGF_RADICES(960, 3, 5, 4, 16)
LGF_RADICES(1024, 4, 16, 16)
#undef LGF_RADICES

template <typename C, int P, int NP, int SP, int SJ, bool PFAST, bool INV, int ZIN = 0, int ZOUT = 0,
          class Post = NoPost>
__device__ __forceinline__ void sfft(C *s, const C *tw, const Post &post = Post()) {
    RadixOf<P>::template Run<C, NP, SP, SJ, PFAST, INV, ZIN, ZOUT, Post, false>::run(s, tw, post, nullptr);
}
// the same with the last stage's twiddles read from a table built by
// last_stage_twiddles (all R-1 powers per butterfly class k)
template <typename C, int P, int NP, int SP, int SJ, bool PFAST, bool INV, int ZIN = 0, int ZOUT = 0,
          class Post = NoPost>
__device__ __forceinline__ void sfft_tt(C *s, const C *tw, const C *twt, const Post &post = Post()) {
    RadixOf<P>::template Run<C, NP, SP, SJ, PFAST, INV, ZIN, ZOUT, Post, true>::run(s, tw, post, twt);
}
// table of the last stage (radix R, Ns = P / R butterfly classes):
// t[k (R - 1) + r - 1] = w^(k r), forward sign, k < Ns, 1 <= r < R
template <typename C, int P, int R>
__device__ __forceinline__ void last_stage_twiddles(C *t, const C *__restrict__ tw) {
    constexpr int Ns = P / R;
    for (int e = threadIdx.x; e < Ns * (R - 1); e += kFftThreads) {
        const int k = e / (R - 1), r = e % (R - 1) + 1;
        t[e] = tw_half<C, P>(tw, (k * r) % P);
    }
}

}  // namespace lgfib
