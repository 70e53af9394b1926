// kg_fft.hpp -- device building blocks of the line FFTs (gfx950).
//
// The method needs two 3D FFTs per time step (Sec. 1.1.2, closing paragraph).
// Each 3D transform is done one axis at a time, every line by a group of
// threads of one workgroup.  A line of NL points (a power of two) is held as
// E = min(8, NL) complex values per thread by TPL = NL / E threads; thread t
// always owns positions {t + j*TPL : j < E}.  The transform is a Stockham
// decimation-in-time sequence of radix-R stages (R in {2, 4, 8}): stage s
// with L = product of the earlier radices computes, for butterfly i,
//     out[(i / L) * L * R + (i % L) + s' * L]
//         = sum_r w_R^(r s') * ( w_{L R}^(r (i % L)) * in[i + r * NL / R] ),
// which reads positions {t + j*TPL} in every stage and, in the last stage,
// also writes them.  Between stages the values go through LDS; the first
// stage takes them from registers and the last one leaves them in registers,
// so callers load and store global memory directly in the owned pattern.
#pragma once

#include <hip/hip_runtime.h>

namespace kg {

// Rounding of the transforms.  Every kernel inlines its own copy of these
// routines, and a compiler free to fuse a product into a following add picks
// the fusions per kernel, so two kernels could round the same transform
// differently.  The routines below therefore switch contraction off and
// write their fused multiply-adds explicitly: a transform rounds the same
// way in every kernel that runs it.  (The resting field that a step's z pass
// leaves and the one rebuilt from a stored level by another kernel must
// agree bit for bit for a checkpoint to resume bitwise.)
template <typename T>
__device__ __forceinline__ T fmx(T a, T b, T c)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b)
{
    cx<T> r;
    r.re = a;
    r.im = b;
    return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b)
{
#pragma clang fp contract(off)
    return mk(a.re + b.re, a.im + b.im);
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b)
{
#pragma clang fp contract(off)
    return mk(a.re - b.re, a.im - b.im);
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
#pragma clang fp contract(off)
    return mk(fmx(a.re, b.re, -(a.im * b.im)), fmx(a.re, b.im, a.im * b.re));
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b)
{
#pragma clang fp contract(off)
    return mk(fmx(a.re, b.re, a.im * b.im), fmx(a.im, b.re, -(a.re * b.im)));
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s)
{
#pragma clang fp contract(off)
    return mk(a.re * s, a.im * s);
}

// Streaming global accesses (each value is read or written once per pass):
// nontemporal hints keep them from displacing reused data in the caches.
template <typename T>
__device__ __forceinline__ cx<T> ld_nt(const cx<T> *p)
{
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
    return mk(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void st_nt(cx<T> *p, cx<T> a)
{
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
}

// Multiply by -i (DIR = -1, forward) or +i (DIR = +1, inverse).
template <int DIR, typename T>
__device__ __forceinline__ cx<T> rot90(cx<T> a)
{
    if constexpr (DIR < 0)
        return mk(a.im, -a.re);
    else
        return mk(-a.im, a.re);
}

// In-place DFT of R values with roots w_R = exp(DIR * 2 pi i / R).
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T> (&x)[R])
{
#pragma clang fp contract(off)
    if constexpr (R == 2) {
        cx<T> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = a - b;
    } else if constexpr (R == 3) {
        // w_3 = -1/2 + DIR i sqrt(3)/2
        const T h = (T)0.86602540378443864676372317075293618347;
        const cx<T> t1 = x[1] + x[2];
        const cx<T> t2 = mk(fmx(t1.re, (T)-0.5, x[0].re), fmx(t1.im, (T)-0.5, x[0].im));
        const cx<T> d = rot90<DIR>(x[1] - x[2]);
        x[0] = x[0] + t1;
        x[1] = mk(fmx(d.re, h, t2.re), fmx(d.im, h, t2.im));
        x[2] = mk(fmx(d.re, -h, t2.re), fmx(d.im, -h, t2.im));
    } else if constexpr (R == 4) {
        cx<T> y0 = x[0] + x[2], y1 = x[0] - x[2];
        cx<T> y2 = x[1] + x[3], y3 = rot90<DIR>(x[1] - x[3]);
        x[0] = y0 + y2;
        x[2] = y0 - y2;
        x[1] = y1 + y3;
        x[3] = y1 - y3;
    } else if constexpr (R == 8) {
        // Split into a[r] = x[r] + x[r+4] (even outputs) and
        // b[r] = (x[r] - x[r+4]) w_8^r (odd outputs), then two DFT-4.
        const T s = (T)0.70710678118654752440084436210484903928;
        cx<T> a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a[r] = x[r] + x[r + 4];
            b[r] = x[r] - x[r + 4];
        }
        // w_8^1 = (1 + DIR i)/sqrt2, w_8^2 = DIR i, w_8^3 = (-1 + DIR i)/sqrt2
        b[1] = mk(s * (b[1].re - (T)DIR * b[1].im), s * (b[1].im + (T)DIR * b[1].re));
        b[2] = rot90<DIR>(b[2]);
        b[3] = mk(s * (-b[3].re - (T)DIR * b[3].im), s * (-b[3].im + (T)DIR * b[3].re));
        dft<4, DIR>(a);
        dft<4, DIR>(b);
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            x[2 * s2] = a[s2];
            x[2 * s2 + 1] = b[s2];
        }
    }
}

// Radix plan of a line of NL points.
//   NL = 2^a (2 <= NL <= 4096): E = min(8, NL) values per thread; the first
//     stage takes the remainder radix (2 or 4) when a is not a multiple of 3,
//     every other stage is radix 8.
//   NL = 3 * 2^a (12 <= NL <= 3072): E = 12; a radix-3 stage, then a radix-2
//     stage when a is odd, then radix-4 stages.
// Every radix divides E, which keeps thread t on positions {t + j*TPL}.
template <int NL>
struct Radix {
    static constexpr bool THREE = (NL % 3 == 0);
    static constexpr int BASE = THREE ? NL / 3 : NL;
    static constexpr int log2n()
    {
        int l = 0;
        while ((1 << l) < BASE) ++l;
        return l;
    }
    static constexpr int LG = log2n();
    static constexpr int E = THREE ? 12 : (NL >= 8 ? 8 : NL);
    static constexpr int TPL = NL / E;
    static constexpr int REM = THREE ? (LG & 1) : LG % 3;
    static constexpr int NST = THREE ? 1 + REM + LG / 2 : LG / 3 + (REM ? 1 : 0);
    static constexpr int radix(int s)
    {
        if (THREE) return s == 0 ? 3 : (REM && s == 1) ? 2 : 4;
        return (REM && s == 0) ? (1 << REM) : 8;
    }
    static constexpr int lbefore(int s)
    {
        int l = 1;
        for (int q = 0; q < s; ++q) l *= radix(q);
        return l;
    }
    static_assert((1 << LG) == BASE, "line length must be 2^a or 3 * 2^a");
    static_assert(!THREE || NL >= 12, "3 * 2^a lines need at least 12 points");
    static_assert(TPL * E == NL, "positions must divide evenly among threads");
};

// LDS slot of line position p: one padding slot after every 2^SH positions
// (SH = 0: none), so the strided writes of the early stages spread over the
// LDS banks.  The y and z passes interleave W lines per slot and use SH = 3.
template <int SH = 3>
__device__ __forceinline__ int lpos(int p) { return SH > 0 ? p + (p >> SH) : p; }
template <int NL, int SH = 3>
constexpr int lslots() { return SH > 0 ? NL + NL / (1 << SH) : NL; }

// SH = SWZ: no padding; instead bits 0-2 of a position are XORed with bits
// 3-5 and bit 3 with bit 6, a bijection on every aligned block of 128
// positions.  LDS serves the lanes of a wavefront in groups of 128 bytes
// (8 lanes of 16-byte values, 16 lanes of 8-byte ones); within such a group
// the strided stage writes of a contiguous radix-8 line (positions 8t + s,
// and 64(t/8) + 8s + t%8) then hit distinct banks, and the contiguous reads
// t + j*TPL stay a permutation of one bank row.  It needs no LDS beyond the
// line and less index arithmetic than padding.
constexpr int SWZ = -1;
template <int NL, int SH>
__device__ __forceinline__ int lslot(int p)
{
    if constexpr (SH == SWZ) {
        static_assert(NL % 128 == 0, "the swizzle permutes whole blocks of 128 positions");
        return p ^ ((p >> 3) & 7) ^ (((p >> 6) & 1) << 3);
    } else {
        return lpos<SH>(p);
    }
}

// Synchronisation between the stages of one line: the whole workgroup
// (lines spread over several waves) or one wave (every thread of the line,
// and of every line sharing its LDS, sits in the same wavefront; LDS
// operations of a wave complete in issue order, so a compiler fence is enough).
enum { SYNC_BLOCK = 0, SYNC_WAVE = 1 };
template <int SY>
__device__ __forceinline__ void stage_sync()
{
    if constexpr (SY == SYNC_BLOCK) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Twiddles w^r, r = 1..R-1, of one butterfly from the table entries w, w^2
// and w^4 (each at most two products away from a table value).
template <int R, typename T>
__device__ __forceinline__ void twiddles(cx<T> (&w)[R], const cx<T> *__restrict__ tw, int idx)
{
#pragma clang fp contract(off)
    w[1] = tw[idx];
    if constexpr (R == 3) w[2] = tw[2 * idx];
    if constexpr (R >= 4) {
        w[2] = tw[2 * idx];
        w[3] = cmul(w[1], w[2]);
    }
    if constexpr (R == 8) {
        w[4] = tw[4 * idx];
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
    }
}

// Twiddle base values (w, w^2, w^4) of every twiddled stage of a line,
// loaded into registers ahead of the transform: the stages then wait on no
// memory.  Only for lines whose twiddled stages are all radix 8 with one
// butterfly per thread, i.e. 2^a lines of at least 16 points (their only
// non-radix-8 stage is the first, which needs no twiddles).
template <typename T, int NL>
struct TwPre {
    static constexpr bool OK = !Radix<NL>::THREE && Radix<NL>::E == 8 && NL >= 16;
    cx<T> w[Radix<NL>::NST][3];
};

template <typename T, int NL, int S = 1>
__device__ __forceinline__ void twiddle_preload(TwPre<T, NL> &p, const cx<T> *__restrict__ tw,
                                                int t, int twm)
{
    using P = Radix<NL>;
    static_assert(TwPre<T, NL>::OK, "twiddle preloading needs radix-8 twiddled stages");
    if constexpr (S < P::NST) {
        constexpr int R = P::radix(S), L = P::lbefore(S);
        static_assert(R == 8, "twiddled stages must be radix 8");
        const int idx = (t % L) * (NL / (L * R)) * twm;
        p.w[S][0] = tw[idx];
        p.w[S][1] = tw[2 * idx];
        p.w[S][2] = tw[4 * idx];
        twiddle_preload<T, NL, S + 1>(p, tw, t, twm);
    }
}

// Stockham stages S..NST-1 of a line.  v holds the owned positions on entry
// to stage 0 and on exit from the last stage.  lds points at slot 0 of this
// line in an LDS buffer where consecutive slots are `ls` elements apart (the
// line needs lslots<NL>() slots).  tw is the table exp(-2 pi i j / NTAB) with
// NTAB = NL * twm.  Callers must make sure nobody still reads the LDS line.
// With a TwPre (pre non-null) the twiddles come from its registers instead
// of the table.
template <typename T, int NL, int DIR, int SY = SYNC_BLOCK, int SH = 3, int S = 0>
__device__ __forceinline__ void fft_line(cx<T> (&v)[Radix<NL>::E], cx<T> *lds, int ls, int t,
                                         const cx<T> *__restrict__ tw, int twm,
                                         const TwPre<T, NL> *pre = nullptr)
{
#pragma clang fp contract(off)
    using P = Radix<NL>;
    constexpr int E = P::E, TPL = P::TPL;
    constexpr int R = P::radix(S), L = P::lbefore(S);
    constexpr bool last = (S == P::NST - 1);
    if constexpr (S > 0) {
        stage_sync<SY>();
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = lds[lslot<NL, SH>(t + j * TPL) * ls];
        if constexpr (!last) stage_sync<SY>();
    }
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        const int i = t + TPL * b;
        const int k = i % L;  // L is a compile-time constant
        cx<T> x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = v[b + r * (E / R)];
        if constexpr (L > 1) {
            cx<T> w[R];
            if constexpr (R == 8 && TwPre<T, NL>::OK) {
                if (pre) {
                    w[1] = pre->w[S][0];
                    w[2] = pre->w[S][1];
                    w[3] = cmul(w[1], w[2]);
                    w[4] = pre->w[S][2];
                    w[5] = cmul(w[1], w[4]);
                    w[6] = cmul(w[2], w[4]);
                    w[7] = cmul(w[3], w[4]);
                } else {
                    twiddles<R>(w, tw, k * (NL / (L * R)) * twm);
                }
            } else {
                twiddles<R>(w, tw, k * (NL / (L * R)) * twm);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) x[r] = (DIR < 0) ? cmul(x[r], w[r]) : cmulc(x[r], w[r]);
        }
        dft<R, DIR>(x);
        if constexpr (last) {
#pragma unroll
            for (int s = 0; s < R; ++s) v[b + s * (E / R)] = x[s];
        } else {
            const int base = (i / L) * L * R + k;
#pragma unroll
            for (int s = 0; s < R; ++s) lds[lslot<NL, SH>(base + s * L) * ls] = x[s];
        }
    }
    if constexpr (!last) fft_line<T, NL, DIR, SY, SH, S + 1>(v, lds, ls, t, tw, twm, pre);
}

}  // namespace kg
