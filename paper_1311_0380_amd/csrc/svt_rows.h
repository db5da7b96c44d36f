// Row loops of the SVT fit kernel (arXiv:1311.0380, Sec. 2).  A road's
// combinations are split into rows: two of its layers index the rows, the
// other two (the inner layers, a before b in layer order) are looped over
// inside each row.  For one row these loops give
// every combination's constraint rows y3..y5 and chi2 in fp64, the pass
// count and the best.  Below, p2/n2 are the staged hit list and hit count
// of inner layer a, p3/n3 those of inner layer b.
//
// Every quantity is an integer below 2^53 whenever chi2 <= cut < 2^48, so
// the cut, the count and the minimum are exact.  When cut < 2^44 the
// combination index rides in the fraction bits of the value being minimised,
// chi2 + (i2 * 16 + i3) / 256, which is then exact too (the "fraction form"):
// one v_min_f64 keeps both the smallest chi2 and, among equal ones, the
// lowest index.  Otherwise a compare-and-select keeps them (general form).
//
// Rows are expected sorted by (n3, n2), largest first, within a wavefront, so
// that the first lane holds the wavefront's largest (n3, n2); every lane is
// active.  Within a row the combinations run in (i_a, i_b) order, which is
// their order in the combination index k because a comes before b.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svt {
namespace {

// DPP controls: row_shr:n shifts within a row of 16 lanes; row_bcast:15 and
// row_bcast:31 carry lane 15 / lane 31 into the following rows.
constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int Ctrl, int RowMask, bool Bound>
__device__ __forceinline__ uint32_t dpp(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, Ctrl, RowMask, 0xF, Bound);
}

// Inclusive prefix sum across the wavefront (all lanes active).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    x += dpp<kRowShr + 1, 0xF, true>(x);
    x += dpp<kRowShr + 2, 0xF, true>(x);
    x += dpp<kRowShr + 4, 0xF, true>(x);
    x += dpp<kRowShr + 8, 0xF, true>(x);
    x += dpp<kRowBcast15, 0xA, false>(x);
    x += dpp<kRowBcast31, 0xC, false>(x);
    return x;
}

// Sum and minimum across the wavefront (all lanes active), as uniform values.
__device__ __forceinline__ uint32_t wave_sum(uint32_t x)
{
    return __builtin_amdgcn_readlane(wave_incl_scan(x), 63);
}

template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp_or_max(uint32_t x)
{
    // lanes without a source keep 0xFFFFFFFF, the identity of min
    return (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, Ctrl, RowMask, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t x)
{
    x = min(x, dpp_or_max<kRowShr + 1, 0xF>(x));
    x = min(x, dpp_or_max<kRowShr + 2, 0xF>(x));
    x = min(x, dpp_or_max<kRowShr + 4, 0xF>(x));
    x = min(x, dpp_or_max<kRowShr + 8, 0xF>(x));
    x = min(x, dpp_or_max<kRowBcast15, 0xA>(x));
    x = min(x, dpp_or_max<kRowBcast31, 0xC>(x));
    return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

struct Row {
    double z3, z4, z5;   // constraint rows with layers 0, 1 and the XFT words
    double a3, a4, a5;   // column of layer 2
    double c3, c4, c5;   // column of layer 3
    double best;         // fraction form: chi2 + idx / 256; else chi2 of the best
    uint32_t bidx;       // (i_a << 4) | i_b of the best (general form), ~0 if none
    uint32_t np;         // passing combinations
};

// ---- fraction form (cut < 2^44) ------------------------------------------
// v = chi2 + i3 / 256 is exact below 2^45; a chi2 at or above 2^45 rounds to
// a value still above cut + 1, so v <= cut + 1/2 is exactly chi2 <= cut.

// v_min_f64 without the NaN-quieting max that a library fmin puts in front
// of it (no value here is a NaN).
__device__ __forceinline__ double dmin(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// np += (v <= lim) as one compare into VCC and one add of its carry, in
// place of a compare, a select and an add.
__device__ __forceinline__ void count_le(uint32_t &np, double v, double lim)
{
    asm("v_cmp_le_f64_e32 vcc, %1, %2\n\tv_addc_co_u32_e32 %0, vcc, 0, %0, vcc"
        : "+v"(np)
        : "v"(v), "v"(lim)
        : "vcc");
}

// The road key of a row's best, chi2 << 16 | i0 << 12 | i1 << 8 | i2 << 4 | i3,
// and whether the row has a passing combination.  rowbits holds the row
// layers' indices at their places in the key; sa and sb are the places
// (12 - 4 * layer) of inner layers a and b.  In the fraction form
// 256 * best = 256 chi2 + (i_a * 16 + i_b) is an integer below 2^52, which
// fma(best, 256, 2^52) places in the low mantissa bits exactly.
template <bool F>
__device__ __forceinline__ bool row_key(const Row &st, double cut, uint32_t rowbits, uint32_t sa,
                                        uint32_t sb, unsigned long long &key)
{
    if constexpr (F) {
        const double t = fma(st.best, 256.0, 0x1p52);
        const unsigned long long k =
            (unsigned long long)__double_as_longlong(t) & 0x000FFFFFFFFFFFFFull;
        const uint32_t lo = (uint32_t)k;
        key = ((k >> 8) << 16) |
              (rowbits | (((lo >> 4) & 15u) << sa) | ((lo & 15u) << sb));
        return st.best < cut + 1.0;
    } else {
        key = ((unsigned long long)st.best << 16) |
              (rowbits | (((st.bidx >> 4) & 15u) << sa) | ((st.bidx & 15u) << sb));
        return st.bidx != 0xFFFFFFFFu;
    }
}

// Small rows, fully unrolled: N2 = the wavefront's largest n2, N3 = its n3
// (the same in every lane).  All hits are loaded up front.  i2 past the
// lane's n2 is masked off, so its word is read unclamped (the staged hit
// array carries a pad of 16 words for this).
template <int N2, int N3>
__device__ __forceinline__ void frac_small(Row &st, const int16_t *hit, uint32_t p2, uint32_t p3,
                                           uint32_t n2, double lim)
{
    double h2[N2], h3[N3];
#pragma unroll
    for (int i = 0; i < N2; ++i) h2[i] = (double)hit[p2 + i];
#pragma unroll
    for (int i = 0; i < N3; ++i) h3[i] = (double)hit[p3 + i];
#pragma unroll
    for (int i2 = 0; i2 < N2; ++i2) {
        if (i2 == 0 || (uint32_t)i2 < n2) {
            const double q3 = fma(st.a3, h2[i2], st.z3);
            const double q4 = fma(st.a4, h2[i2], st.z4);
            const double q5 = fma(st.a5, h2[i2], st.z5);
#pragma unroll
            for (int i3 = 0; i3 < N3; ++i3) {
                const double y3 = fma(st.c3, h3[i3], q3);
                const double y4 = fma(st.c4, h3[i3], q4);
                const double y5 = fma(st.c5, h3[i3], q5);
                const double v =
                    fma(y5, y5, fma(y4, y4, fma(y3, y3, (i2 * 16 + i3) * (1.0 / 256))));
                count_le(st.np, v, lim);
                st.best = dmin(st.best, v);
            }
        }
        // keep the scheduler from interleaving all N2 * N3 combinations,
        // which would cost more registers than it gains
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int N3>
__device__ __forceinline__ void frac_uniform(Row &st, const int16_t *hit, uint32_t p2, uint32_t p3,
                                             uint32_t n2, uint32_t n2w, double lim)
{
    constexpr int H = N3 <= 8 ? N3 : 1;
    double h3[H];
    if constexpr (N3 <= 8) {
#pragma unroll
        for (int i3 = 0; i3 < N3; ++i3) h3[i3] = (double)hit[p3 + i3];
    }
    double h2n = (double)hit[p2];
    double f2 = 0.0;
    for (uint32_t i2 = 0; i2 < n2w; ++i2, f2 += 1.0 / 16) {
        const double h2 = h2n;
        h2n = (double)hit[p2 + (i2 + 1 < n2 ? i2 + 1 : n2 - 1)];   // next, in flight
        if (i2 < n2) {
            const double q3 = fma(st.a3, h2, st.z3);
            const double q4 = fma(st.a4, h2, st.z4);
            const double q5 = fma(st.a5, h2, st.z5);
            double bi = __builtin_inf();
            if constexpr (N3 <= 8) {
#pragma unroll
                for (int i3 = 0; i3 < N3; ++i3) {
                    const double y3 = fma(st.c3, h3[i3], q3);
                    const double y4 = fma(st.c4, h3[i3], q4);
                    const double y5 = fma(st.c5, h3[i3], q5);
                    const double v = fma(y5, y5, fma(y4, y4, fma(y3, y3, i3 * (1.0 / 256))));
                    count_le(st.np, v, lim);
                    bi = dmin(bi, v);
                }
            } else {
                double f3 = 0.0;
#pragma unroll 4
                for (int i3 = 0; i3 < N3; ++i3, f3 += 1.0 / 256) {
                    const double h = (double)hit[p3 + i3];
                    const double y3 = fma(st.c3, h, q3);
                    const double y4 = fma(st.c4, h, q4);
                    const double y5 = fma(st.c5, h, q5);
                    const double v = fma(y5, y5, fma(y4, y4, fma(y3, y3, f3)));
                    count_le(st.np, v, lim);
                    bi = dmin(bi, v);
                }
            }
            st.best = dmin(st.best, bi + f2);
        }
    }
}

// Rows of different (n2, n3) in one wavefront: indices are clamped into the
// row's lists.  A clamped duplicate has the chi2 of a real combination and a
// larger fraction, so it never wins; it is kept out of the pass count.
__device__ __forceinline__ void frac_mixed(Row &st, const int16_t *hit, uint32_t p2, uint32_t p3,
                                           uint32_t n2, uint32_t n3, uint32_t n2w, uint32_t n3w,
                                           double lim)
{
    double f2 = 0.0;
    for (uint32_t i2 = 0; i2 < n2w; ++i2, f2 += 1.0 / 16) {
        const double h2 = (double)hit[p2 + (i2 < n2 ? i2 : n2 - 1)];
        const double q3 = fma(st.a3, h2, st.z3);
        const double q4 = fma(st.a4, h2, st.z4);
        const double q5 = fma(st.a5, h2, st.z5);
        double bi = __builtin_inf(), f3 = 0.0;
        for (uint32_t i3 = 0; i3 < n3w; ++i3, f3 += 1.0 / 256) {
            const double h = (double)hit[p3 + (i3 < n3 ? i3 : n3 - 1)];
            const double y3 = fma(st.c3, h, q3);
            const double y4 = fma(st.c4, h, q4);
            const double y5 = fma(st.c5, h, q5);
            const double v = fma(y5, y5, fma(y4, y4, fma(y3, y3, f3)));
            st.np += (v <= lim && i2 < n2 && i3 < n3) ? 1u : 0u;
            bi = dmin(bi, v);
        }
        st.best = dmin(st.best, bi + f2);
    }
}

// ---- general form (any cut < 2^48) ----------------------------------------

__device__ __forceinline__ void gen_combo(Row &st, double q3, double q4, double q5, double h3,
                                          double cut, uint32_t idx)
{
    const double y3 = fma(st.c3, h3, q3);
    const double y4 = fma(st.c4, h3, q4);
    const double y5 = fma(st.c5, h3, q5);
    const double c = fma(y5, y5, fma(y4, y4, y3 * y3));
    st.np += (c <= cut) ? 1u : 0u;
    const bool better = c < st.best;
    st.best = better ? c : st.best;
    st.bidx = better ? idx : st.bidx;
}

template <int N3>
__device__ __forceinline__ void gen_uniform(Row &st, const int16_t *hit, uint32_t p2, uint32_t p3,
                                            uint32_t n2, uint32_t n2w, double cut)
{
    for (uint32_t i2 = 0; i2 < n2w; ++i2) {
        if (i2 < n2) {
            const double h2 = (double)hit[p2 + i2];
            const double q3 = fma(st.a3, h2, st.z3);
            const double q4 = fma(st.a4, h2, st.z4);
            const double q5 = fma(st.a5, h2, st.z5);
#pragma unroll 4
            for (int i3 = 0; i3 < N3; ++i3)
                gen_combo(st, q3, q4, q5, (double)hit[p3 + i3], cut, (i2 << 4) | (uint32_t)i3);
        }
    }
}

__device__ __forceinline__ void gen_mixed(Row &st, const int16_t *hit, uint32_t p2, uint32_t p3,
                                          uint32_t n2, uint32_t n3, uint32_t n2w, uint32_t n3w,
                                          double cut)
{
    const double never = cut + 2.0;
    for (uint32_t i2 = 0; i2 < n2w; ++i2) {
        const double h2 = (double)hit[p2 + (i2 < n2 ? i2 : n2 - 1)];
        const double q3 = fma(st.a3, h2, st.z3);
        const double q4 = fma(st.a4, h2, st.z4);
        const double q5 = fma(st.a5, h2, st.z5);
        for (uint32_t i3 = 0; i3 < n3w; ++i3) {
            const double h = (double)hit[p3 + (i3 < n3 ? i3 : n3 - 1)];
            const double y3 = fma(st.c3, h, q3);
            const double y4 = fma(st.c4, h, q4);
            const double y5 = fma(st.c5, h, q5);
            double c = fma(y5, y5, fma(y4, y4, y3 * y3));
            c = (i2 < n2 && i3 < n3) ? c : never;
            st.np += (c <= cut) ? 1u : 0u;
            const bool better = c < st.best;
            st.best = better ? c : st.best;
            st.bidx = better ? ((i2 << 4) | i3) : st.bidx;
        }
    }
}

}  // namespace
}  // namespace svt
