// Exact unsigned 32-bit division by a run-time invariant divisor through a
// multiply-high, after T. Granlund and P. L. Montgomery, "Division by
// Invariant Integers using Multiplication" (PLDI 1994), figure 4.1:
// with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
//   t = mulhi(m, n);  q = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0)
// equals floor(n / d) for every 32-bit n and every d >= 1.
#pragma once

#include <cstdint>

#ifndef HOUGH_HD
#if defined(__HIPCC__)
#define HOUGH_HD __host__ __device__
#else
#define HOUGH_HD
#endif
#endif

namespace hough {

struct FastDiv32 {
    uint32_t m = 1;
    uint32_t sh1 = 0;
    uint32_t sh2 = 0;
};

inline FastDiv32 make_fastdiv32(uint32_t d)
{
    FastDiv32 f;
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) ++l;
    f.m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    f.sh1 = l < 1 ? l : 1;
    f.sh2 = l > 0 ? l - 1 : 0;
    return f;
}

HOUGH_HD inline uint32_t fastdiv32(uint32_t n, const FastDiv32 &f)
{
    const uint32_t t = uint32_t((uint64_t(f.m) * n) >> 32);
    return (t + ((n - t) >> f.sh1)) >> f.sh2;
}

// floor(u * nbins / span) for 0 <= u < span as one multiply-high and a
// shift: b = (u * m) >> (32 + s) with m = ceil(nbins * 2^(32+s) / span) and
// the smallest s >= 0 such that span^2 <= 2^(32+s).  Exact: u*m / 2^(32+s)
// exceeds u*nbins/span by less than span / 2^(32+s) <= 1/span, while
// u*nbins/span sits at least 1/span below the next integer (its fractional
// part is r/span with r <= span - 1).  Usable when m < 2^32.
struct BinMagic {
    uint32_t m = 0;
    uint32_t s = 0;
    bool ok = false;
};

inline BinMagic make_binmagic(uint64_t span, uint32_t nbins)
{
    BinMagic b;
    if (span == 0 || span >= (uint64_t(1) << 32) || nbins == 0) return b;
    const unsigned __int128 sq = (unsigned __int128)span * span;
    uint32_t s = 0;
    while (((unsigned __int128)1 << (32 + s)) < sq) ++s;
    const unsigned __int128 num = (unsigned __int128)nbins << (32 + s);
    const unsigned __int128 m = (num + span - 1) / span;
    if (m >= ((unsigned __int128)1 << 32)) return b;
    b.m = uint32_t(m);
    b.s = s;
    b.ok = true;
    return b;
}

// The sufficient condition above is far from necessary.  A smaller shift s'
// (down to 0, which saves an instruction per use) is accepted when the
// multiply-high is exact on every u in [0, span): the approximation
// f(u) = (u * m') >> (32 + s') is non-decreasing, so it equals the step
// function floor(u * nbins / span) everywhere iff it does at both ends of
// every step [ceil(k span / nbins), ceil((k + 1) span / nbins) - 1].
inline bool binmagic_exact(uint64_t span, uint32_t nbins, uint32_t m, uint32_t s)
{
    auto f = [&](uint64_t u) { return ((u * m) >> 32) >> s; };
    for (uint64_t k = 0; k < nbins; ++k) {
        const uint64_t a = (k * span + nbins - 1) / nbins;
        const uint64_t b = ((k + 1) * span + nbins - 1) / nbins;
        if (a >= b) continue;
        if (f(a) != k || f(b - 1) != k) return false;
    }
    return true;
}

inline BinMagic make_binmagic_min(uint64_t span, uint32_t nbins)
{
    BinMagic b = make_binmagic(span, nbins);
    if (!b.ok) return b;
    for (uint32_t s = 0; s < b.s; ++s) {
        const unsigned __int128 num = (unsigned __int128)nbins << (32 + s);
        const unsigned __int128 m = (num + span - 1) / span;
        if (m >= ((unsigned __int128)1 << 32)) continue;
        if (binmagic_exact(span, nbins, uint32_t(m), s)) {
            b.m = uint32_t(m);
            b.s = s;
            return b;
        }
    }
    return b;
}

HOUGH_HD inline uint32_t binmagic_apply(uint32_t u, uint32_t m, uint32_t s)
{
    return uint32_t(((uint64_t(u) * m) >> 32) >> s);
}

}  // namespace hough
