// tiles.hpp -- launch shapes of the element kernels, usable on host and device.
//
// Every kernel maps one thread to one (i,j) column of an element (a vertical
// line of nodes along t) and packs `epb` elements into one workgroup.  BP3.5
// works on the Nq x Nq GLL columns; BP1.0 and BP3.0 on the Ng x Ng GL columns
// (the GLL phases use a subset of those threads).  Exceptions: with one element
// per workgroup, BP1.0 and BP3.0 run the line-per-lane even-odd kernels of
// bp10t.hpp (one lane per GLL column) and bp30t.hpp (one lane per Gauss
// column), and BP3.5 at Nq >= 11 that of bp35t.hpp.
#pragma once

#include <array>

#include "fem_device.hpp"

namespace fem {

constexpr int kMaxThreads = 512;
constexpr int kMaxLds = 160 * 1024;   // gfx950 LDS per workgroup

constexpr int columns(int op, int nq) { return op == 1 ? nq * nq : (nq + 1) * (nq + 1); }

// LDS values of one BP3.0 element slot (three regions reused across phases).
constexpr int bp30_slot_values(int nq, int bytes)
{
    const int ng = nq + 1;
    const int pq = lds_row(nq, bytes), pg = lds_row(ng, bytes);
    const int r1a = nq * nq * pq, r1b = ng * ng * pg, r1c = nq * ng * pg;
    const int r1 = r1a > r1b ? (r1a > r1c ? r1a : r1c) : (r1b > r1c ? r1b : r1c);
    const int r2a = nq * nq * pg, r2b = ng * ng * pg;
    const int r2 = r2a > r2b ? r2a : r2b;
    return r1 + r2 + ng * ng * pg;
}

// BP1.0 with one element per workgroup runs the line-per-lane kernel
// (bp10t.hpp): ceil(Nq^2 / 64) waves, one for Nq <= 8.
constexpr bool bp10_wave(int nq, int epb) { return epb == 1; }

// Values of the interpolation half tables (LDS copies at high Nq).
constexpr int interp_half_values(int nq)
{
    const int ng = nq + 1;
    return ((ng + 1) / 2) * ((nq + 1) / 2) + (ng / 2) * (nq / 2 > 0 ? nq / 2 : 1);
}

// Row length of the line-per-lane BP1.0 kernel's LDS volumes: the bank
// model's, except FP64 at Nq = 16, where odd rows keep the workgroup under
// 80 KB of LDS (two workgroups per CU).
constexpr int bp10t_row(int nq, int bytes) { return bytes == 8 && nq == 16 ? 17 : lds_row(nq, bytes); }

// The BP1.0 line kernel stages the scaled Jacobians in rows of odd length
// (so the lanes of an r-direction pass, one row apart, fall on distinct
// banks) where their stored layout puts those lanes 256 bytes apart: Ng W
// bytes a multiple of 256 (Ng = 16 for every value size).
constexpr bool bp10t_remap_w(int ng, int gbytes) { return (ng * geo_vec(ng, gbytes) * gbytes) % 256 == 0; }
constexpr int bp10t_wrow(int ng) { return ng | 1; }

constexpr int bp10t_lds_bytes(int nq, int bytes, int gbytes)
{
    const int ng = nq + 1;
    const int p = bp10t_row(nq, bytes);
    const int av = ng * nq * p;                                                // [c][j][i] volume
    const int wv = bp10t_remap_w(ng, gbytes) ? (ng * ng * bp10t_wrow(ng) * gbytes + bytes - 1) / bytes
                                             : (ng * ng * ng * gbytes + 8 + bytes - 1) / bytes;   // staged wJ
    const int tab = nq >= 12 ? interp_half_values(nq) : 0;   // LDS tables
    return ((av > wv ? av : wv) + ng * ng * p + tab) * bytes;
}

// BP3.0 with one element per workgroup runs the line-per-lane kernel
// (bp30t.hpp): one lane per Gauss column, three Ng^3 LDS volumes -- or two
// (bp30t2.hpp) in FP64 arithmetic from Nq = 11, where the third volume kept a
// second workgroup off the CU (measured at E = 65536: Nq = 11 2.6 -> 4.1,
// Nq = 13 2.7 -> 4.2, Nq = 14 2.8 -> 4.1, Nq = 15 3.4 -> 4.4, Nq = 16 1.5 ->
// 3.0 TB/s; Nq = 12 at E = 131072: 4.15 -> 3.87 ms with three waves per SIMD).
constexpr bool bp30_line(int nq, int epb) { return epb == 1; }
constexpr bool bp30t_two_volumes(int nq, int bytes) { return bytes == 8 && nq >= 11; }

constexpr int bp30t_lds_bytes(int nq, int bytes)
{
    const int ng = nq + 1;
    const bool tlds = nq >= 11 || (bytes == 8 && nq >= 10);
    const int tab = tlds ? interp_half_values(nq) + 2 * ((ng + 1) / 2) * (ng / 2) : 0;   // LDS tables
    return ((bp30t_two_volumes(nq, bytes) ? 2 : 3) * ng * ng * lds_row(ng, bytes) + tab) * bytes;
}

// BP3.5 with one element per workgroup and Nq >= 9 runs the line-per-lane
// kernel (bp35t.hpp): two Nq^3 LDS volumes and the derivative half tables.
// Against the column kernel's best packing (E = 131072): Nq = 9 1.02x FP64,
// 1.05x FP32, 1.23x BF16, 1.27x BF16 factors with FP64 fields; Nq = 10
// 1.10x, 1.12x, 1.58x, 1.32x.
constexpr bool bp35_line(int nq, int epb) { return epb == 1 && nq >= 9; }

constexpr int bp35t_lds_bytes(int nq, int bytes)
{
    return (2 * nq * nq * lds_row(nq, bytes) + 2 * ((nq + 1) / 2) * (nq / 2)) * bytes;
}

// LDS bytes of one workgroup for values of `bytes` bytes (tables included);
// gbytes: stored size of a geometric value (BP1.0 one-wave staging).
constexpr int lds_bytes(int op, int nq, int epb, int bytes, int gbytes = 8)
{
    const int ng = nq + 1;
    const int pq = lds_row(nq, bytes), pg = lds_row(ng, bytes);
    if (op == 0 && bp10_wave(nq, epb)) return bp10t_lds_bytes(nq, bytes, gbytes);
    if (op == 2 && bp30_line(nq, epb)) return bp30t_lds_bytes(nq, bytes);
    if (op == 1 && bp35_line(nq, epb)) return bp35t_lds_bytes(nq, bytes);
    if (op == 1) return (nq * nq + 3 * epb * nq * nq * pq) * bytes;
    if (op == 0) {
        const int slot = nq * nq * pq + nq * nq * pg + nq * ng * pg;
        return (ng * nq + epb * slot) * bytes;
    }
    return (ng * nq + ng * ng + epb * bp30_slot_values(nq, bytes)) * bytes;
}

constexpr int threads_for(int op, int nq, int epb)
{
    return op == 0 && bp10_wave(nq, epb) ? round_up_wave(nq * nq) : round_up_wave(columns(op, nq) * epb);
}

// Up to four supported elements-per-workgroup values: 1, then those that fill
// at least 80% of the lanes of the workgroup's waves within the thread and
// LDS limits (sized for 8-byte values, the largest).
constexpr std::array<int, 4> epb_choices(int op, int nq)
{
    std::array<int, 4> out{0, 0, 0, 0};
    const int cand[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 21, 32, 64};
    int cnt = 0;
    for (int c : cand) {
        if (cnt == 4) break;
        const int th = threads_for(op, nq, c);
        if (th > kMaxThreads || lds_bytes(op, nq, c, 8) > kMaxLds) continue;
        const int used = columns(op, nq) * c;
        if (c == 1 || used * 5 >= th * 4) out[cnt++] = c;
    }
    return out;
}

// One element per workgroup when its columns already fill 80% of the lanes,
// else the smallest packing that does.
constexpr int epb_default(int op, int nq)
{
    if (op == 0 && nq >= 5) return 1;  // the line-per-lane BP1.0 kernel (measured fastest, N = 4..15)
    if (op == 2 && nq >= 4) return 1;  // the line-per-lane BP3.0 kernel (FP64, N = 3..15)
    const int cols = columns(op, nq);
    if (cols * 5 >= round_up_wave(cols) * 4) return 1;
    const auto ch = epb_choices(op, nq);
    for (int c : ch)
        if (c > 1) return c;
    return 1;
}

}  // namespace fem
