// Supported 1D lengths and their compile-time radix plans.
//
// Every axis of a 3D transform is a batch of 1D DFTs (paper Sec. III-A: the 3D
// FFT is the tensor product of 1D FFTs along x, y and z).  The GPU kernels are
// specialised per length: the radix sequence of the Stockham passes, the
// number of threads that cooperate on one line and the per-thread register
// footprint are constants, so every butterfly is fully unrolled.
//
// This header is plain C++ (no HIP) so the host-side plan can use it too.
#pragma once

// Lengths with a compiled kernel: products 2^a 3^b 5^c 7^d up to 4096 that
// cover every workload shape (including the 480, 720 and 840 grids of the
// paper's GPU runs) plus a spread of common sizes, and 11 and 13 times powers
// of two (the generic odd-prime radix).
#define FFT3D_FOR_EACH_LENGTH(X)                                                      \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(14) X(15) X(16) X(20)       \
    X(21) X(24) X(25) X(28) X(30) X(32) X(35) X(40) X(42) X(48) X(50) X(56) X(60)     \
    X(64) X(70) X(75) X(80) X(84) X(96) X(100) X(105) X(112) X(120) X(125) X(128)     \
    X(140) X(150) X(160) X(168) X(192) X(200) X(210) X(240) X(250) X(256) X(280)      \
    X(300) X(320) X(384) X(400) X(420) X(480) X(500) X(512) X(600) X(640) X(720)      \
    X(750) X(768) X(800) X(840) X(960) X(1000) X(1024) X(2048) X(4096)                \
    X(11) X(13) X(22) X(26) X(44) X(52) X(88) X(104) X(176) X(208)

namespace fft3d {

// Radix sequence of a length-n Stockham FFT.  np passes with radices r[0..np);
// tpl threads cooperate on one line; pass p has n / r[p] butterflies, split
// round-robin over the tpl threads (a thread may have one masked butterfly).
struct RadixPlan {
    int n;
    int np;
    int r[12];
    int tpl;
};

constexpr RadixPlan radix_plan(int n)
{
    RadixPlan p{n, 0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, 1};
    if (n < 1) {
        p.np = -1;
        return p;
    }
    int m = n, a = 0, b = 0, c = 0, d = 0, e = 0, f = 0;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    while (m % 5 == 0) { m /= 5; ++c; }
    while (m % 7 == 0) { m /= 7; ++d; }
    while (m % 11 == 0) { m /= 11; ++e; }  // the generic prime radix (dft_prime)
    while (m % 13 == 0) { m /= 13; ++f; }
    if (m != 1) {
        p.np = -1;
        return p;
    }
    // power-of-two part: as few passes as possible, radices no larger than 16,
    // the larger radices first
    while (a > 12) { p.r[p.np++] = 16; a -= 4; }
    switch (a) {
    case 1: p.r[p.np++] = 2; break;
    case 2: p.r[p.np++] = 4; break;
    case 3: p.r[p.np++] = 8; break;
    case 4: p.r[p.np++] = 16; break;
    case 5: p.r[p.np++] = 8; p.r[p.np++] = 4; break;
    case 6: p.r[p.np++] = 8; p.r[p.np++] = 8; break;
    case 7: p.r[p.np++] = 16; p.r[p.np++] = 8; break;
    case 8: p.r[p.np++] = 8; p.r[p.np++] = 8; p.r[p.np++] = 4; break;  // not 16 x 16: half the registers
    case 9: p.r[p.np++] = 8; p.r[p.np++] = 8; p.r[p.np++] = 8; break;
    case 10: p.r[p.np++] = 16; p.r[p.np++] = 8; p.r[p.np++] = 8; break;
    case 11: p.r[p.np++] = 16; p.r[p.np++] = 16; p.r[p.np++] = 8; break;
    case 12: p.r[p.np++] = 16; p.r[p.np++] = 16; p.r[p.np++] = 16; break;
    default: break;
    }
    // a factor 3 and a factor 5 together as one radix-15 pass (the
    // prime-factor butterfly) where no radix-16 pass sets the threads per
    // line: one pass fewer, and the larger largest radix means fewer threads
    // per line (840: 56 instead of 105, so strided tiles hold 16 lines
    // instead of 8).  With a radix-16 pass the threads per line stay n/16 and
    // a radix-15 pass would give each thread two butterflies (more registers).
    bool has16 = false;
    for (int i = 0; i < p.np; ++i) has16 = has16 || p.r[i] == 16;
    const int p15 = has16 ? 0 : (b < c ? b : c);
    for (int i = 0; i < p15; ++i) p.r[p.np++] = 15;
    for (int i = p15; i < b; ++i) p.r[p.np++] = 3;
    for (int i = p15; i < c; ++i) p.r[p.np++] = 5;
    for (int i = 0; i < d; ++i) p.r[p.np++] = 7;
    for (int i = 0; i < e; ++i) p.r[p.np++] = 11;
    for (int i = 0; i < f; ++i) p.r[p.np++] = 13;
    int rmax = 1;
    for (int i = 0; i < p.np; ++i) rmax = p.r[i] > rmax ? p.r[i] : rmax;
    p.tpl = n / rmax;
    return p;
}

// The same radices in the reverse pass order (ord 1), the alternative order
// the autotuner may pick for the line kernels; ord 0 is radix_plan(n).
constexpr RadixPlan radix_plan(int n, int ord)
{
    RadixPlan p = radix_plan(n);
    if (ord == 1)
        for (int i = 0, j = p.np - 1; i < j; ++i, --j) {
            const int t = p.r[i];
            p.r[i] = p.r[j];
            p.r[j] = t;
        }
    return p;
}

// Whether the reverse order is a different plan (not a palindrome of radices).
constexpr bool radix_order_distinct(int n)
{
    const RadixPlan p = radix_plan(n);
    for (int i = 0; i < p.np; ++i)
        if (p.r[i] != p.r[p.np - 1 - i]) return true;
    return false;
}

// Product of the radices of passes [0, pass): the sub-transform length that
// pass `pass` starts from.
constexpr int radix_ns(const RadixPlan& p, int pass)
{
    int ns = 1;
    for (int i = 0; i < pass; ++i) ns *= p.r[i];
    return ns;
}

// Complex values one thread holds during its widest pass.
constexpr int radix_ept(const RadixPlan& p)
{
    int e = 1;
    for (int i = 0; i < p.np; ++i) {
        int bf = p.n / p.r[i];
        int nb = (bf + p.tpl - 1) / p.tpl;
        e = nb * p.r[i] > e ? nb * p.r[i] : e;
    }
    return e;
}

// Per-pass twiddle table: pass p (radix R, sub-length Ns > 1) stores, for each
// k < Ns, the R roots W_n^(r * k * n / (Ns*R)), r = 0..R-1 (r = 0 is 1), so one
// butterfly's roots are contiguous.  Offsets are in complex entries.
constexpr int pass_table_offset(const RadixPlan& p, int pass)
{
    int off = 0;
    for (int i = 1; i < pass; ++i) off += radix_ns(p, i) * p.r[i];
    return off;
}

constexpr int pass_table_size(const RadixPlan& p)
{
    return p.np < 2 ? 0 : pass_table_offset(p, p.np);
}

inline bool length_supported(long long n)
{
#define FFT3D_LEN_CASE(L) case L:
    switch (n) {
        FFT3D_FOR_EACH_LENGTH(FFT3D_LEN_CASE)
        return true;
    default:
        return false;
    }
#undef FFT3D_LEN_CASE
}

}  // namespace fft3d
