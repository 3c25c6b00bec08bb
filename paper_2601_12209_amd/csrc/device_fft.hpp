// Device-side building blocks: complex arithmetic, radix-2/3/4/5/7/8/15/16
// butterflies and the Stockham pass driver used by every stage kernel.
//
// A length-N line is transformed by the passes of radix_plan(N).  Pass p
// (radix R, sub-transform length Ns before it) treats butterfly j < N/R:
//   inputs   a[r] = data[j + r*N/R],               r < R
//   twiddle  a[r] *= W_N^(r * (j mod Ns) * N/(Ns*R))   (staged in LDS)
//   DFT_R    on a
//   outputs  data'[(j / Ns)*Ns*R + (j mod Ns) + r*Ns] = a[r]
// (the self-sorting Stockham formulation: natural order in and out, no bit
// reversal).  Pass 0 reads through a caller-supplied loader (global memory),
// the last pass writes through a caller-supplied storer, and the passes in
// between exchange through LDS.  The butterflies are written for the forward
// sign (exponent -1); the conjugate-sign transform is taken as conj(F(conj x)),
// which the kernels apply at load and store time.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "fft_lengths.hpp"

#define FD __device__ __forceinline__

namespace fft3d {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <typename T> FD cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> FD cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> FD cpx<T> operator*(cpx<T> a, T s) { return {a.re * s, a.im * s}; }
// Fused multiply-add, explicit so that every kernel variant rounds the same
// way (the library is compiled without automatic contraction).
FD float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
FD double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> FD cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {fmadd(a.re, b.re, -(a.im * b.im)), fmadd(a.re, b.im, a.im * b.re)};
}
template <typename T> FD cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
template <typename T> FD cpx<T> mul_i(cpx<T> a) { return {-a.im, a.re}; }     // i * a
template <typename T> FD cpx<T> mul_negi(cpx<T> a) { return {a.im, -a.re}; }  // -i * a

// Global accesses marked non-temporal (streamed data that should not displace
// reusable lines from the caches); one 8- or 16-byte access per value.
template <typename T> FD void store_nt(cpx<T>* p, cpx<T> v)
{
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 w = {v.re, v.im};
    __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
}
template <typename T> FD cpx<T> load_nt(const cpx<T>* p)
{
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 w = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return cpx<T>{w.x, w.y};
}

// cos/sin constants of the small DFTs, in long double so each precision gets
// its correctly rounded value.
#define K_SQRT1_2 0.707106781186547524400844362104849039L
#define K_SIN_PI_3 0.866025403784438646763723170752936183L
#define K_COS_2PI_5 0.309016994374947424102293417182819059L
#define K_COS_4PI_5 (-0.809016994374947424102293417182819059L)
#define K_SIN_2PI_5 0.951056516295153572116439333379382143L
#define K_SIN_4PI_5 0.587785252292473129168705954639072769L
#define K_COS_2PI_7 0.623489801858733530525004884004239811L
#define K_COS_4PI_7 (-0.222520933956314404288902564496794759L)
#define K_COS_6PI_7 (-0.900968867902419126236102319507445051L)
#define K_SIN_2PI_7 0.781831482468029808708444526674057750L
#define K_SIN_4PI_7 0.974927912181823607018131682993931217L
#define K_SIN_6PI_7 0.433883739117558120475768332848358755L
#define K_COS_PI_8 0.923879532511286756128183189396788933L
#define K_SIN_PI_8 0.382683432365089771728459984030398866L

// ---------------------------------------------------------------- DFT_R
// Forward sign: X[k] = sum_j x[j] exp(-2 pi i j k / R), in place, natural order.

template <typename T> FD void dft2(cpx<T>* v)
{
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <typename T> FD void dft3(cpx<T>* v)
{
    const T h = (T)K_SIN_PI_3;
    cpx<T> s = v[1] + v[2];
    cpx<T> m = v[0] - s * (T)0.5;
    cpx<T> d = (v[1] - v[2]) * h;
    v[0] = v[0] + s;
    v[1] = m + mul_negi(d);
    v[2] = m + mul_i(d);
}

template <typename T> FD void dft4v(cpx<T>& x0, cpx<T>& x1, cpx<T>& x2, cpx<T>& x3)
{
    cpx<T> s02 = x0 + x2, d02 = x0 - x2, s13 = x1 + x3, d13 = x1 - x3;
    x0 = s02 + s13;
    x2 = s02 - s13;
    x1 = d02 + mul_negi(d13);
    x3 = d02 + mul_i(d13);
}

template <typename T> FD void dft4(cpx<T>* v) { dft4v(v[0], v[1], v[2], v[3]); }

template <typename T> FD void dft5(cpx<T>* v)
{
    const T c1 = (T)K_COS_2PI_5, c2 = (T)K_COS_4PI_5, s1 = (T)K_SIN_2PI_5, s2 = (T)K_SIN_4PI_5;
    cpx<T> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
    cpx<T> x0 = v[0];
    cpx<T> a1 = x0 + t1 * c1 + t2 * c2;
    cpx<T> a2 = x0 + t1 * c2 + t2 * c1;
    cpx<T> b1 = t3 * s1 + t4 * s2;
    cpx<T> b2 = t3 * s2 - t4 * s1;
    v[0] = x0 + t1 + t2;
    v[1] = a1 + mul_negi(b1);
    v[4] = a1 + mul_i(b1);
    v[2] = a2 + mul_negi(b2);
    v[3] = a2 + mul_i(b2);
}

// radix 7 from the mirrored pairs t_j = x_j + x_{7-j}, d_j = x_j - x_{7-j}:
// X_k = x_0 + sum_j t_j cos(2 pi jk/7) - i sum_j d_j sin(2 pi jk/7), and
// X_{7-k} the same with +i, for k = 1..3 (jk reduced mod 7 by symmetry).
template <typename T> FD void dft7(cpx<T>* v)
{
    const T c1 = (T)K_COS_2PI_7, c2 = (T)K_COS_4PI_7, c3 = (T)K_COS_6PI_7;
    const T s1 = (T)K_SIN_2PI_7, s2 = (T)K_SIN_4PI_7, s3 = (T)K_SIN_6PI_7;
    const cpx<T> t1 = v[1] + v[6], t2 = v[2] + v[5], t3 = v[3] + v[4];
    const cpx<T> d1 = v[1] - v[6], d2 = v[2] - v[5], d3 = v[3] - v[4];
    const cpx<T> x0 = v[0];
    const cpx<T> a1 = x0 + t1 * c1 + t2 * c2 + t3 * c3;
    const cpx<T> a2 = x0 + t1 * c2 + t2 * c3 + t3 * c1;
    const cpx<T> a3 = x0 + t1 * c3 + t2 * c1 + t3 * c2;
    const cpx<T> b1 = d1 * s1 + d2 * s2 + d3 * s3;
    const cpx<T> b2 = d1 * s2 - d2 * s3 - d3 * s1;
    const cpx<T> b3 = d1 * s3 - d2 * s1 + d3 * s2;
    v[0] = x0 + t1 + t2 + t3;
    v[1] = a1 + mul_negi(b1);
    v[6] = a1 + mul_i(b1);
    v[2] = a2 + mul_negi(b2);
    v[5] = a2 + mul_i(b2);
    v[3] = a3 + mul_negi(b3);
    v[4] = a3 + mul_i(b3);
}

// radix 8 as 2 x 4: u_j = x_j + x_{j+4}, v_j = (x_j - x_{j+4}) W8^j, then DFT4
// of u gives the even outputs and DFT4 of v the odd ones.
template <typename T> FD void dft8(cpx<T>* x)
{
    const T r = (T)K_SQRT1_2;
    cpx<T> u0 = x[0] + x[4], u1 = x[1] + x[5], u2 = x[2] + x[6], u3 = x[3] + x[7];
    cpx<T> v0 = x[0] - x[4], v1 = x[1] - x[5], v2 = x[2] - x[6], v3 = x[3] - x[7];
    v1 = cpx<T>{(v1.re + v1.im) * r, (v1.im - v1.re) * r};   // * (1 - i)/sqrt2
    v2 = mul_negi(v2);                                        // * -i
    v3 = cpx<T>{(v3.im - v3.re) * r, -(v3.re + v3.im) * r};  // * (-1 - i)/sqrt2
    dft4v(u0, u1, u2, u3);
    dft4v(v0, v1, v2, v3);
    x[0] = u0; x[2] = u1; x[4] = u2; x[6] = u3;
    x[1] = v0; x[3] = v1; x[5] = v2; x[7] = v3;
}

// radix 16 as 4 x 4: DFT4 over m of x_{j+4m}, twiddle W16^(j q), DFT4 over j.
template <typename T> FD void dft16(cpx<T>* x)
{
    const T c = (T)K_COS_PI_8, s = (T)K_SIN_PI_8, r = (T)K_SQRT1_2;
    cpx<T> y[16];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        cpx<T> a = x[j], b = x[j + 4], cc = x[j + 8], d = x[j + 12];
        dft4v(a, b, cc, d);
        y[4 * j + 0] = a; y[4 * j + 1] = b; y[4 * j + 2] = cc; y[4 * j + 3] = d;
    }
    // twiddles W16^(j q) for j, q in 1..3 (exponents 1, 2, 3, 2, 4, 6, 3, 6, 9)
    y[5] = cmul(y[5], cpx<T>{c, -s});    // e = 1
    y[6] = cpx<T>{(y[6].re + y[6].im) * r, (y[6].im - y[6].re) * r};  // e = 2
    y[7] = cmul(y[7], cpx<T>{s, -c});    // e = 3
    y[9] = cpx<T>{(y[9].re + y[9].im) * r, (y[9].im - y[9].re) * r};  // e = 2
    y[10] = mul_negi(y[10]);             // e = 4
    y[11] = cpx<T>{(y[11].im - y[11].re) * r, -(y[11].re + y[11].im) * r};  // e = 6
    y[13] = cmul(y[13], cpx<T>{s, -c});  // e = 3
    y[14] = cpx<T>{(y[14].im - y[14].re) * r, -(y[14].re + y[14].im) * r};  // e = 6
    y[15] = cmul(y[15], cpx<T>{-c, s});  // e = 9
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        cpx<T> a = y[q], b = y[4 + q], cc = y[8 + q], d = y[12 + q];
        dft4v(a, b, cc, d);
        x[q] = a; x[q + 4] = b; x[q + 8] = cc; x[q + 12] = d;
    }
}

// radix 15 by the prime-factor map (3 and 5 are coprime): with the inputs
// indexed n = (5 n1 + 3 n2) mod 15 and the outputs k = (10 k1 + 6 k2) mod 15,
// W15^(nk) = W3^(n1 k1) W5^(n2 k2), so the DFT is five DFT3s over n1 followed
// by three DFT5s over n2, with no twiddles in between.
template <typename T> FD void dft15(cpx<T>* x)
{
    cpx<T> a[5][3];
#pragma unroll
    for (int n2 = 0; n2 < 5; ++n2)
#pragma unroll
        for (int n1 = 0; n1 < 3; ++n1) a[n2][n1] = x[(5 * n1 + 3 * n2) % 15];
#pragma unroll
    for (int n2 = 0; n2 < 5; ++n2) dft3(a[n2]);
    cpx<T> b[3][5];
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1)
#pragma unroll
        for (int n2 = 0; n2 < 5; ++n2) b[k1][n2] = a[n2][k1];
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) dft5(b[k1]);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 5; ++k2) x[(10 * k1 + 6 * k2) % 15] = b[k1][k2];
}

// ---------------------------------------------------------------- odd primes
// cos and sin of 2 pi m / P for the generic prime radix, evaluated at compile
// time in long double by their Taylor series (the argument is first reduced
// to [0, pi/2] by symmetry) and rounded once to the kernel's precision.
constexpr long double kPiL = 3.14159265358979323846264338327950288L;

constexpr long double taylor_sin(long double x)
{
    long double term = x, sum = x;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2 * k) * (2 * k + 1));
        sum += term;
    }
    return sum;
}

constexpr long double taylor_cos(long double x)
{
    long double term = 1, sum = 1;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2 * k - 1) * (2 * k));
        sum += term;
    }
    return sum;
}

// cos(2 pi m / P) and sin(2 pi m / P), 0 < m < P.
constexpr long double cos_2pi(int m, int P)
{
    const long double x = 2 * kPiL * m / P;  // in [0, 2 pi)
    if (x > kPiL) return cos_2pi(P - m, P);  // cos is even about pi
    return x <= kPiL / 2 ? taylor_cos(x) : -taylor_cos(kPiL - x);
}

constexpr long double sin_2pi(int m, int P)
{
    const long double x = 2 * kPiL * m / P;
    if (x > kPiL) return -sin_2pi(P - m, P);
    return x <= kPiL / 2 ? taylor_sin(x) : taylor_sin(kPiL - x);
}

// The length-P DFT of an odd prime P from the mirrored pairs t_j = x_j +
// x_(P-j), d_j = x_j - x_(P-j), j = 1..(P-1)/2:
//   X_k = x_0 + sum_j t_j cos(2 pi jk/P) - i sum_j d_j sin(2 pi jk/P)
// and X_(P-k) the same with +i, for k = 1..(P-1)/2 (jk reduced mod P).  The
// generic form of the radix-7 butterfly, O(P^2) real multiply-adds.
template <typename T, int P>
struct PrimeRoots {
    T c[P], s[P];
    constexpr PrimeRoots() : c(), s()
    {
        for (int m = 0; m < P; ++m) {
            c[m] = (T)cos_2pi(m, P);
            s[m] = (T)sin_2pi(m, P);
        }
    }
};

template <int P, typename T> FD void dft_prime(cpx<T>* v)
{
    constexpr int H = (P - 1) / 2;
    constexpr PrimeRoots<T, P> W{};  // folded at compile time
    cpx<T> t[H + 1], d[H + 1];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        t[j] = v[j] + v[P - j];
        d[j] = v[j] - v[P - j];
    }
    const cpx<T> x0 = v[0];
    cpx<T> s0 = x0;
#pragma unroll
    for (int j = 1; j <= H; ++j) s0 = s0 + t[j];
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        cpx<T> a = x0, b = {(T)0, (T)0};
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const T c = W.c[(j * k) % P], s = W.s[(j * k) % P];
            a = a + t[j] * c;
            b = b + d[j] * s;
        }
        v[k] = a + mul_negi(b);
        v[P - k] = a + mul_i(b);
    }
    v[0] = s0;
}

template <int R, typename T> FD void dft_radix(cpx<T>* v)
{
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 3) dft3(v);
    else if constexpr (R == 4) dft4(v);
    else if constexpr (R == 5) dft5(v);
    else if constexpr (R == 7) dft7(v);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 11 || R == 13) dft_prime<R>(v);
    else if constexpr (R == 15) dft15(v);
    else if constexpr (R == 16) dft16(v);
    else static_assert(R == 2, "unsupported radix");
}

// ------------------------------------------------------------ pass driver
//
// TPL threads cooperate on one line; pass p has N/R butterflies, thread tj
// takes butterflies tj, tj + TPL, ... (the last may be masked).  TPL defaults
// to N / (largest radix), one butterfly per thread in the widest pass; a
// smaller TPL gives each thread more butterflies, so more lines fit in a
// workgroup.  Between passes the outputs go through LDS: either as complex
// values, or (SPLIT) real parts first and imaginary parts second through a
// real-valued buffer of half the size.

template <int N, int TPL_, int P, int ORD = 0>
struct PassInfo {
    static constexpr RadixPlan PL = radix_plan(N, ORD);
    static constexpr int R = PL.r[P];
    static constexpr int BF = N / R;             // butterflies in this pass
    static constexpr int NS = radix_ns(PL, P);   // sub-transform length before it
    static constexpr int TPL = TPL_;
    static constexpr int NB = (BF + TPL - 1) / TPL;  // butterflies per thread
    static constexpr bool FULL = (BF % TPL) == 0;
    static constexpr int TWSTEP = N / (NS * R);
    static constexpr bool LAST = (P + 1 == PL.np);
};

template <int N, int TPL, int ORD = 0>
constexpr int driver_ept()
{
    constexpr RadixPlan PL = radix_plan(N, ORD);
    int e = 1;
    for (int i = 0; i < PL.np; ++i) {
        const int bf = N / PL.r[i];
        const int nb = (bf + TPL - 1) / TPL;
        e = nb * PL.r[i] > e ? nb * PL.r[i] : e;
    }
    return e;
}

// LDS view of one line: element e sits at base[e * es + (e >> 3) * pad].
// The optional pad (one slot per eight elements) breaks the power-of-two
// strides of the Stockham writes on contiguous lines across LDS banks.
template <typename U>
struct LdsView {
    U* base;
    int es;
    int pad;
    FD U& operator[](int e) const { return base[e * es + (e >> 3) * pad]; }
};

// Pass-0 inputs through the loader.
template <typename T, int N, int TPL, int ORD, class Load>
FD void load_first(cpx<T>* v, int tj, Load& load)
{
    using PI = PassInfo<N, TPL, 0, ORD>;
#pragma unroll
    for (int i = 0; i < PI::NB; ++i) {
        const int j = tj + i * TPL;
        if (PI::FULL || j < PI::BF) {
#pragma unroll
            for (int r = 0; r < PI::R; ++r) v[i * PI::R + r] = load(j + r * PI::BF);
        }
    }
}

// Twiddles and the radix-R DFTs of pass P, in registers.  twl is the
// per-pass twiddle table staged in LDS (layout in fft_lengths.hpp): the roots
// of butterfly k are R contiguous entries, so they load as wide LDS reads.
template <typename T, int N, int TPL, int P, int ORD>
FD void compute_pass(cpx<T>* v, int tj, const cpx<T>* twl)
{
    using PI = PassInfo<N, TPL, P, ORD>;
    constexpr int R = PI::R;
#pragma unroll
    for (int i = 0; i < PI::NB; ++i) {
        const int j = tj + i * TPL;
        if (PI::FULL || j < PI::BF) {
            if constexpr (PI::NS > 1) {
                const cpx<T>* w = twl + pass_table_offset(PI::PL, P) + (j % PI::NS) * R;
#pragma unroll
                for (int r = 1; r < R; ++r) v[i * R + r] = cmul(v[i * R + r], w[r]);
            }
            dft_radix<R>(v + i * R);
        }
    }
}

// Copy the per-pass twiddle table of the length-N kernel from global memory
// into LDS (all threads of the workgroup; visible after the next barrier).
template <typename T, int N, int ORD = 0>
FD void stage_pass_twiddles(cpx<T>* twl, const cpx<T>* __restrict__ twp, int t, int nthreads)
{
    constexpr int S = pass_table_size(radix_plan(N, ORD));
    for (int i = t; i < S; i += nthreads) twl[i] = twp[i];
}

template <typename T, int N, int ORD = 0>
constexpr size_t pass_table_bytes()
{
    return (size_t)pass_table_size(radix_plan(N, ORD)) * sizeof(cpx<T>);
}

// Bytes of a kernel's LDS data region rounded up so the twiddle table that
// follows it is 16-byte aligned.
__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Visit every output of pass P: f(register index, output element).
template <int N, int TPL, int P, int ORD, class F>
FD void for_outputs(int tj, F&& f)
{
    using PI = PassInfo<N, TPL, P, ORD>;
#pragma unroll
    for (int i = 0; i < PI::NB; ++i) {
        const int j = tj + i * TPL;
        if (PI::FULL || j < PI::BF) {
            const int k = j % PI::NS;
            const int o = (j / PI::NS) * PI::NS * PI::R + k;
#pragma unroll
            for (int r = 0; r < PI::R; ++r) f(i * PI::R + r, o + r * PI::NS);
        }
    }
}

// Visit every input of pass P: f(register index, input element).
template <int N, int TPL, int P, int ORD, class F>
FD void for_inputs(int tj, F&& f)
{
    using PI = PassInfo<N, TPL, P, ORD>;
#pragma unroll
    for (int i = 0; i < PI::NB; ++i) {
        const int j = tj + i * TPL;
        if (PI::FULL || j < PI::BF) {
#pragma unroll
            for (int r = 0; r < PI::R; ++r) f(i * PI::R + r, j + r * PI::BF);
        }
    }
}

// Outputs of pass P -> LDS -> inputs of pass P+1.  LEAD: a barrier is needed
// first because other threads may still read this LDS.
template <typename T, int N, int TPL, int P, bool SPLIT, bool LEAD, int ORD>
FD void exchange(cpx<T>* v, int tj, const LdsView<cpx<T>>& L, const LdsView<T>& Ls)
{
    if constexpr (!SPLIT) {
        if constexpr (LEAD) __syncthreads();
        for_outputs<N, TPL, P, ORD>(tj, [&](int q, int e) { L[e] = v[q]; });
        __syncthreads();
        for_inputs<N, TPL, P + 1, ORD>(tj, [&](int q, int e) { v[q] = L[e]; });
    } else {
        if constexpr (LEAD) __syncthreads();
        for_outputs<N, TPL, P, ORD>(tj, [&](int q, int e) { Ls[e] = v[q].re; });
        __syncthreads();
        for_inputs<N, TPL, P + 1, ORD>(tj, [&](int q, int e) { v[q].re = Ls[e]; });
        __syncthreads();
        for_outputs<N, TPL, P, ORD>(tj, [&](int q, int e) { Ls[e] = v[q].im; });
        __syncthreads();
        for_inputs<N, TPL, P + 1, ORD>(tj, [&](int q, int e) { v[q].im = Ls[e]; });
    }
}

template <typename T, int N, int TPL, int P, bool SPLIT, bool SRC_LDS, bool DST_LDS, int ORD, class Store>
FD void passes_from(cpx<T>* v, int tj, const cpx<T>* twl, const LdsView<cpx<T>>& L,
                    const LdsView<T>& Ls, Store& store)
{
    compute_pass<T, N, TPL, P, ORD>(v, tj, twl);
    if constexpr (PassInfo<N, TPL, P, ORD>::LAST) {
        if constexpr (DST_LDS && (P > 0 || SRC_LDS)) __syncthreads();
        for_outputs<N, TPL, P, ORD>(tj, [&](int q, int e) { store(e, v[q]); });
    } else {
        exchange<T, N, TPL, P, SPLIT, (P > 0 || SRC_LDS), ORD>(v, tj, L, Ls);
        passes_from<T, N, TPL, P + 1, SPLIT, SRC_LDS, DST_LDS, ORD>(v, tj, twl, L, Ls, store);
    }
}

// Full length-N forward FFT of one line by TPL cooperating threads (thread
// index tj < TPL), twiddles from the LDS table twl (staged beforehand).  SRC_LDS: the loader reads this workgroup's LDS, so no
// LDS write may happen before every thread has loaded.  DST_LDS: the storer
// writes LDS, so no store may happen before every thread has read its
// inputs.  The loader is called for pass-0 inputs, the storer for the final
// outputs (natural order).  For N == 1 it is a copy.  ORD selects the pass
// order of the radices (radix_plan(N, ORD)); twl must hold that order's table.
template <typename T, int N, int TPL = radix_plan(N).tpl, bool SPLIT = false, bool SRC_LDS = false,
          bool DST_LDS = false, int ORD = 0, class Load, class Store>
FD void fft_line(const LdsView<cpx<T>>& L, const LdsView<T>& Ls, int tj, const cpx<T>* twl, Load& load,
                 Store& store)
{
    if constexpr (N == 1) {
        if (tj == 0) store(0, load(0));  // one slot per line, touched by one thread
    } else {
        cpx<T> v[driver_ept<N, TPL, ORD>()];
        load_first<T, N, TPL, ORD>(v, tj, load);
        passes_from<T, N, TPL, 0, SPLIT, SRC_LDS, DST_LDS, ORD>(v, tj, twl, L, Ls, store);
    }
}

// ------------------------------------------------------------ tile lookup

// Workgroup coordinates within its tile and the tile's grid.
struct TileCoord {
    int64_t bx, by, gx, gy;
};

// A launch of one tile uses blockIdx and gridDim.  A grouped launch (a.tiles
// set, a 1D grid) reserves gmax workgroups per tile: workgroup w belongs to
// tile w / gmax, whose entry replaces the per-tile fields of `a`; workgroups
// past the tile's own grid have no work (false: the whole workgroup returns
// before any barrier).
template <typename Args>
FD bool tile_coord(Args& a, TileCoord& c)
{
    if (a.tiles == nullptr) {
        c.bx = blockIdx.x;
        c.by = blockIdx.y;
        c.gx = gridDim.x;
        c.gy = gridDim.y;
        return true;
    }
    // 32-bit index arithmetic: a grid's workgroup counts fit in 32 bits (and
    // a 64-bit division here costs the kernel a scratch stack frame)
    const uint32_t w = blockIdx.x, gmax = (uint32_t)a.gmax, nt = (uint32_t)a.ntiles;
    uint32_t t, local;
    if (nt > 0) {  // runs of nt tiles, each run's workgroups interleaved
        const uint32_t span = nt * gmax, run = w / span, r = w - run * span;
        local = r / nt;
        t = run * nt + (r - local * nt);
    } else {
        t = w / gmax;
        local = w - t * gmax;
    }
    const auto& e = a.tiles[t];
    const uint32_t gx = (uint32_t)e.gx;
    if (local >= gx * (uint32_t)e.gy) return false;
    if (e.in) a.in = e.in;  // else the launch's buffers (the tiles of one transform)
    if (e.out) a.out = e.out;
    a.off = e.off;
    a.off_o = e.off_o;
    a.A = e.A;
    a.B = e.B;
    a.kx0 = e.kx0;
    a.ky0 = e.ky0;
    c.gx = e.gx;
    c.gy = e.gy;
    const uint32_t by = local / gx;
    c.by = by;
    c.bx = local - by * gx;
    return true;
}

}  // namespace fft3d
