/*
 * FP64 CPU oracle for the pencil 3D FFT.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU library never links, calls or
 * includes anything from here, and nothing here is taken from the GPU library:
 * the two share no kernels, headers, tables or helpers.
 *
 * What is computed (paper, Sec. III-A, the displayed 3D DFT definition):
 *
 *   X[kx,ky,kz] = sum_{x,y,z} A[x,y,z] * exp(-2*pi*i*(kx*x/Nx + ky*y/Ny + kz*z/Nz))
 *
 * A fast transform reaches exactly this result up to rounding, so the oracle is
 * that definition: once as a literal triple sum (oracle_brute3d,
 * oracle_dft3d_points) and once as three passes of 1D DFTs, one per axis,
 * because the 3D sum is a tensor product of three 1D sums (same section: the
 * 3D transform is evaluated as 1D transforms along x, then y, then z).  Each 1D
 * DFT is a textbook recursive decimation-in-time split on the smallest prime
 * factor, with a plain O(p^2) combine for any prime p.  All arithmetic is
 * double; unit roots are built in long double and rounded once.
 *
 * Array layout: element (x,y,z) sits at x + Nx*(y + Ny*z) (x fastest, the
 * contiguous dimension of the stage-1 layout, Sec. IV-A).  Complex values are
 * interleaved (re, im) doubles.
 *
 * Readings of points the paper leaves open:
 *  - inverse = exponent sign +1 and scale 1/N; "backward" = sign +1 unscaled
 *    (the adjoint of the forward).  Inverse stage order is z, y, x (Sec. IV-A,
 *    inverse mirrors the forward); for the exact DFT the order does not matter.
 *  - real-to-complex keeps kx = 0..Nx/2 of the full forward DFT (Sec. V-B,
 *    Hermitian symmetry).  complex-to-real extends each x-line Hermitian-wise,
 *    ignoring the imaginary parts of the kx = 0 and kx = Nx/2 bins, after the
 *    inverse along z and y.
 *  - Poisson multiplier (periodic box of length 2*pi): M(k) = -1/|k|^2 with
 *    integer wavenumbers k_j = j for j <= n/2 and j - n above, M(0) = 0.
 *
 * Real-to-real transforms (DCT-II/III, DST-II/III) and the transforms and
 * Poisson solve of the (Periodic, Periodic, Bounded) topology are below,
 * with their own readings.
 *
 * Parity status: every exported function is pinned by the CPU tests against
 * closed forms, invariants, brute force, numpy.fft and scipy.fft's DCT/DST;
 * none is unpinned.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex dcplx;

/* ---------------------------------------------------------------- roots */

/* cos and sin of 2*pi*j/n in long double.  The angle is first reduced to a
 * quadrant with integer arithmetic, then to [0, pi/4] by the complementary
 * angle, so multiples of pi/2 come out exactly (0 and +-1). */
static void unit_root(long j, long n, long double *c, long double *s)
{
    const long double half_pi = 1.570796326794896619231321691639751442L;
    j %= n;
    if (j < 0) j += n;
    long q = (4 * j) / n;          /* quadrant 0..3 */
    long r = 4 * j - q * n;        /* angle within quadrant = (pi/2) * r / n */
    long double cq, sq;
    if (2 * r <= n) {
        long double t = half_pi * (long double)r / (long double)n;
        cq = cosl(t);
        sq = sinl(t);
    } else {
        long double t = half_pi * (long double)(n - r) / (long double)n;
        cq = sinl(t);
        sq = cosl(t);
    }
    switch (q) {
    case 0: *c = cq;  *s = sq;  break;
    case 1: *c = -sq; *s = cq;  break;
    case 2: *c = -cq; *s = -sq; break;
    default: *c = sq; *s = -cq; break;
    }
}

/* w[j] = exp(sign * 2*pi*i * j / n), j = 0..n-1 */
static dcplx *make_roots(long n, int sign)
{
    dcplx *w = (dcplx *)malloc(sizeof(dcplx) * (size_t)n);
    if (!w) return NULL;
    for (long j = 0; j < n; j++) {
        long double c, s;
        unit_root(j, n, &c, &s);
        w[j] = (double)c + I * (double)(sign < 0 ? -s : s);
    }
    return w;
}

static long smallest_prime_factor(long n)
{
    if (n % 2 == 0) return 2;
    for (long p = 3; p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/* ------------------------------------------------------------ 1D DFT */

/* X[k] = sum_j x[j*s] * W^(j*k) for k < n, where W = w[N/n] is the n-th root
 * drawn from the table w of N-th roots (n divides N).
 *
 * Decimation in time on the smallest prime factor p of n (m = n/p): the p
 * subsequences x[r], x[r+p], ... have length-m DFTs Y_r, and
 *   X[k + q*m] = sum_r W^(r*(k + q*m)) * Y_r[k],   k < m, q < p.
 * tmp holds at least 2n entries; this level keeps its Y_r in tmp[0..n) and
 * hands tmp+n to the level below. */
static void dft_rec(long n, const dcplx *x, long s, dcplx *X,
                    const dcplx *w, long N, dcplx *tmp)
{
    if (n == 1) {
        X[0] = x[0];
        return;
    }
    long p = smallest_prime_factor(n);
    long m = n / p;
    dcplx *Y = tmp;
    for (long r = 0; r < p; r++)
        dft_rec(m, x + r * s, s * p, Y + r * m, w, N, tmp + n);
    long step = N / n;
    for (long q = 0; q < p; q++) {
        for (long k = 0; k < m; k++) {
            long kk = k + q * m;
            dcplx acc = 0;
            for (long r = 0; r < p; r++)
                acc += w[((r * kk) % n) * step] * Y[r * m + k];
            X[kk] = acc;
        }
    }
}

/* One 1D DFT of a contiguous line; sign -1 forward, +1 conjugate exponent. */
int oracle_dft1d(long n, const double *in, double *out, int sign)
{
    if (n < 1 || !in || !out) return -1;
    dcplx *w = make_roots(n, sign);
    dcplx *tmp = (dcplx *)malloc(sizeof(dcplx) * (size_t)(2 * n));
    dcplx *res = (dcplx *)malloc(sizeof(dcplx) * (size_t)n);
    if (!w || !tmp || !res) {
        free(w); free(tmp); free(res);
        return -2;
    }
    dft_rec(n, (const dcplx *)in, 1, res, w, n, tmp);
    memcpy(out, res, sizeof(dcplx) * (size_t)n);
    free(w); free(tmp); free(res);
    return 0;
}

/* Apply the length-len 1D DFT along one axis of a 3D array in place.
 * axis 0 = x (stride 1), 1 = y (stride nx), 2 = z (stride nx*ny). */
static int dft_axis(dcplx *a, long nx, long ny, long nz, int axis, int sign)
{
    long len, stride, n1, n2, s1, s2;
    if (axis == 0) {
        len = nx; stride = 1;       n1 = ny; s1 = nx; n2 = nz; s2 = nx * ny;
    } else if (axis == 1) {
        len = ny; stride = nx;      n1 = nx; s1 = 1;  n2 = nz; s2 = nx * ny;
    } else {
        len = nz; stride = nx * ny; n1 = nx; s1 = 1;  n2 = ny; s2 = nx;
    }
    dcplx *w = make_roots(len, sign);
    if (!w) return -2;
    int err = 0;
#pragma omp parallel
    {
        dcplx *line = (dcplx *)malloc(sizeof(dcplx) * (size_t)len);
        dcplx *res = (dcplx *)malloc(sizeof(dcplx) * (size_t)len);
        dcplx *tmp = (dcplx *)malloc(sizeof(dcplx) * (size_t)(2 * len));
        int ok = line && res && tmp;
        if (!ok) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (long l = 0; l < n1 * n2; l++) {
            if (!ok) continue;
            long i1 = l % n1, i2 = l / n1;
            dcplx *base = a + i1 * s1 + i2 * s2;
            for (long j = 0; j < len; j++) line[j] = base[j * stride];
            dft_rec(len, line, 1, res, w, len, tmp);
            for (long j = 0; j < len; j++) base[j * stride] = res[j];
        }
        free(line); free(res); free(tmp);
    }
    free(w);
    return err;
}

/* ------------------------------------------------------------ 3D C2C */

/* sign -1: forward (unscaled).  sign +1: scale != 0 gives the inverse (1/N),
 * scale == 0 the unscaled backward.  Forward runs x, y, z; sign +1 runs z, y,
 * x (the mirrored order). */
int oracle_c2c3d(long nx, long ny, long nz, const double *in, double *out,
                 int sign, int scale)
{
    if (nx < 1 || ny < 1 || nz < 1 || !in || !out) return -1;
    long n = nx * ny * nz;
    dcplx *a = (dcplx *)out;
    if ((const void *)in != (void *)out)
        memmove(a, in, sizeof(dcplx) * (size_t)n);
    int err = 0;
    if (sign < 0) {
        for (int ax = 0; ax < 3 && !err; ax++) err = dft_axis(a, nx, ny, nz, ax, -1);
    } else {
        for (int ax = 2; ax >= 0 && !err; ax--) err = dft_axis(a, nx, ny, nz, ax, +1);
        if (!err && scale) {
            double f = 1.0 / (double)n;
            for (long i = 0; i < n; i++) a[i] *= f;
        }
    }
    return err;
}

/* ------------------------------------------------------- brute force */

/* The literal triple sum of the 3D DFT definition, O(N^2).  Each phase is the
 * product of three table entries indexed by (k*j mod n) per axis. */
int oracle_brute3d(long nx, long ny, long nz, const double *in, double *out,
                   int sign)
{
    if (nx < 1 || ny < 1 || nz < 1 || !in || !out) return -1;
    dcplx *wx = make_roots(nx, sign), *wy = make_roots(ny, sign), *wz = make_roots(nz, sign);
    if (!wx || !wy || !wz) {
        free(wx); free(wy); free(wz);
        return -2;
    }
    const dcplx *a = (const dcplx *)in;
    dcplx *X = (dcplx *)out;
    long n = nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < n; k++) {
        long kx = k % nx, ky = (k / nx) % ny, kz = k / (nx * ny);
        dcplx acc = 0;
        for (long z = 0; z < nz; z++)
            for (long y = 0; y < ny; y++)
                for (long x = 0; x < nx; x++)
                    acc += a[x + nx * (y + ny * z)] * wx[(kx * x) % nx] *
                           wy[(ky * y) % ny] * wz[(kz * z) % nz];
        X[k] = acc;
    }
    free(wx); free(wy); free(wz);
    return 0;
}

/* Selected outputs of the 3D DFT by the definition, each an O(N) sum.
 * k holds npts triples (kx, ky, kz).  If real_input is nonzero, `in` holds N
 * doubles (a real field); otherwise N interleaved complex values.  The sum is
 * taken z-outer so each inner x-sum is contiguous. */
int oracle_dft3d_points(long nx, long ny, long nz, const double *in,
                        int real_input, long npts, const long *k, double *out,
                        int sign)
{
    if (nx < 1 || ny < 1 || nz < 1 || !in || !out || npts < 0) return -1;
    dcplx *wx = make_roots(nx, sign), *wy = make_roots(ny, sign), *wz = make_roots(nz, sign);
    if (!wx || !wy || !wz) {
        free(wx); free(wy); free(wz);
        return -2;
    }
    for (long p = 0; p < npts; p++) {
        long kx = k[3 * p], ky = k[3 * p + 1], kz = k[3 * p + 2];
        if (kx < 0 || ky < 0 || kz < 0 || kx >= nx || ky >= ny || kz >= nz) {
            free(wx); free(wy); free(wz);
            return -1;
        }
        double sre = 0, sim = 0;
#pragma omp parallel for reduction(+ : sre, sim) schedule(static)
        for (long z = 0; z < nz; z++) {
            dcplx accz = 0;
            for (long y = 0; y < ny; y++) {
                dcplx accy = 0;
                long row = nx * (y + ny * z);
                if (real_input) {
                    for (long x = 0; x < nx; x++) accy += in[row + x] * wx[(kx * x) % nx];
                } else {
                    const dcplx *a = (const dcplx *)in;
                    for (long x = 0; x < nx; x++) accy += a[row + x] * wx[(kx * x) % nx];
                }
                accz += accy * wy[(ky * y) % ny];
            }
            dcplx t = accz * wz[(kz * z) % nz];
            sre += creal(t);
            sim += cimag(t);
        }
        out[2 * p] = sre;
        out[2 * p + 1] = sim;
    }
    free(wx); free(wy); free(wz);
    return 0;
}

/* ------------------------------------------------------------ R2C / C2R */

/* Real input (N doubles) -> kx = 0..Nx/2 of its forward 3D DFT, stored as an
 * (Nx/2+1) x Ny x Nz complex array (x fastest). */
int oracle_r2c3d(long nx, long ny, long nz, const double *in, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !in || !out) return -1;
    long n = nx * ny * nz, nh = nx / 2 + 1;
    dcplx *full = (dcplx *)malloc(sizeof(dcplx) * (size_t)n);
    if (!full) return -2;
    for (long i = 0; i < n; i++) full[i] = in[i];
    int err = 0;
    for (int ax = 0; ax < 3 && !err; ax++) err = dft_axis(full, nx, ny, nz, ax, -1);
    if (!err) {
        dcplx *X = (dcplx *)out;
        for (long zy = 0; zy < ny * nz; zy++)
            for (long kx = 0; kx < nh; kx++) X[kx + nh * zy] = full[kx + nx * zy];
    }
    free(full);
    return err;
}

/* Half spectrum (Nx/2+1) x Ny x Nz -> real Nx x Ny x Nz.  First the sign +1
 * DFT along z and then y on the half spectrum; then every x-line is extended
 * to the full length by H[Nx-k] = conj(H[k]) (with the imaginary parts of the
 * k = 0 bin and, for even Nx, the k = Nx/2 bin dropped), transformed with
 * sign +1 along x, and its real part kept.  scale != 0 multiplies by 1/N (the
 * inverse of oracle_r2c3d); scale == 0 is unscaled. */
int oracle_c2r3d(long nx, long ny, long nz, const double *in, double *out,
                 int scale)
{
    if (nx < 1 || ny < 1 || nz < 1 || !in || !out) return -1;
    long nh = nx / 2 + 1, nhalf = nh * ny * nz;
    dcplx *h = (dcplx *)malloc(sizeof(dcplx) * (size_t)nhalf);
    if (!h) return -2;
    memcpy(h, in, sizeof(dcplx) * (size_t)nhalf);
    int err = dft_axis(h, nh, ny, nz, 2, +1);
    if (!err) err = dft_axis(h, nh, ny, nz, 1, +1);
    if (err) {
        free(h);
        return err;
    }
    dcplx *w = make_roots(nx, +1);
    if (!w) {
        free(h);
        return -2;
    }
    double f = scale ? 1.0 / ((double)nx * (double)ny * (double)nz) : 1.0;
#pragma omp parallel
    {
        dcplx *line = (dcplx *)malloc(sizeof(dcplx) * (size_t)nx);
        dcplx *res = (dcplx *)malloc(sizeof(dcplx) * (size_t)nx);
        dcplx *tmp = (dcplx *)malloc(sizeof(dcplx) * (size_t)(2 * nx));
        int ok = line && res && tmp;
        if (!ok) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (long zy = 0; zy < ny * nz; zy++) {
            if (!ok) continue;
            const dcplx *src = h + nh * zy;
            for (long kx = 0; kx < nh; kx++) line[kx] = src[kx];
            line[0] = creal(line[0]);
            if (nx % 2 == 0) line[nx / 2] = creal(line[nx / 2]);
            for (long kx = nh; kx < nx; kx++) line[kx] = conj(line[nx - kx]);
            dft_rec(nx, line, 1, res, w, nx, tmp);
            for (long x = 0; x < nx; x++) out[x + nx * zy] = creal(res[x]) * f;
        }
        free(line); free(res); free(tmp);
    }
    free(w);
    free(h);
    return err;
}

/* ------------------------------------------------------------ Poisson */

static double wavenumber(long j, long n) { return (double)(2 * j <= n ? j : j - n); }

/* phi = c2r( M .* r2c(f) ) / N with M(k) = -1/|k|^2, M(0) = 0, integer
 * wavenumbers (periodic box of side 2*pi).  This is the spectral Poisson solve
 * lap(phi) = f for a zero-mean f, written as the three steps it is made of. */
int oracle_poisson3d(long nx, long ny, long nz, const double *f, double *phi)
{
    if (nx < 1 || ny < 1 || nz < 1 || !f || !phi) return -1;
    long nh = nx / 2 + 1;
    dcplx *H = (dcplx *)malloc(sizeof(dcplx) * (size_t)(nh * ny * nz));
    if (!H) return -2;
    int err = oracle_r2c3d(nx, ny, nz, f, (double *)H);
    if (!err) {
        for (long kz = 0; kz < nz; kz++)
            for (long ky = 0; ky < ny; ky++)
                for (long kx = 0; kx < nh; kx++) {
                    double a = wavenumber(kx, nx), b = wavenumber(ky, ny), c = wavenumber(kz, nz);
                    double k2 = a * a + b * b + c * c;
                    double m = (k2 == 0.0) ? 0.0 : -1.0 / k2;
                    H[kx + nh * (ky + ny * kz)] *= m;
                }
        err = oracle_c2r3d(nx, ny, nz, (const double *)H, phi, 1);
    }
    free(H);
    return err;
}

/* ------------------------------------------------------- R2R along z */

/* Real-to-real transforms of one real sequence of length n (the DCT and DST
 * that the paper's plan supports besides C2C and R2C, Sec. V-B), written as
 * the plain O(n^2) sums, in the unnormalised convention of FFTW's REDFT and
 * RODFT kinds:
 *   kind 0, DCT-II : Y_k = 2 sum_{j<n} x_j cos(pi (j+1/2) k / n)
 *   kind 1, DCT-III: Y_k = x_0 + 2 sum_{0<j<n} x_j cos(pi j (k+1/2) / n)
 *   kind 2, DST-II : Y_k = 2 sum_{j<n} x_j sin(pi (j+1/2) (k+1) / n)
 *   kind 3, DST-III: Y_k = (-1)^k x_{n-1} + 2 sum_{j<n-1} x_j sin(pi (j+1) (k+1/2) / n)
 * Kinds 1 and 3 undo kinds 0 and 2 up to the factor 2n.  Every angle is an
 * integer multiple of 2 pi / (4n) and is taken from the long-double root
 * table of that order. */
static double r2r_term(long n, long j, long k, int kind, const long double *c4, const long double *s4)
{
    long m;
    switch (kind) {
    case 0: m = ((2 * j + 1) * k) % (4 * n); return (double)c4[m];
    case 1: m = (j * (2 * k + 1)) % (4 * n); return (double)c4[m];
    case 2: m = ((2 * j + 1) * (k + 1)) % (4 * n); return (double)s4[m];
    default: m = ((j + 1) * (2 * k + 1)) % (4 * n); return (double)s4[m];
    }
}

static int r2r_tables(long n, long double **c4, long double **s4)
{
    *c4 = (long double *)malloc(sizeof(long double) * (size_t)(4 * n));
    *s4 = (long double *)malloc(sizeof(long double) * (size_t)(4 * n));
    if (!*c4 || !*s4) {
        free(*c4); free(*s4);
        return -2;
    }
    for (long m = 0; m < 4 * n; m++) unit_root(m, 4 * n, &(*c4)[m], &(*s4)[m]);
    return 0;
}

/* out = kind(in) for one line; in and out are n doubles (need not differ). */
static void r2r_line(long n, const double *in, double *out, int kind, const long double *c4,
                     const long double *s4)
{
    for (long k = 0; k < n; k++) {
        double acc = 0.0;
        for (long j = 0; j < n; j++) {
            double w;
            if (kind == 1 && j == 0) w = 1.0;
            else if (kind == 3 && j == n - 1) w = (k % 2 == 0) ? 1.0 : -1.0;
            else w = 2.0 * r2r_term(n, j, k, kind, c4, s4);
            acc += w * in[j];
        }
        out[k] = acc;
    }
}

int oracle_r2r1d(long n, const double *in, double *out, int kind)
{
    if (n < 1 || !in || !out || kind < 0 || kind > 3) return -1;
    long double *c4, *s4;
    if (r2r_tables(n, &c4, &s4)) return -2;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!tmp) {
        free(c4); free(s4);
        return -2;
    }
    r2r_line(n, in, tmp, kind, c4, s4);
    memcpy(out, tmp, sizeof(double) * (size_t)n);
    free(tmp); free(c4); free(s4);
    return 0;
}

/* The R2R transform of `kind` along z of a complex (nxh x ny x nz) array, on
 * the real and the imaginary parts separately (the transform is real-linear),
 * times `scale`. */
static int r2r_axis_z(dcplx *a, long nxh, long ny, long nz, int kind, double scale)
{
    long double *c4, *s4;
    if (r2r_tables(nz, &c4, &s4)) return -2;
    int err = 0;
#pragma omp parallel
    {
        double *re = (double *)malloc(sizeof(double) * (size_t)nz);
        double *im = (double *)malloc(sizeof(double) * (size_t)nz);
        double *ro = (double *)malloc(sizeof(double) * (size_t)nz);
        double *io = (double *)malloc(sizeof(double) * (size_t)nz);
        int ok = re && im && ro && io;
        if (!ok) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (long l = 0; l < nxh * ny; l++) {
            if (!ok) continue;
            for (long z = 0; z < nz; z++) {
                re[z] = creal(a[l + nxh * ny * z]);
                im[z] = cimag(a[l + nxh * ny * z]);
            }
            r2r_line(nz, re, ro, kind, c4, s4);
            r2r_line(nz, im, io, kind, c4, s4);
            for (long z = 0; z < nz; z++) a[l + nxh * ny * z] = (ro[z] + I * io[z]) * scale;
        }
        free(re); free(im); free(ro); free(io);
    }
    free(c4); free(s4);
    return err;
}

/* Forward transform of the (Periodic, Periodic, Bounded) topology (the
 * Poisson solver case of Sec. VI-B): real f (Nx x Ny x Nz) -> its DFT along x
 * (kx = 0..Nx/2 kept, Hermitian symmetry) and y, then along the bounded z
 * axis the DCT-II (bc 0: homogeneous Neumann walls) or the DST-II (bc 1:
 * homogeneous Dirichlet walls), all unscaled; out is (Nx/2+1) x Ny x Nz
 * complex. */
int oracle_ppb_forward3d(long nx, long ny, long nz, const double *f, double *out, int bc)
{
    if (nx < 1 || ny < 1 || nz < 1 || !f || !out || bc < 0 || bc > 1) return -1;
    long n = nx * ny * nz, nh = nx / 2 + 1;
    dcplx *full = (dcplx *)malloc(sizeof(dcplx) * (size_t)n);
    if (!full) return -2;
    for (long i = 0; i < n; i++) full[i] = f[i];
    int err = dft_axis(full, nx, ny, nz, 0, -1);
    if (!err) err = dft_axis(full, nx, ny, nz, 1, -1);
    dcplx *H = (dcplx *)out;
    if (!err) {
        for (long zy = 0; zy < ny * nz; zy++)
            for (long kx = 0; kx < nh; kx++) H[kx + nh * zy] = full[kx + nx * zy];
        err = r2r_axis_z(H, nh, ny, nz, bc == 0 ? 0 : 2, 1.0);
    }
    free(full);
    return err;
}

/* Inverse of oracle_ppb_forward3d: along z the DCT-III (bc 0) or DST-III
 * (bc 1) divided by 2 Nz, then the inverse DFT along y (1/Ny) and the
 * Hermitian-extended inverse DFT of every x-line (1/Nx, real part kept; the
 * imaginary parts of the kx = 0 and kx = Nx/2 bins dropped as in
 * oracle_c2r3d). */
int oracle_ppb_inverse3d(long nx, long ny, long nz, const double *in, double *out, int bc)
{
    if (nx < 1 || ny < 1 || nz < 1 || !in || !out || bc < 0 || bc > 1) return -1;
    long nh = nx / 2 + 1, nhalf = nh * ny * nz;
    dcplx *h = (dcplx *)malloc(sizeof(dcplx) * (size_t)nhalf);
    if (!h) return -2;
    memcpy(h, in, sizeof(dcplx) * (size_t)nhalf);
    int err = r2r_axis_z(h, nh, ny, nz, bc == 0 ? 1 : 3, 1.0 / (2.0 * (double)nz));
    if (!err) err = dft_axis(h, nh, ny, nz, 1, +1);
    dcplx *w = err ? NULL : make_roots(nx, +1);
    if (!err && !w) err = -2;
    if (err) {
        free(h);
        return err;
    }
    const double f = 1.0 / ((double)nx * (double)ny);
#pragma omp parallel
    {
        dcplx *line = (dcplx *)malloc(sizeof(dcplx) * (size_t)nx);
        dcplx *res = (dcplx *)malloc(sizeof(dcplx) * (size_t)nx);
        dcplx *tmp = (dcplx *)malloc(sizeof(dcplx) * (size_t)(2 * nx));
        int ok = line && res && tmp;
        if (!ok) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (long zy = 0; zy < ny * nz; zy++) {
            if (!ok) continue;
            const dcplx *src = h + nh * zy;
            for (long kx = 0; kx < nh; kx++) line[kx] = src[kx];
            line[0] = creal(line[0]);
            if (nx % 2 == 0) line[nx / 2] = creal(line[nx / 2]);
            for (long kx = nh; kx < nx; kx++) line[kx] = conj(line[nx - kx]);
            dft_rec(nx, line, 1, res, w, nx, tmp);
            for (long x = 0; x < nx; x++) out[x + nx * zy] = creal(res[x]) * f;
        }
        free(line); free(res); free(tmp);
    }
    free(w);
    free(h);
    return err;
}

/* Spectral Poisson solve of the (Periodic, Periodic, Bounded) topology:
 * phi = ppb_inverse( M .* ppb_forward(f) ).  x and y are periodic of side
 * 2 pi (integer wavenumbers as in oracle_poisson3d); z is the interval
 * (0, pi) of Nz cells with values at the cell centres pi (j + 1/2) / Nz, whose
 * Neumann modes cos(k z) (bc 0, k = 0..Nz-1) and Dirichlet modes sin(k z)
 * (bc 1, k = 1..Nz) have integer wavenumbers.  M = -1/|k|^2, and 0 for the
 * all-zero wavenumber (Neumann only). */
int oracle_poisson_ppb3d(long nx, long ny, long nz, const double *f, double *phi, int bc)
{
    if (nx < 1 || ny < 1 || nz < 1 || !f || !phi || bc < 0 || bc > 1) return -1;
    long nh = nx / 2 + 1;
    dcplx *H = (dcplx *)malloc(sizeof(dcplx) * (size_t)(nh * ny * nz));
    if (!H) return -2;
    int err = oracle_ppb_forward3d(nx, ny, nz, f, (double *)H, bc);
    if (!err) {
        for (long kz = 0; kz < nz; kz++)
            for (long ky = 0; ky < ny; ky++)
                for (long kx = 0; kx < nh; kx++) {
                    double a = wavenumber(kx, nx), b = wavenumber(ky, ny);
                    double c = (double)(bc == 0 ? kz : kz + 1);
                    double k2 = a * a + b * b + c * c;
                    double m = (k2 == 0.0) ? 0.0 : -1.0 / k2;
                    H[kx + nh * (ky + ny * kz)] *= m;
                }
        err = oracle_ppb_inverse3d(nx, ny, nz, (const double *)H, phi, bc);
    }
    free(H);
    return err;
}

/* Host threads OpenMP will use for the calls above. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
