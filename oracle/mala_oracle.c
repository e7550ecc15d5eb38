/*
 * FP64 CPU oracle for the MALA grid-inference path -- TEST INFRASTRUCTURE.
 *
 * This file is the plain, slow, obviously-correct reference that the GPU
 * library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes (arXiv:2411.19617, "MALA"):
 *  - neighbour sets of each grid point (Sec. 3.2.2, Eq. ionicdensity): every
 *    periodic image of every atom closer than the cutoff, self weight 1,
 *    element weight 1 (single species), smooth cosine cutoff function;
 *  - expansion coefficients u^j of the ionic density in hyperspherical
 *    harmonics U^j (Eq. SNAPExpansion), U^j taken as the spin-j irreducible
 *    representation of the SU(2) element fixed by the neighbour vector,
 *    written out from its defining polynomial (no recursion);
 *  - Clebsch-Gordan coefficients from the Racah closed form;
 *  - bispectrum components B(j1,j2,j) as the rotation-invariant triple
 *    products of u (Sec. 3.2.2, count of Eq. snap_dim);
 *  - the feed-forward network x_{l+1} = sigma(W_l x_l + b_l) (Sec. 2.4,
 *    Eq. ffnn) with input standardisation and an affine output transform;
 *  - DOS as the spatial sum of the LDOS times the volume element
 *    (Eq. DOS.from.ldos), energy integrals with Fermi-Dirac weights of a
 *    piecewise-linear DOS written through polylogarithms
 *    (Sec. 3.4, Eqs. ldosintegralsummation, fermidiracspecial), the Fermi
 *    level as the root of the electron-count equation
 *    (Eq. NumberElectrons_from_DOS) by bisection, the band energy
 *    (Eq. band.energy) and the density (Eq. density.from.ldos).
 *
 * All arithmetic is double precision.  Loops follow the definitions with no
 * blocking, symmetry folding or reordering.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_KB_EV 8.617333262e-5     /* Boltzmann constant, eV/K (CODATA 2018) */
#define OR_RFAC0 0.99363            /* theta0 = rfac0 * pi * r / rcut */
#define OR_TJMAX 14

typedef double complex cplx;

/* ------------------------------------------------------------ factorials */
static double fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= (double)i;
    return f;
}

static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    return fact(n) / (fact(k) * fact(n - k));
}

static cplx cpow_int(cplx z, int n)
{
    cplx r = 1.0;
    for (int i = 0; i < n; i++) r *= z;
    return r;
}

/* ------------------------------------------------------------ Clebsch-Gordan
 * <j1 m1 j2 m2 | j m> in the Condon-Shortley convention from the Racah
 * closed form.  All angular momenta are passed doubled (2j, 2m).          */
double oracle_cg(int j1, int m1, int j2, int m2, int j, int m)
{
    if (m1 + m2 != m) return 0.0;
    if (j < abs(j1 - j2) || j > j1 + j2 || ((j1 + j2 + j) & 1)) return 0.0;
    if (abs(m1) > j1 || abs(m2) > j2 || abs(m) > j) return 0.0;
    if (((j1 + m1) & 1) || ((j2 + m2) & 1) || ((j + m) & 1)) return 0.0;
    /* integer factorial arguments */
    int a = (j1 + j2 - j) / 2, b = (j1 - j2 + j) / 2, c = (-j1 + j2 + j) / 2;
    int d = (j1 + j2 + j) / 2 + 1;
    double pre = (j + 1.0) * fact(a) * fact(b) * fact(c) / fact(d);
    pre *= fact((j1 + m1) / 2) * fact((j1 - m1) / 2) * fact((j2 + m2) / 2) *
           fact((j2 - m2) / 2) * fact((j + m) / 2) * fact((j - m) / 2);
    double s = 0.0;
    for (int k = 0; k <= d; k++) {
        int f1 = a - k, f2 = (j1 - m1) / 2 - k, f3 = (j2 + m2) / 2 - k;
        int f4 = (j - j2 + m1) / 2 + k, f5 = (j - j1 - m2) / 2 + k;
        if (f1 < 0 || f2 < 0 || f3 < 0 || f4 < 0 || f5 < 0) continue;
        double t = 1.0 / (fact(k) * fact(f1) * fact(f2) * fact(f3) * fact(f4) * fact(f5));
        s += (k & 1) ? -t : t;
    }
    return sqrt(pre) * s;
}

/* ------------------------------------------------------------ geometry
 * Map a neighbour vector (relative to the grid point) to the Cayley-Klein
 * parameters of g = exp(-i theta0 n.sigma) = [[a, b], [-conj(b), conj(a)]],
 * theta0 = rfac0 * pi * r / rcut.  At r = 0 the element is the identity.  */
void oracle_cayley_klein(double dx, double dy, double dz, double rcut,
                         double *a_re, double *a_im, double *b_re, double *b_im)
{
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r == 0.0) {
        *a_re = 1.0; *a_im = 0.0; *b_re = 0.0; *b_im = 0.0;
        return;
    }
    double th = OR_RFAC0 * OR_PI * r / rcut;
    double nx = dx / r, ny = dy / r, nz = dz / r;
    double c = cos(th), s = sin(th);
    *a_re = c;
    *a_im = -nz * s;
    *b_re = -ny * s;
    *b_im = -nx * s;
}

double oracle_cutoff(double r, double rcut)
{
    if (r >= rcut) return 0.0;
    return 0.5 * (cos(OR_PI * r / rcut) + 1.0);
}

/* ------------------------------------------------------------ U^j
 * Spin-j irrep of g, doubled index J = 2j, rows ma = j + m and columns
 * mb = j + m' in 0..J: U[ma][mb] is the coefficient of xi^mb eta^(J-mb) in
 * (a xi - conj(b) eta)^ma (b xi + conj(a) eta)^(J-ma), times
 * sqrt(mb! (J-mb)! / (ma! (J-ma)!)).  out is (J+1)^2 complex, row-major.  */
void oracle_wigner_u(int J, double a_re, double a_im, double b_re, double b_im,
                     double *out /* [(J+1)^2][2] */)
{
    cplx a = a_re + I * a_im, b = b_re + I * b_im;
    cplx mbc = -conj(b), ac = conj(a);
    for (int ma = 0; ma <= J; ma++) {
        for (int mb = 0; mb <= J; mb++) {
            cplx coef = 0.0;
            for (int s = 0; s <= ma; s++) {
                int t = mb - s;                 /* power of xi from the second factor */
                if (t < 0 || t > J - ma) continue;
                coef += binom(ma, s) * binom(J - ma, t) * cpow_int(a, s) *
                        cpow_int(mbc, ma - s) * cpow_int(b, t) * cpow_int(ac, J - ma - t);
            }
            double norm = sqrt(fact(mb) * fact(J - mb) / (fact(ma) * fact(J - ma)));
            cplx v = coef * norm;
            out[2 * (ma * (J + 1) + mb)] = creal(v);
            out[2 * (ma * (J + 1) + mb) + 1] = cimag(v);
        }
    }
}

/* offset of level J inside the packed full-u array: sum_{J'<J} (J'+1)^2 */
static int u_off(int J)
{
    int o = 0;
    for (int k = 0; k < J; k++) o += (k + 1) * (k + 1);
    return o;
}

int oracle_u_size(int twojmax) { return u_off(twojmax + 1); }

/* u^J = I + sum_k fc(r_k) U^J(g_k) for J = 0..twojmax.  disp is [n][3]
 * (neighbour minus grid point).  Only neighbours with r < rcut count.     */
void oracle_ui(const double *disp, int n, double rcut, int twojmax, double *u /* [size][2] */)
{
    int size = u_off(twojmax + 1);
    memset(u, 0, sizeof(double) * 2 * size);
    for (int J = 0; J <= twojmax; J++)
        for (int ma = 0; ma <= J; ma++) u[2 * (u_off(J) + ma * (J + 1) + ma)] = 1.0;
    double *U = malloc(sizeof(double) * 2 * (twojmax + 1) * (twojmax + 1));
    for (int k = 0; k < n; k++) {
        double dx = disp[3 * k], dy = disp[3 * k + 1], dz = disp[3 * k + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r >= rcut) continue;
        double fc = oracle_cutoff(r, rcut);
        double ar, ai, br, bi;
        oracle_cayley_klein(dx, dy, dz, rcut, &ar, &ai, &br, &bi);
        for (int J = 0; J <= twojmax; J++) {
            oracle_wigner_u(J, ar, ai, br, bi, U);
            int o = u_off(J);
            for (int e = 0; e < (J + 1) * (J + 1); e++) {
                u[2 * (o + e)] += fc * U[2 * e];
                u[2 * (o + e) + 1] += fc * U[2 * e + 1];
            }
        }
    }
    free(U);
}

/* ------------------------------------------------------------ bispectrum */
int oracle_n_triples(int twojmax)
{
    int n = 0;
    for (int j1 = 0; j1 <= twojmax; j1++)
        for (int j2 = 0; j2 <= j1; j2++)
            for (int j = j1 - j2; j <= j1 + j2 && j <= twojmax; j += 2)
                if (j >= j1) n++;
    return n;
}

/* triples [n][3] in output order (doubled indices) */
void oracle_triples(int twojmax, int *out)
{
    int n = 0;
    for (int j1 = 0; j1 <= twojmax; j1++)
        for (int j2 = 0; j2 <= j1; j2++)
            for (int j = j1 - j2; j <= j1 + j2 && j <= twojmax; j += 2)
                if (j >= j1) {
                    out[3 * n] = j1; out[3 * n + 1] = j2; out[3 * n + 2] = j;
                    n++;
                }
}

static cplx uel(const double *u, int J, int ma, int mb)
{
    int e = u_off(J) + ma * (J + 1) + mb;
    return u[2 * e] + I * u[2 * e + 1];
}

/* B(j1,j2,j) = sum_{m,m'} conj(u^j_{m m'}) Z^j_{m m'}(j1,j2) with
 * Z^j_{m m'} = sum_{m1,m1'} C^{j m}_{j1 m1 j2 m-m1} C^{j m'}_{j1 m1' j2 m'-m1'}
 *              u^{j1}_{m1 m1'} u^{j2}_{m-m1, m'-m1'}.
 * Indices are doubled; m runs over -j..j in steps of 2 (doubled units).
 * Writes n_triples real parts to B and the largest |imag| to *max_imag.   */
void oracle_bispectrum(const double *u, int twojmax, double *B, double *max_imag)
{
    int nt = oracle_n_triples(twojmax);
    int *tr = malloc(sizeof(int) * 3 * nt);
    oracle_triples(twojmax, tr);
    double mi = 0.0;
    for (int t = 0; t < nt; t++) {
        int j1 = tr[3 * t], j2 = tr[3 * t + 1], j = tr[3 * t + 2];
        cplx sum = 0.0;
        for (int m = -j; m <= j; m += 2) {
            for (int mp = -j; mp <= j; mp += 2) {
                cplx z = 0.0;
                for (int m1 = -j1; m1 <= j1; m1 += 2) {
                    int m2 = m - m1;
                    if (m2 < -j2 || m2 > j2) continue;
                    double c1 = oracle_cg(j1, m1, j2, m2, j, m);
                    for (int m1p = -j1; m1p <= j1; m1p += 2) {
                        int m2p = mp - m1p;
                        if (m2p < -j2 || m2p > j2) continue;
                        double c2 = oracle_cg(j1, m1p, j2, m2p, j, mp);
                        z += c1 * c2 * uel(u, j1, (j1 + m1) / 2, (j1 + m1p) / 2) *
                             uel(u, j2, (j2 + m2) / 2, (j2 + m2p) / 2);
                    }
                }
                sum += conj(uel(u, j, (j + m) / 2, (j + mp) / 2)) * z;
            }
        }
        B[t] = creal(sum);
        if (fabs(cimag(sum)) > mi) mi = fabs(cimag(sum));
    }
    if (max_imag) *max_imag = mi;
    free(tr);
}

/* ------------------------------------------------------------ neighbours
 * Grid point p = (i, j, k), flat index p = (i*Ny + j)*Nz + k, position
 * (i Lx/Nx, j Ly/Ny, k Lz/Nz).  Neighbours: all periodic images R + n*L of
 * all atoms with |R + n*L - r_p| < rcut, found by brute force over a box of
 * image shifts that covers the cutoff sphere.                              */
static void grid_point(const int *N, const double *L, int64_t p, double *r)
{
    int64_t k = p % N[2], j = (p / N[2]) % N[1], i = p / ((int64_t)N[1] * N[2]);
    r[0] = (double)i * L[0] / N[0];
    r[1] = (double)j * L[1] / N[1];
    r[2] = (double)k * L[2] / N[2];
}

int oracle_neighbours(const double *pos, int n_atoms, const double *L, const int *N,
                      double rcut, int64_t p, double *disp, int max_nbr)
{
    double r[3];
    grid_point(N, L, p, r);
    int nmax[3];
    for (int d = 0; d < 3; d++) nmax[d] = (int)ceil(rcut / L[d]) + 1;
    int cnt = 0;
    for (int a = 0; a < n_atoms; a++) {
        for (int nx = -nmax[0]; nx <= nmax[0]; nx++)
            for (int ny = -nmax[1]; ny <= nmax[1]; ny++)
                for (int nz = -nmax[2]; nz <= nmax[2]; nz++) {
                    double dx = pos[3 * a] + nx * L[0] - r[0];
                    double dy = pos[3 * a + 1] + ny * L[1] - r[1];
                    double dz = pos[3 * a + 2] + nz * L[2] - r[2];
                    if (dx * dx + dy * dy + dz * dz < rcut * rcut) {
                        if (cnt < max_nbr) {
                            disp[3 * cnt] = dx; disp[3 * cnt + 1] = dy; disp[3 * cnt + 2] = dz;
                        }
                        cnt++;
                    }
                }
    }
    return cnt;
}

/* Gaussian descriptors: the Gaussian representation of the ionic positions
 * that gives the structure factor (Eq. structurefactor_gaussian), a
 * normalised Gaussian of width sigma on every atom and periodic image:
 *   G(r) = sum_{atoms, images, |r-R| < cutoff} (2 pi sigma^2)^(-3/2) exp(-|r-R|^2 / (2 sigma^2)),
 * at the listed flat grid points.                                          */
void oracle_gaussian(const double *pos, int n_atoms, const double *L, const int *N, double sigma,
                     double cutoff, const int64_t *pts, int64_t n_pts, double *out, int nthreads)
{
    const double norm = pow(2.0 * OR_PI * sigma * sigma, -1.5);
    int nmax[3];
    for (int d = 0; d < 3; d++) nmax[d] = (int)ceil(cutoff / L[d]) + 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t q = 0; q < n_pts; q++) {
        double r[3];
        grid_point(N, L, pts[q], r);
        double sum = 0.0;
        for (int a = 0; a < n_atoms; a++)
            for (int nx = -nmax[0]; nx <= nmax[0]; nx++)
                for (int ny = -nmax[1]; ny <= nmax[1]; ny++)
                    for (int nz = -nmax[2]; nz <= nmax[2]; nz++) {
                        double dx = pos[3 * a] + nx * L[0] - r[0];
                        double dy = pos[3 * a + 1] + ny * L[1] - r[1];
                        double dz = pos[3 * a + 2] + nz * L[2] - r[2];
                        double d2 = dx * dx + dy * dy + dz * dz;
                        if (d2 < cutoff * cutoff) sum += exp(-d2 / (2.0 * sigma * sigma));
                    }
        out[q] = norm * sum;
    }
}

/* B at the listed flat grid points; B_out is [n_pts][n_triples].
 * Returns the largest neighbour count seen (or -1 if max_nbr overflowed). */
int oracle_descriptors(const double *pos, int n_atoms, const double *L, const int *N,
                       double rcut, int twojmax, const int64_t *pts, int64_t n_pts,
                       double *B_out, double *max_imag_out, int nthreads)
{
    const int max_nbr = 4096;
    int nt = oracle_n_triples(twojmax);
    int usz = oracle_u_size(twojmax);
    int worst = 0, overflow = 0;
    double mi_all = 0.0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(max : worst, mi_all) reduction(| : overflow)
#endif
    {
        double *disp = malloc(sizeof(double) * 3 * max_nbr);
        double *u = malloc(sizeof(double) * 2 * usz);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
        for (int64_t q = 0; q < n_pts; q++) {
            int cnt = oracle_neighbours(pos, n_atoms, L, N, rcut, pts[q], disp, max_nbr);
            if (cnt > max_nbr) { overflow = 1; cnt = max_nbr; }
            if (cnt > worst) worst = cnt;
            oracle_ui(disp, cnt, rcut, twojmax, u);
            double mi;
            oracle_bispectrum(u, twojmax, B_out + q * nt, &mi);
            if (mi > mi_all) mi_all = mi;
        }
        free(disp);
        free(u);
    }
    if (max_imag_out) *max_imag_out = mi_all;
    return overflow ? -1 : worst;
}

/* ------------------------------------------------------------ network
 * x0 = (B - mean) / std; x_{l+1} = act(W_l x_l + b_l) for every layer
 * (activation on the output layer too when out_act != 0), act = LeakyReLU
 * with the given negative slope; then ldos = out_scale * y + out_shift.
 * W[l] is [widths[l+1]][widths[l]] row-major; all pointers are concatenated
 * per layer in Wcat / bcat.                                                */
void oracle_mlp(const double *B, int64_t n_pts, int n_layers, const int *widths,
                const double *Wcat, const double *bcat, const double *in_mean,
                const double *in_std, const double *out_scale, const double *out_shift,
                double slope, int out_act, double *ldos, int nthreads)
{
    int wmax = 0;
    for (int l = 0; l <= n_layers; l++) if (widths[l] > wmax) wmax = widths[l];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *x = malloc(sizeof(double) * wmax), *y = malloc(sizeof(double) * wmax);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t p = 0; p < n_pts; p++) {
            for (int i = 0; i < widths[0]; i++)
                x[i] = (B[p * widths[0] + i] - in_mean[i]) / in_std[i];
            const double *W = Wcat, *b = bcat;
            for (int l = 0; l < n_layers; l++) {
                int fin = widths[l], fout = widths[l + 1];
                for (int o = 0; o < fout; o++) {
                    double s = b[o];
                    for (int i = 0; i < fin; i++) s += W[o * fin + i] * x[i];
                    int act = (l < n_layers - 1) || out_act;
                    y[o] = (act && s < 0.0) ? slope * s : s;
                }
                memcpy(x, y, sizeof(double) * fout);
                W += fout * fin;
                b += fout;
            }
            int nout = widths[n_layers];
            for (int e = 0; e < nout; e++)
                ldos[p * nout + e] = out_scale[e] * x[e] + out_shift[e];
        }
        free(x);
        free(y);
    }
}

/* ------------------------------------------------------------ grid ACE
 * Grid-centred atomic cluster expansion descriptors (Sec. 3.2.3, Eqs.
 * unweighted_ionicdensity, gridatom_basis, grid_base, product_grid_basis,
 * ace_grid) with one chemical element:
 *   phi_nlm(d) = R_n(|d|) Y_l^m(d/|d|),  R_n(r) = T_n(2 r / rcut - 1) fc(r)
 *   (Chebyshev polynomial of the first kind times the cosine cutoff, which
 *   makes every basis function vanish smoothly at the cutoff),
 *   A_nlm = sum over atom images within rcut of phi_nlm(R - r) plus the
 *   grid point's own delta, which projects onto l = 0 only:
 *   R_n(0) Y_0^0 = (-1)^n / sqrt(4 pi);
 *   rank 1: B = A_n00 (real);
 *   rank 2: B = sum_m (-1)^m A_{n1 l m} A_{n2 l -m};
 *   rank 3: B = sum_{m1+m2+m3=0} (l1 l2 l3; m1 m2 m3) A_{n1 l1 m1} A_{n2 l2 m2} A_{n3 l3 m3}
 *   (Wigner 3j symbol), l1+l2+l3 even and triangle.
 * Order: rank 1 for n = 0..nmax-1; rank 2 for l = 0..lmax, n1 <= n2; rank 3
 * over multisets of three (n, l) pairs, key p = n (lmax+1) + l, p1 <= p2 <= p3.
 * Y_l^m: orthonormal complex spherical harmonics with the Condon-Shortley
 * phase.                                                                   */

/* Y_l^m(theta, phi) from the explicit associated Legendre sum. */
cplx oracle_ylm(int l, int m, double x, double y, double z)
{
    double r = sqrt(x * x + y * y + z * z);
    double t = z / r, st = sqrt(fmax(0.0, 1.0 - t * t));
    double phi = atan2(y, x);
    int am = abs(m);
    /* d^am/dt^am P_l(t), P_l(t) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) t^(l-2k) */
    double dp = 0.0;
    for (int k = 0; 2 * k <= l; k++) {
        int pw = l - 2 * k;
        if (pw < am) continue;
        double c = ((k & 1) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l) / pow(2.0, l);
        double f = 1.0;
        for (int i = 0; i < am; i++) f *= (pw - i);
        dp += c * f * pow(t, pw - am);
    }
    double plm = ((am & 1) ? -1.0 : 1.0) * pow(st, am) * dp;     /* Condon-Shortley phase */
    double nrm = sqrt((2 * l + 1) / (4.0 * OR_PI) * fact(l - am) / fact(l + am));
    cplx v = nrm * plm * cexp(I * am * phi);
    if (m < 0) v = ((am & 1) ? -1.0 : 1.0) * conj(v);
    return v;
}

/* Wigner 3j symbol by the Racah formula (integer angular momenta). */
double oracle_wigner3j(int l1, int l2, int l3, int m1, int m2, int m3)
{
    if (m1 + m2 + m3 != 0) return 0.0;
    if (l3 < abs(l1 - l2) || l3 > l1 + l2) return 0.0;
    if (abs(m1) > l1 || abs(m2) > l2 || abs(m3) > l3) return 0.0;
    double tri = fact(l1 + l2 - l3) * fact(l1 - l2 + l3) * fact(-l1 + l2 + l3) / fact(l1 + l2 + l3 + 1);
    double pre = sqrt(tri * fact(l1 + m1) * fact(l1 - m1) * fact(l2 + m2) * fact(l2 - m2) * fact(l3 + m3) *
                      fact(l3 - m3));
    double s = 0.0;
    for (int k = 0; k <= l1 + l2 + l3; k++) {
        int a = l1 + l2 - l3 - k, b = l1 - m1 - k, c = l2 + m2 - k, d = l3 - l2 + m1 + k, e = l3 - l1 - m2 + k;
        if (a < 0 || b < 0 || c < 0 || d < 0 || e < 0) continue;
        s += ((k & 1) ? -1.0 : 1.0) / (fact(k) * fact(a) * fact(b) * fact(c) * fact(d) * fact(e));
    }
    return (((l1 - l2 - m3) & 1) ? -1.0 : 1.0) * pre * s;
}

/* R_n(r) = T_n(2 r / rcut - 1) fc(r), T_n from its definition cos(n acos x). */
double oracle_ace_radial(int n, double r, double rcut)
{
    if (r >= rcut) return 0.0;
    double x = 2.0 * r / rcut - 1.0;
    return cos(n * acos(fmax(-1.0, fmin(1.0, x)))) * oracle_cutoff(r, rcut);
}

static int ace_triangle_even(int a, int b, int c)
{
    return c >= abs(a - b) && c <= a + b && ((a + b + c) % 2 == 0);
}

int oracle_ace_count(int nmax, int lmax)
{
    int np = nmax * (lmax + 1), n3 = 0;
    for (int p1 = 0; p1 < np; p1++)
        for (int p2 = p1; p2 < np; p2++)
            for (int p3 = p2; p3 < np; p3++)
                if (ace_triangle_even(p1 % (lmax + 1), p2 % (lmax + 1), p3 % (lmax + 1))) n3++;
    return nmax + (lmax + 1) * nmax * (nmax + 1) / 2 + n3;
}

/* The grid basis A_nlm (Eq. grid_base) of flat grid point p: A[n*nl + l*l + l + m]
 * for n < nmax, l <= lmax, nl = (lmax+1)^2.  Returns the neighbour count, or
 * -1 if it exceeds max_nbr (disp holds 3*max_nbr doubles). */
static int ace_point_basis(const double *pos, int n_atoms, const double *L, const int *N, double rcut, int nmax,
                           int lmax, int64_t p, double *disp, int max_nbr, cplx *A)
{
    int nl = (lmax + 1) * (lmax + 1);
    int cnt = oracle_neighbours(pos, n_atoms, L, N, rcut, p, disp, max_nbr);
    if (cnt > max_nbr) return -1;
    for (int i = 0; i < nmax * nl; i++) A[i] = 0.0;
    for (int n = 0; n < nmax; n++)                  /* the grid point's own delta */
        A[n * nl] = ((n & 1) ? -1.0 : 1.0) / sqrt(4.0 * OR_PI);
    for (int k = 0; k < cnt; k++) {
        double dx = disp[3 * k], dy = disp[3 * k + 1], dz = disp[3 * k + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0) {                               /* an atom on the point: l = 0 only */
            for (int n = 0; n < nmax; n++)
                A[n * nl] += oracle_ace_radial(n, 0.0, rcut) / sqrt(4.0 * OR_PI);
            continue;
        }
        for (int l = 0; l <= lmax; l++)
            for (int m = -l; m <= l; m++) {
                cplx y = oracle_ylm(l, m, dx, dy, dz);
                for (int n = 0; n < nmax; n++) A[n * nl + l * l + l + m] += oracle_ace_radial(n, r, rcut) * y;
            }
    }
    return cnt;
}

/* Descriptors at the listed flat grid points; out is [n_pts][count]. */
int oracle_ace(const double *pos, int n_atoms, const double *L, const int *N, double rcut, int nmax,
               int lmax, const int64_t *pts, int64_t n_pts, double *out, int nthreads)
{
    const int max_nbr = 4096;
    int nd = oracle_ace_count(nmax, lmax), nl = (lmax + 1) * (lmax + 1);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int overflow = 0;
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        double *disp = malloc(sizeof(double) * 3 * max_nbr);
        cplx *A = malloc(sizeof(cplx) * nmax * nl);     /* A[n][l*l + l + m] */
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t q = 0; q < n_pts; q++) {
            if (ace_point_basis(pos, n_atoms, L, N, rcut, nmax, lmax, pts[q], disp, max_nbr, A) < 0) {
                overflow = 1;
                continue;
            }
            double *o = out + q * nd;
            int d = 0;
            for (int n = 0; n < nmax; n++) o[d++] = creal(A[n * nl]);
            for (int l = 0; l <= lmax; l++)
                for (int n1 = 0; n1 < nmax; n1++)
                    for (int n2 = n1; n2 < nmax; n2++) {
                        cplx s = 0.0;
                        for (int m = -l; m <= l; m++)
                            s += ((m & 1) ? -1.0 : 1.0) * A[n1 * nl + l * l + l + m] * A[n2 * nl + l * l + l - m];
                        o[d++] = creal(s);
                    }
            int np = nmax * (lmax + 1);
            for (int p1 = 0; p1 < np; p1++)
                for (int p2 = p1; p2 < np; p2++)
                    for (int p3 = p2; p3 < np; p3++) {
                        int n1 = p1 / (lmax + 1), l1 = p1 % (lmax + 1), n2 = p2 / (lmax + 1), l2 = p2 % (lmax + 1);
                        int n3 = p3 / (lmax + 1), l3 = p3 % (lmax + 1);
                        if (!ace_triangle_even(l1, l2, l3)) continue;
                        cplx s = 0.0;
                        for (int m1 = -l1; m1 <= l1; m1++)
                            for (int m2 = -l2; m2 <= l2; m2++) {
                                int m3 = -m1 - m2;
                                if (abs(m3) > l3) continue;
                                s += oracle_wigner3j(l1, l2, l3, m1, m2, m3) * A[n1 * nl + l1 * l1 + l1 + m1] *
                                     A[n2 * nl + l2 * l2 + l2 + m2] * A[n3 * nl + l3 * l3 + l3 + m3];
                            }
                        o[d++] = creal(s);
                    }
        }
        free(disp);
        free(A);
    }
    return overflow ? -1 : 0;
}

/* Rank 4 (Eq. ace_grid with N = 4): the generalized Clebsch-Gordan
 * coefficient of the coupling tree ((l1 l2) L, (l3 l4) L) -> 0,
 *   C(m; L) = <l1 m1 l2 m2 | L M> <l3 m3 l4 m4 | L, -M> <L M L, -M | 0 0>,
 *   M = m1 + m2 = -(m3 + m4),  <L M L, -M | 0 0> = (-1)^(L-M) / sqrt(2L+1),
 * the intermediate coupling L being the one entry of the multiset L of the
 * equation for four factors (zero unless m1+m2+m3+m4 = 0). */
double oracle_ace_gcg4(int l1, int l2, int l3, int l4, int L, int m1, int m2, int m3, int m4)
{
    if (m1 + m2 + m3 + m4 != 0) return 0.0;
    int M = m1 + m2;
    if (abs(M) > L) return 0.0;
    double c12 = oracle_cg(2 * l1, 2 * m1, 2 * l2, 2 * m2, 2 * L, 2 * M);
    double c34 = oracle_cg(2 * l3, 2 * m3, 2 * l4, 2 * m4, 2 * L, -2 * M);
    return c12 * c34 * (((L - M) & 1) ? -1.0 : 1.0) / sqrt(2.0 * L + 1.0);
}

/* Rank-4 descriptors B = sum over m1..m4 of C(m; L) A_{n1 l1 m1} A_{n2 l2 m2}
 * A_{n3 l3 m3} A_{n4 l4 m4} at the listed flat grid points, for the n_desc
 * descriptors desc[5k..5k+4] = (p1, p2, p3, p4, L) with key p = n (lmax+1) + l
 * (the set itself, which couplings are kept, is chosen by the caller);
 * out is [n_pts][n_desc]. */
int oracle_ace4(const double *pos, int n_atoms, const double *L, const int *N, double rcut, int nmax, int lmax,
                const int *desc, int n_desc, const int64_t *pts, int64_t n_pts, double *out, int nthreads)
{
    const int max_nbr = 4096;
    int nl = (lmax + 1) * (lmax + 1);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int overflow = 0;
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        double *disp = malloc(sizeof(double) * 3 * max_nbr);
        cplx *A = malloc(sizeof(cplx) * nmax * nl);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t q = 0; q < n_pts; q++) {
            if (ace_point_basis(pos, n_atoms, L, N, rcut, nmax, lmax, pts[q], disp, max_nbr, A) < 0) {
                overflow = 1;
                continue;
            }
            for (int k = 0; k < n_desc; k++) {
                const int *d = desc + 5 * k;
                int n[4], l[4];
                for (int i = 0; i < 4; i++) {
                    n[i] = d[i] / (lmax + 1);
                    l[i] = d[i] % (lmax + 1);
                }
                cplx s = 0.0;
                for (int m1 = -l[0]; m1 <= l[0]; m1++)
                    for (int m2 = -l[1]; m2 <= l[1]; m2++)
                        for (int m3 = -l[2]; m3 <= l[2]; m3++) {
                            int m4 = -m1 - m2 - m3;
                            if (abs(m4) > l[3]) continue;
                            double c = oracle_ace_gcg4(l[0], l[1], l[2], l[3], d[4], m1, m2, m3, m4);
                            if (c == 0.0) continue;
                            s += c * A[n[0] * nl + l[0] * l[0] + l[0] + m1] * A[n[1] * nl + l[1] * l[1] + l[1] + m2] *
                                 A[n[2] * nl + l[2] * l[2] + l[2] + m3] * A[n[3] * nl + l[3] * l[3] + l[3] + m4];
                        }
                out[q * n_desc + k] = creal(s);
            }
        }
        free(disp);
        free(A);
    }
    return overflow ? -1 : 0;
}

/* ------------------------------------------------------------ descriptor VJP
 * The descriptor factor of the force expression (Eq. forcesmala): for
 * weights gB(p) over the n_B components, the gradient of
 * L = sum_p sum_l gB_l(p) B_l(p) with respect to every atom position.
 * Chain rule in the order of the definitions:
 *   B(u) is a sum of triple products Re(conj(x) C C y z) with x = u^j,
 *   y = u^j1, z = u^j2; with dL = sum Re(conj(Y) du) the product rule gives
 *   Y_x += g C C y z,  Y_y += g C C x conj(z),  Y_z += g C C x conj(y);
 *   u^J = I + sum_k fc(r_k) U^J(Delta_k), Delta_k = R_atom(k) + shift - r_p,
 *   so dL/dR_atom = sum over its images k of
 *   sum_J sum_{m m'} Re(conj(Y^J_{m m'}) d(fc U^J_{m m'})/dDelta_k).        */

/* Y [size][2] (all rows of every level) for one point's u and weights gB. */
void oracle_u_adjoint(const double *u, int twojmax, const double *gB, double *Y)
{
    int nt = oracle_n_triples(twojmax), size = u_off(twojmax + 1);
    int *tr = malloc(sizeof(int) * 3 * nt);
    oracle_triples(twojmax, tr);
    memset(Y, 0, sizeof(double) * 2 * size);
    for (int t = 0; t < nt; t++) {
        int j1 = tr[3 * t], j2 = tr[3 * t + 1], j = tr[3 * t + 2];
        double g = gB[t];
        for (int m = -j; m <= j; m += 2)
            for (int mp = -j; mp <= j; mp += 2) {
                int ex = u_off(j) + ((j + m) / 2) * (j + 1) + (j + mp) / 2;
                cplx x = u[2 * ex] + I * u[2 * ex + 1];
                for (int m1 = -j1; m1 <= j1; m1 += 2) {
                    int m2 = m - m1;
                    if (m2 < -j2 || m2 > j2) continue;
                    double c1 = oracle_cg(j1, m1, j2, m2, j, m);
                    for (int m1p = -j1; m1p <= j1; m1p += 2) {
                        int m2p = mp - m1p;
                        if (m2p < -j2 || m2p > j2) continue;
                        double c = g * c1 * oracle_cg(j1, m1p, j2, m2p, j, mp);
                        int ey = u_off(j1) + ((j1 + m1) / 2) * (j1 + 1) + (j1 + m1p) / 2;
                        int ez = u_off(j2) + ((j2 + m2) / 2) * (j2 + 1) + (j2 + m2p) / 2;
                        cplx y = u[2 * ey] + I * u[2 * ey + 1], z = u[2 * ez] + I * u[2 * ez + 1];
                        cplx yx = c * y * z, yy = c * x * conj(z), yz = c * x * conj(y);
                        Y[2 * ex] += creal(yx); Y[2 * ex + 1] += cimag(yx);
                        Y[2 * ey] += creal(yy); Y[2 * ey + 1] += cimag(yy);
                        Y[2 * ez] += creal(yz); Y[2 * ez + 1] += cimag(yz);
                    }
                }
            }
    }
    free(tr);
}

/* d a / d Delta_d and d b / d Delta_d (complex, d = x, y, z) of the
 * Cayley-Klein parameters of oracle_cayley_klein: with theta = k r,
 * k = rfac0 pi / rcut, n = Delta / r, dr/dDelta_d = n_d,
 * dn_i/dDelta_d = (delta_id - n_i n_d) / r:
 *   a = cos theta - i n_z sin theta,  b = -sin theta (n_y + i n_x).       */
void oracle_dcayley_klein(double dx, double dy, double dz, double rcut, double *da /* [3][2] */,
                          double *db /* [3][2] */)
{
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double n[3] = {dx / r, dy / r, dz / r};
    double k = OR_RFAC0 * OR_PI / rcut, th = k * r, c = cos(th), s = sin(th);
    for (int d = 0; d < 3; d++) {
        double dth = k * n[d];
        double dn[3];
        for (int i = 0; i < 3; i++) dn[i] = ((i == d ? 1.0 : 0.0) - n[i] * n[d]) / r;
        cplx dA = -s * dth - I * (dn[2] * s + n[2] * c * dth);
        cplx dB = -c * dth * (n[1] + I * n[0]) - s * (dn[1] + I * dn[0]);
        da[2 * d] = creal(dA); da[2 * d + 1] = cimag(dA);
        db[2 * d] = creal(dB); db[2 * d + 1] = cimag(dB);
    }
}

/* d fc / d r of oracle_cutoff (0 at and past rcut). */
double oracle_dcutoff(double r, double rcut)
{
    if (r >= rcut) return 0.0;
    return -0.5 * OR_PI / rcut * sin(OR_PI * r / rcut);
}

/* dU^J along one direction, given the parameters (a, b) and their
 * derivatives (da, db) in that direction: the product rule applied to each
 * monomial a^s (-conj b)^(ma-s) b^t (conj a)^(J-ma-t) of oracle_wigner_u.  */
void oracle_dwigner_u(int J, double a_re, double a_im, double b_re, double b_im, double da_re,
                      double da_im, double db_re, double db_im, double *out /* [(J+1)^2][2] */)
{
    cplx a = a_re + I * a_im, b = b_re + I * b_im, da = da_re + I * da_im, db = db_re + I * db_im;
    cplx mbc = -conj(b), ac = conj(a), dmbc = -conj(db), dac = conj(da);
    for (int ma = 0; ma <= J; ma++)
        for (int mb = 0; mb <= J; mb++) {
            cplx coef = 0.0;
            for (int s = 0; s <= ma; s++) {
                int t = mb - s;
                if (t < 0 || t > J - ma) continue;
                int p1 = s, p2 = ma - s, p3 = t, p4 = J - ma - t;
                cplx f1 = cpow_int(a, p1), f2 = cpow_int(mbc, p2), f3 = cpow_int(b, p3), f4 = cpow_int(ac, p4);
                cplx d = 0.0;
                if (p1 > 0) d += p1 * cpow_int(a, p1 - 1) * da * f2 * f3 * f4;
                if (p2 > 0) d += f1 * p2 * cpow_int(mbc, p2 - 1) * dmbc * f3 * f4;
                if (p3 > 0) d += f1 * f2 * p3 * cpow_int(b, p3 - 1) * db * f4;
                if (p4 > 0) d += f1 * f2 * f3 * p4 * cpow_int(ac, p4 - 1) * dac;
                coef += binom(ma, s) * binom(J - ma, t) * d;
            }
            double norm = sqrt(fact(mb) * fact(J - mb) / (fact(ma) * fact(J - ma)));
            out[2 * (ma * (J + 1) + mb)] = creal(coef * norm);
            out[2 * (ma * (J + 1) + mb) + 1] = cimag(coef * norm);
        }
}

/* dL/dR [n_atoms][3] for L = sum over the listed grid points p of
 * sum_l gB[p][l] B_l(p) (gB is [n_pts][n_triples]).  Per-thread partial
 * sums are added in thread order at the end.                              */
int oracle_descriptors_vjp(const double *pos, int n_atoms, const double *L, const int *N,
                           double rcut, int twojmax, const int64_t *pts, int64_t n_pts,
                           const double *gB, double *dLdR, int nthreads)
{
    const int max_nbr = 4096;
    int nt = oracle_n_triples(twojmax), usz = oracle_u_size(twojmax);
    int nmax[3];
    for (int d = 0; d < 3; d++) nmax[d] = (int)ceil(rcut / L[d]) + 1;
    int nthr = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    nthr = omp_get_max_threads();
#endif
    double *part = calloc((size_t)nthr * n_atoms * 3, sizeof(double));
    int overflow = 0;
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = part + (size_t)tid * n_atoms * 3;
        double *disp = malloc(sizeof(double) * 3 * max_nbr);
        int *atom = malloc(sizeof(int) * max_nbr);
        double *u = malloc(sizeof(double) * 2 * usz), *Y = malloc(sizeof(double) * 2 * usz);
        int w = twojmax + 1;
        double *U = malloc(sizeof(double) * 2 * w * w), *dU = malloc(sizeof(double) * 2 * w * w);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
        for (int64_t q = 0; q < n_pts; q++) {
            double r[3];
            grid_point(N, L, pts[q], r);
            int cnt = 0;
            for (int a = 0; a < n_atoms; a++)
                for (int nx = -nmax[0]; nx <= nmax[0]; nx++)
                    for (int ny = -nmax[1]; ny <= nmax[1]; ny++)
                        for (int nz = -nmax[2]; nz <= nmax[2]; nz++) {
                            double dx = pos[3 * a] + nx * L[0] - r[0];
                            double dy = pos[3 * a + 1] + ny * L[1] - r[1];
                            double dz = pos[3 * a + 2] + nz * L[2] - r[2];
                            if (dx * dx + dy * dy + dz * dz < rcut * rcut) {
                                if (cnt < max_nbr) {
                                    disp[3 * cnt] = dx; disp[3 * cnt + 1] = dy; disp[3 * cnt + 2] = dz;
                                    atom[cnt] = a;
                                }
                                cnt++;
                            }
                        }
            if (cnt > max_nbr) {
                overflow = 1;
                continue;
            }
            oracle_ui(disp, cnt, rcut, twojmax, u);
            oracle_u_adjoint(u, twojmax, gB + q * nt, Y);
            for (int k = 0; k < cnt; k++) {
                double dx = disp[3 * k], dy = disp[3 * k + 1], dz = disp[3 * k + 2];
                double rr = sqrt(dx * dx + dy * dy + dz * dz);
                if (rr == 0.0) continue;          /* an atom on the point: u gets +I, no direction */
                double fc = oracle_cutoff(rr, rcut), dfc = oracle_dcutoff(rr, rcut);
                double ar, ai, br, bi, da[6], db[6];
                oracle_cayley_klein(dx, dy, dz, rcut, &ar, &ai, &br, &bi);
                oracle_dcayley_klein(dx, dy, dz, rcut, da, db);
                double nrm[3] = {dx / rr, dy / rr, dz / rr};
                for (int J = 0; J <= twojmax; J++) {
                    int o = u_off(J), ne = (J + 1) * (J + 1);
                    oracle_wigner_u(J, ar, ai, br, bi, U);
                    for (int d = 0; d < 3; d++) {
                        oracle_dwigner_u(J, ar, ai, br, bi, da[2 * d], da[2 * d + 1], db[2 * d], db[2 * d + 1], dU);
                        double s = 0.0;
                        for (int e = 0; e < ne; e++) {
                            double vr = dfc * nrm[d] * U[2 * e] + fc * dU[2 * e];
                            double vi = dfc * nrm[d] * U[2 * e + 1] + fc * dU[2 * e + 1];
                            s += Y[2 * (o + e)] * vr + Y[2 * (o + e) + 1] * vi;   /* Re(conj(Y) v) */
                        }
                        acc[3 * atom[k] + d] += s;
                    }
                }
            }
        }
        free(disp); free(atom); free(u); free(Y); free(U); free(dU);
    }
    for (int i = 0; i < n_atoms * 3; i++) {
        double s = 0.0;
        for (int t = 0; t < nthr; t++) s += part[(size_t)t * n_atoms * 3 + i];
        dLdR[i] = s;
    }
    free(part);
    return overflow ? -1 : 0;
}

/* ------------------------------------------------------------ network VJP
 * The middle factor of the force expression (Eq. forcesmala): for a vector
 * v(p) over the energies, g(p) = (dd(p)/dB(p))^T v(p), by backpropagation
 * through the network of oracle_mlp in FP64.  Layer l forms
 * z_l = W_l x_{l-1} + b_l and x_l = sigma(z_l) (on the output layer only
 * when out_act), x_0 = (B - mean)/std, d_e = s_e x_L,e + c_e.  With
 * sigma'(z) = 1 for z > 0 and slope otherwise:
 *   delta_L = s .* v .* sigma'(z_L)    (sigma' = 1 without output activation)
 *   delta_{l-1} = (W_l^T delta_l) .* sigma'(z_{l-1})
 *   g = (W_1^T delta_1) ./ std.
 * margin[p] (if not NULL) = min over the units that pass through sigma of
 * |z| / (|b| + sum_i |W_i x_i|): the distance of each unit from its kink
 * relative to the size of the terms that form z.  Evaluated in another
 * precision, a unit can land on the other side of its kink only where this
 * is at that precision's rounding level; there the derivative jumps.       */
void oracle_mlp_vjp(const double *B, int64_t n_pts, int n_layers, const int *widths,
                    const double *Wcat, const double *bcat, const double *in_mean,
                    const double *in_std, const double *out_scale, double slope, int out_act,
                    const double *v, double *g, double *margin, int nthreads)
{
    int wmax = 0;
    for (int l = 0; l <= n_layers; l++) if (widths[l] > wmax) wmax = widths[l];
    const double **Wl = malloc(sizeof(double *) * n_layers), **bl = malloc(sizeof(double *) * n_layers);
    {
        const double *W = Wcat, *b = bcat;
        for (int l = 0; l < n_layers; l++) {
            Wl[l] = W; bl[l] = b;
            W += (size_t)widths[l + 1] * widths[l];
            b += widths[l + 1];
        }
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        /* x[l] = layer l's output (x[0] = scaled input), z[l] = its pre-activation */
        double *x = malloc(sizeof(double) * (n_layers + 1) * wmax);
        double *z = malloc(sizeof(double) * (n_layers + 1) * wmax);
        double *dl = malloc(sizeof(double) * wmax), *dn = malloc(sizeof(double) * wmax);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t p = 0; p < n_pts; p++) {
            double mrg = INFINITY;
            for (int i = 0; i < widths[0]; i++)
                x[i] = (B[p * widths[0] + i] - in_mean[i]) / in_std[i];
            for (int l = 0; l < n_layers; l++) {
                int fin = widths[l], fout = widths[l + 1];
                const double *xi = x + (size_t)l * wmax;
                double *zo = z + (size_t)(l + 1) * wmax, *xo = x + (size_t)(l + 1) * wmax;
                int act = (l < n_layers - 1) || out_act;
                for (int o = 0; o < fout; o++) {
                    double s = bl[l][o], mag = fabs(bl[l][o]);
                    for (int i = 0; i < fin; i++) {
                        s += Wl[l][(size_t)o * fin + i] * xi[i];
                        mag += fabs(Wl[l][(size_t)o * fin + i] * xi[i]);
                    }
                    zo[o] = s;
                    xo[o] = (act && s <= 0.0) ? slope * s : s;
                    if (act && mag > 0.0 && fabs(s) / mag < mrg) mrg = fabs(s) / mag;
                }
            }
            /* backward */
            int nout = widths[n_layers];
            const double *zL = z + (size_t)n_layers * wmax;
            for (int e = 0; e < nout; e++) {
                double d = out_scale[e] * v[p * nout + e];
                if (out_act && !(zL[e] > 0.0)) d *= slope;
                dl[e] = d;
            }
            for (int l = n_layers - 1; l >= 0; l--) {
                int fin = widths[l], fout = widths[l + 1];
                for (int i = 0; i < fin; i++) {
                    double s = 0.0;
                    for (int o = 0; o < fout; o++) s += Wl[l][(size_t)o * fin + i] * dl[o];
                    if (l > 0 && !(z[(size_t)l * wmax + i] > 0.0)) s *= slope;
                    dn[i] = s;
                }
                memcpy(dl, dn, sizeof(double) * fin);
            }
            for (int i = 0; i < widths[0]; i++) g[p * widths[0] + i] = dl[i] / in_std[i];
            if (margin) margin[p] = mrg;
        }
        free(x); free(z); free(dl); free(dn);
    }
    free(Wl);
    free(bl);
}

/* ------------------------------------------------------------ DOS
 * D_e = dV * sum_p d_e(p): the spatial integral of the LDOS as a sum over
 * grid points times the volume element.                                    */
void oracle_dos(const double *ldos, int64_t n_pts, int n_e, double dV, double *dos)
{
    for (int e = 0; e < n_e; e++) dos[e] = 0.0;
    for (int64_t p = 0; p < n_pts; p++)
        for (int e = 0; e < n_e; e++) dos[e] += ldos[p * n_e + e];
    for (int e = 0; e < n_e; e++) dos[e] *= dV;
}

/* ------------------------------------------------------------ polylog
 * Li_s(-y) for 0 <= y <= 1 and s >= 1 as the alternating series
 * -sum_{k>=0} (-1)^k y^(k+1)/(k+1)^s, summed with the Cohen-Rodriguez
 * Villegas-Zagier acceleration (Exp. Math. 9 (2000), Algorithm 1), valid
 * because y^(k+1)/(k+1)^s is a moment sequence.  40 terms: error
 * ~ (3+sqrt 8)^-40.                                                        */
double oracle_li_neg(int s, double y)
{
    if (y == 0.0) return 0.0;
    if (s == 1) return -log1p(y);
    const int n = 40;
    double d = pow(3.0 + sqrt(8.0), n);
    d = 0.5 * (d + 1.0 / d);
    double b = -1.0, c = -d, sum = 0.0, yk = y;
    for (int k = 0; k < n; k++) {
        c = b - c;
        sum += c * yk / pow((double)(k + 1), s);
        b = (double)(k + n) * (double)(k - n) * b / ((k + 0.5) * (k + 1.0));
        yk *= y;
    }
    return -sum / d;
}

/* Antiderivatives in x = beta (e - mu) of f = 1/(1+e^x) times 1, x, x^2:
 *   G0 = x - ln(1+e^x), G1 = x^2/2 - x ln(1+e^x) - Li2(-e^x),
 *   G2 = x^3/3 - x^2 ln(1+e^x) - 2x Li2(-e^x) + 2 Li3(-e^x),
 * from d/dx Li_s(-e^x) = Li_{s-1}(-e^x) and f = 1 + Li0(-e^x).  For x > 0
 * the same functions are written with the inversion formulas of Li2, Li3
 * so that only Li_s(-e^-x) appears.                                        */
static void g012(double x, double *g0, double *g1, double *g2)
{
    if (x <= 0.0) {
        double y = exp(x), Lg = log1p(y);
        double l2 = oracle_li_neg(2, y), l3 = oracle_li_neg(3, y);
        *g0 = x - Lg;
        *g1 = 0.5 * x * x - x * Lg - l2;
        *g2 = x * x * x / 3.0 - x * x * Lg - 2.0 * x * l2 + 2.0 * l3;
    } else {
        double y = exp(-x), Lg = log1p(y);
        double l2 = oracle_li_neg(2, y), l3 = oracle_li_neg(3, y);
        *g0 = -Lg;
        *g1 = OR_PI * OR_PI / 6.0 - x * Lg + l2;
        *g2 = -x * x * Lg + 2.0 * x * l2 + 2.0 * l3;
    }
}

/* Weights of a piecewise-linear DOS on the uniform grid e_i = e0 + i de:
 *   int f(e) D(e) de   = sum_i w_i D_i,
 *   int f(e) e D(e) de = sum_i v_i D_i,
 * exact for D linear between grid points and zero outside.  kT in eV.     */
void oracle_fermi_weights(double e0, double de, int n, double mu, double kT,
                          double *w, double *v)
{
    double beta = 1.0 / kT;
    for (int i = 0; i < n; i++) { w[i] = 0.0; v[i] = 0.0; }
    for (int i = 0; i + 1 < n; i++) {
        double xa = beta * (e0 + i * de - mu), xb = beta * (e0 + (i + 1) * de - mu);
        double a0, a1, a2, b0, b1, b2;
        g012(xa, &a0, &a1, &a2);
        g012(xb, &b0, &b1, &b2);
        double D = xb - xa;                     /* = beta * de */
        /* int f de over the interval, and int f (e - e_i)/de de           */
        double I0 = (b0 - a0) / beta;
        double I1 = ((b1 - a1) - xa * (b0 - a0)) / (beta * D);
        /* int f x de and int f x (e - e_i)/de de, x = beta (e - mu)        */
        double K0 = (b1 - a1) / beta;
        double K1 = ((b2 - a2) - xa * (b1 - a1)) / (beta * D);
        /* hat functions: phi_i = 1 - t, phi_{i+1} = t, t = (e - e_i)/de   */
        w[i] += I0 - I1;
        w[i + 1] += I1;
        /* e = mu + x / beta */
        v[i] += mu * (I0 - I1) + (K0 - K1) / beta;
        v[i + 1] += mu * I1 + K1 / beta;
    }
}

/* Electronic entropy (Eq. electronicentropyDOS): with x = beta (e - mu) and
 * f = 1/(1+e^x), the integrand -[f ln f + (1-f) ln(1-f)] equals
 * s(x) = ln(1+e^x) - x (1 - f), whose antiderivatives are
 *   S0(x) = int s dx   = -2 Li2(-e^x) - x ln(1+e^x),
 *   S1(x) = int x s dx = -x^2 ln(1+e^x) - 3x Li2(-e^x) + 3 Li3(-e^x)
 * (differentiate with d/dx Li_s(-e^x) = Li_{s-1}(-e^x)); for x > 0 they are
 * rewritten with the inversion formulas for Li2, Li3 so only Li_s(-e^-x) is
 * needed.  There S0 = pi^2/3 + 2 Li2(-e^-x) - x ln(1+e^-x): the constant is
 * left out here and added by the caller to the one interval that crosses
 * x = 0, so that differences far in the tail are not lost to rounding.     */
static void s01(double x, double *s0, double *s1)
{
    if (x <= 0.0) {
        double y = exp(x), Lg = log1p(y);
        double l2 = oracle_li_neg(2, y), l3 = oracle_li_neg(3, y);
        *s0 = -2.0 * l2 - x * Lg;
        *s1 = -x * x * Lg - 3.0 * x * l2 + 3.0 * l3;
    } else {
        double y = exp(-x), Lg = log1p(y);
        double l2 = oracle_li_neg(2, y), l3 = oracle_li_neg(3, y);
        *s0 = 2.0 * l2 - x * Lg;
        *s1 = -x * x * Lg + 3.0 * x * l2 + 3.0 * l3;
    }
}

/* Entropy weights of a piecewise-linear DOS on the uniform grid:
 *   S_s / k_B = int s(beta (e - mu)) D(e) de = sum_i u_i D_i,
 * exact for D linear between grid points and zero outside.  kT in eV.     */
void oracle_entropy_weights(double e0, double de, int n, double mu, double kT, double *u)
{
    double beta = 1.0 / kT;
    for (int i = 0; i < n; i++) u[i] = 0.0;
    for (int i = 0; i + 1 < n; i++) {
        double xa = beta * (e0 + i * de - mu), xb = beta * (e0 + (i + 1) * de - mu);
        double a0, a1, b0, b1;
        s01(xa, &a0, &a1);
        s01(xb, &b0, &b1);
        double d0 = b0 - a0;
        if (xa <= 0.0 && xb > 0.0) d0 += OR_PI * OR_PI / 3.0;   /* S0's jump of constant */
        double D = xb - xa;
        double J0 = d0 / beta;                                 /* int s de       */
        double J1 = ((b1 - a1) - xa * d0) / (beta * D);        /* int s t de     */
        u[i] += J0 - J1;
        u[i + 1] += J1;
    }
}

/* S_s / k_B at Fermi level mu for the DOS on the grid, and the free-energy
 * term -tau S_s = -k_B T (S_s / k_B) in eV (Eq. KSfreeenergy).             */
double oracle_entropy(const double *dos, double e0, double de, int n, double T_K, double mu,
                      double *minus_ts)
{
    double kT = OR_KB_EV * T_K;
    double *u = malloc(sizeof(double) * n);
    oracle_entropy_weights(e0, de, n, mu, kT, u);
    double s = 0.0;
    for (int i = 0; i < n; i++) s += u[i] * dos[i];
    free(u);
    if (minus_ts) *minus_ts = -kT * s;
    return s;
}

static double count_electrons(const double *dos, double e0, double de, int n, double mu,
                              double kT, double *w, double *v)
{
    oracle_fermi_weights(e0, de, n, mu, kT, w, v);
    double s = 0.0;
    for (int i = 0; i < n; i++) s += w[i] * dos[i];
    return s;
}

/* Fermi level by bisection on [e_0, e_{n-1}] (N(mu) < N_e -> raise lo),
 * stopping at hi - lo < tol; then the band energy and the final weights.
 * res = {E_F, E_band, N(E_F), iterations}.  Returns 0, or -4 when N_e is
 * outside [N(e_0), N(e_{n-1})].                                            */
int oracle_fermi(const double *dos, double e0, double de, int n, double T_K, double n_e,
                 double tol, double *res, double *w_out)
{
    double kT = OR_KB_EV * T_K;
    double *w = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n);
    double lo = e0, hi = e0 + (n - 1) * de;
    double nlo = count_electrons(dos, e0, de, n, lo, kT, w, v);
    double nhi = count_electrons(dos, e0, de, n, hi, kT, w, v);
    if (!(nlo <= n_e && n_e <= nhi)) {
        free(w); free(v);
        return -4;
    }
    int it = 0;
    while (hi - lo >= tol && it < 200) {
        double mid = 0.5 * (lo + hi);
        if (count_electrons(dos, e0, de, n, mid, kT, w, v) < n_e) lo = mid; else hi = mid;
        it++;
    }
    double ef = 0.5 * (lo + hi);
    double ne = count_electrons(dos, e0, de, n, ef, kT, w, v);
    double eb = 0.0;
    for (int i = 0; i < n; i++) eb += v[i] * dos[i];
    res[0] = ef; res[1] = eb; res[2] = ne; res[3] = it;
    if (w_out) memcpy(w_out, w, sizeof(double) * n);
    free(w); free(v);
    return 0;
}

/* n(p) = sum_e w_e d_e(p) (Eq. density.from.ldos with the same weights). */
void oracle_density(const double *ldos, int64_t n_pts, int n_e, const double *w, double *dens)
{
    for (int64_t p = 0; p < n_pts; p++) {
        double s = 0.0;
        for (int e = 0; e < n_e; e++) s += w[e] * ldos[p * n_e + e];
        dens[p] = s;
    }
}

double oracle_kb_ev(void) { return OR_KB_EV; }
