// Energy-space observables in FP64 (Sec. 3.4): the DOS from its partial
// sums (Eq. DOS.from.ldos), the Fermi level as the root of
// N_e = int f D (Eq. NumberElectrons_from_DOS), the band energy
// (Eq. band.energy), the electronic entropy and its free-energy term
// (Eqs. electronicentropyDOS, KSfreeenergy) and the Fermi weights that turn
// an LDOS into the density (Eq. density.from.ldos).
//
// D is taken piecewise linear between the energy grid points, and the
// integrals of f, f*e against each linear piece are exact: with
// x = (e - mu)/kT they are differences of the antiderivatives
//   x - ln(1+e^x),  x^2/2 - x ln(1+e^x) - Li2(-e^x),
//   x^3/3 - x^2 ln(1+e^x) - 2x Li2(-e^x) + 2 Li3(-e^x)
// (f written through the polylogarithm as in Eq. fermidiracspecial), used in
// the form that only needs Li_s(-y) with 0 < y <= 1.  Li_s(-y) is summed as
// its power series for y <= 1/2 and as the Taylor series in ln y about y = 1
// (coefficients -eta(s-n)/n!, computed on the host) otherwise.
//
// The root is bracketed like the paper's TOMS748 solver: Newton steps on
// N(mu) (dN/dmu = int D (-df/de) needs only f and the first antiderivative)
// from the zero-temperature root of the piecewise-linear D, kept inside a
// shrinking [lo, hi] and replaced by the midpoint whenever they leave it.
#include <math.h>

#include <mutex>

#include "mala_internal.h"

namespace mala {

constexpr double kPi = 3.14159265358979323846;

// Li_s(-y), s in {2, 3}, 0 <= y <= 1.  coef: [2][kLiTerms] Taylor
// coefficients at y = 1, then [2][kLiPow] inverse powers 1/k^s.
__device__ double li_neg(int s, double y, const double* __restrict__ coef) {
    if (y <= 0.5) {
        const double* ik = coef + 2 * kLiTerms + (s - 2) * kLiPow;
        double term = -y, sum = 0.0;
        for (int k = 1; k < kLiPow; ++k) {
            const double t = term * ik[k];
            sum += t;
            if (fabs(t) <= 1e-18 * fabs(sum)) break;
            term *= -y;
        }
        return sum;
    }
    const double t = log(y);                    // in (-ln 2, 0]
    const double* c = coef + (s - 2) * kLiTerms;
    double acc = c[kLiTerms - 1];
    for (int n = kLiTerms - 2; n >= 0; --n) acc = acc * t + c[n];
    return acc;
}

// G0, G1 (and, for the final pass, G2 and the entropy antiderivatives S0,
// S1) at x (see the file comment), and f(x) = 1/(1+e^x).  The entropy
// kernel -[f ln f + (1-f) ln(1-f)] = ln(1+e^x) - x (1-f) has
//   S0 = -2 Li2(-e^x) - x ln(1+e^x),  S1 = -x^2 ln(1+e^x) - 3x Li2(-e^x) + 3 Li3(-e^x);
// for x > 0 they are written through Li_s(-e^-x), with S0's constant pi^2/3
// left to the one interval that crosses x = 0.
__device__ void gfun(double x, const double* coef, bool final, double& g0, double& g1, double& g2, double& f,
                     double& s0, double& s1) {
    if (x <= 0.0) {
        const double y = exp(x), lg = log1p(y);
        const double l2 = li_neg(2, y, coef);
        g0 = x - lg;
        g1 = 0.5 * x * x - x * lg - l2;
        f = 1.0 / (1.0 + y);
        if (final) {
            const double l3 = li_neg(3, y, coef);
            g2 = x * x * x / 3.0 - x * x * lg - 2.0 * x * l2 + 2.0 * l3;
            s0 = -2.0 * l2 - x * lg;
            s1 = -x * x * lg - 3.0 * x * l2 + 3.0 * l3;
        }
    } else {
        const double y = exp(-x), lg = log1p(y);
        const double l2 = li_neg(2, y, coef);
        g0 = -lg;
        g1 = kPi * kPi / 6.0 - x * lg + l2;
        f = y / (1.0 + y);
        if (final) {
            const double l3 = li_neg(3, y, coef);
            g2 = -x * x * lg + 2.0 * x * l2 + 2.0 * l3;
            s0 = 2.0 * l2 - x * lg;
            s1 = -x * x * lg + 3.0 * x * l2 + 3.0 * l3;
        }
    }
    if (!final) g2 = s0 = s1 = 0.0;
}

// Fixed-shape sum over the 256 threads: butterfly inside each wave, then the
// four wave sums in order.
__device__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

struct FermiShared {
    double D[256], red[256], g0[256], g1[256], g2[256], f[256], cum[256], s0[256], s1[256];
    double mu0;
    int first;
};

// Antiderivatives and f at every grid point for Fermi level mu (one per thread).
__device__ void grid_g(FermiShared& sh, int n_e, double e0, double de, double mu, double kT, const double* coef,
                       bool final) {
    const int e = threadIdx.x;
    if (e < n_e) {
        double g0, g1, g2, f, s0, s1;
        gfun((e0 + e * de - mu) / kT, coef, final, g0, g1, g2, f, s0, s1);
        sh.g0[e] = g0;
        sh.g1[e] = g1;
        sh.g2[e] = g2;
        sh.f[e] = f;
        sh.s0[e] = s0;
        sh.s1[e] = s1;
    }
    __syncthreads();
}

// Hat-piece integrals over interval i = [e_i, e_i + de] from the shared G's:
// wl = int f (1-t), wr = int f t; vl, vr the same with f*e.
__device__ void interval(const FermiShared& sh, int i, double e0, double de, double mu, double kT, double& wl,
                         double& wr, double& vl, double& vr) {
    const double xa = (e0 + i * de - mu) / kT, D = de / kT;
    const double d0 = sh.g0[i + 1] - sh.g0[i], d1 = sh.g1[i + 1] - sh.g1[i], d2 = sh.g2[i + 1] - sh.g2[i];
    const double I0 = d0 * kT;
    const double I1 = (d1 - xa * d0) * kT / D;
    const double K0 = d1 * kT;
    const double K1 = (d2 - xa * d1) * kT / D;
    wl = I0 - I1;
    wr = I1;
    vl = mu * (I0 - I1) + (K0 - K1) * kT;
    vr = mu * I1 + K1 * kT;
}

// N(mu) and dN/dmu.  On [a, b] with t = (e-a)/de, int (-df/de) = f(a) - f(b)
// and int t (-df/de) = (kT/de)(G0(xb) - G0(xa)) - f(b).
__device__ void electrons(FermiShared& sh, int n_e, double e0, double de, double mu, double kT,
                          const double* coef, double& n, double& dn) {
    grid_g(sh, n_e, e0, de, mu, kT, coef, false);
    const int e = threadIdx.x;
    double c = 0.0, dc = 0.0;
    if (e < n_e - 1) {
        double wl, wr, vl, vr;
        interval(sh, e, e0, de, mu, kT, wl, wr, vl, vr);
        c = wl * sh.D[e] + wr * sh.D[e + 1];
        const double P = sh.f[e] - sh.f[e + 1];
        const double Q = kT / de * (sh.g0[e + 1] - sh.g0[e]) - sh.f[e + 1];
        dc = (P - Q) * sh.D[e] + Q * sh.D[e + 1];
    }
    n = block_sum(c, sh.red);
    dn = block_sum(dc, sh.red);
}

// Zero-temperature root of int_{e0}^{mu} D = n_target for the piecewise-linear
// D (a block scan of the trapezoids, then the quadratic on the crossing
// interval); the midpoint of the grid if the count never crosses.
__device__ double zero_t_root(FermiShared& sh, int n_e, double e0, double de, double n_target) {
    const int e = threadIdx.x;
    const double piece = e < n_e - 1 ? 0.5 * de * (sh.D[e] + sh.D[e + 1]) : 0.0;
    sh.cum[e] = piece;
    if (e == 0) sh.mu0 = e0 + 0.5 * (n_e - 1) * de;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {          // inclusive scan
        const double v = e >= off ? sh.cum[e - off] : 0.0;
        __syncthreads();
        sh.cum[e] += v;
        __syncthreads();
    }
    const double after = sh.cum[e], before = after - piece;
    const bool cross = e < n_e - 1 && before <= n_target && n_target < after;
    if (e == 0) sh.first = n_e;
    __syncthreads();
    if (cross) atomicMin(&sh.first, e);               // lowest crossing interval
    __syncthreads();
    if (e == sh.first) {
        // de (D0 t + (D1 - D0) t^2 / 2) = n_target - before, t in [0, 1]
        const double r = (n_target - before) / de, D0 = sh.D[e], k = sh.D[e + 1] - sh.D[e];
        const double den = D0 + sqrt(fmax(D0 * D0 + 2.0 * k * r, 0.0));
        const double t = den > 0.0 ? fmin(fmax(2.0 * r / den, 0.0), 1.0) : 0.5;
        sh.mu0 = e0 + (e + t) * de;
    }
    __syncthreads();
    return sh.mu0;
}

// mode 0: exact solve (DOS, result, weights; window coverage if win != NULL)
// mode 1: estimate from a subsample -> energy window for the stored LDOS
__global__ __launch_bounds__(256) void k_fermi(const double* __restrict__ partials, int n_parts, int n_e,
                                               double dV, double e0, double de, double kT, double n_target,
                                               double* __restrict__ dos_out, double* __restrict__ w_out,
                                               ResultRec* __restrict__ res, WindowRec* __restrict__ win,
                                               const double* __restrict__ coef, int mode, int w_max,
                                               double margin, const int* __restrict__ cap_err) {
    __shared__ FermiShared sh;
    const int e = threadIdx.x;
    double d = 0.0;
    if (e < n_e) {
        // eight independent running sums (loads in flight), combined in a fixed order
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int w = 0;
        for (; w + 8 <= n_parts; w += 8) {
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += partials[(size_t)(w + q) * kMlpMaxOut + e];
        }
        for (; w < n_parts; ++w) acc[0] += partials[(size_t)w * kMlpMaxOut + e];
        d = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        d *= dV;
        if (mode == 0) dos_out[e] = d;
    }
    sh.D[e] = d;
    __syncthreads();
    const double elast = e0 + (n_e - 1) * de;
    double nlo, nhi, dn;
    electrons(sh, n_e, e0, de, e0, kT, coef, nlo, dn);
    electrons(sh, n_e, e0, de, elast, kT, coef, nhi, dn);
    const bool ok = nlo <= n_target && n_target <= nhi;
    if (!ok) {
        if (e == 0) {
            if (mode == 0) {
                res->e_fermi = NAN;
                res->e_band = NAN;
                res->n_found = NAN;
                res->entropy = NAN;
                res->e_entropy = NAN;
                res->n_target = n_target;
                res->iterations = 0;
                res->status = (cap_err && *cap_err) ? -7 : -4;     // MALA_E_CAPACITY first, else MALA_E_NO_ROOT
                res->density_from_window = 0;
                if (win) win->covered = 0;
            } else {
                win->lo = 0;
                win->hi = n_e - 1;
                win->valid = 0;
                win->covered = 0;
                win->e_fermi_est = NAN;
            }
        }
        if (mode == 0 && e < n_e) w_out[e] = 0.0;
        return;
    }
    const double tol = mode == 0 ? 1e-12 : 1e-6;
    double lo = e0, hi = elast;
    double mu = zero_t_root(sh, n_e, e0, de, n_target);
    int it = 0;
    while (it < 200) {
        double n;
        electrons(sh, n_e, e0, de, mu, kT, coef, n, dn);
        ++it;
        if (n == n_target) break;                       // mu is the root
        if (n < n_target) lo = mu;
        else hi = mu;
        double nx = dn > 0.0 ? mu - (n - n_target) / dn : lo;
        // a converged step is taken as it is (it may round onto mu, i.e. onto
        // the end of the bracket just moved there); any other step that
        // leaves the bracket becomes the midpoint
        if (dn > 0.0 && fabs(nx - mu) <= 0.1 * tol) {
            mu = nx;
            break;
        }
        if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
        mu = nx;
        if (hi - lo < tol) break;
    }
    const double ef = mu;
    const double reach = 40.0 * kT;
    if (mode == 1) {
        if (e == 0) {
            int wl = (int)floor((ef - reach - margin - e0) / de), wh = (int)ceil((ef + reach + margin - e0) / de);
            wl = wl < 0 ? 0 : wl;
            wh = wh > n_e - 1 ? n_e - 1 : wh;
            win->lo = wl;
            win->hi = wh;
            win->valid = (wh - wl + 1) <= w_max ? 1 : 0;
            win->covered = 0;
            win->e_fermi_est = ef;
        }
        return;
    }
    grid_g(sh, n_e, e0, de, ef, kT, coef, true);
    double wl = 0, wr = 0, vl = 0, vr = 0, sc = 0;
    if (e < n_e - 1) {
        interval(sh, e, e0, de, ef, kT, wl, wr, vl, vr);
        // entropy (Eq. electronicentropyDOS) on the same hat pieces: int s,
        // int s t over the interval, t = (x - xa)/D
        const double xa = (e0 + e * de - ef) / kT, xb = (e0 + (e + 1) * de - ef) / kT, D = de / kT;
        double d0 = sh.s0[e + 1] - sh.s0[e];
        if (xa <= 0.0 && xb > 0.0) d0 += kPi * kPi / 3.0;
        const double J0 = d0 * kT, J1 = (sh.s1[e + 1] - sh.s1[e] - xa * d0) * kT / D;
        sc = (J0 - J1) * sh.D[e] + J1 * sh.D[e + 1];
    }
    const double s_kb = block_sum(sc, sh.red);
    __syncthreads();
    // reuse the g arrays for the per-interval pieces
    sh.g0[e] = wr;
    sh.g1[e] = vr;
    __syncthreads();
    double we = 0.0, ve = 0.0;
    if (e < n_e) {
        if (e < n_e - 1) { we += wl; ve += vl; }
        if (e >= 1) { we += sh.g0[e - 1]; ve += sh.g1[e - 1]; }
        w_out[e] = we;
    }
    const double nf = block_sum(we * sh.D[e], sh.red);
    const double eb = block_sum(ve * sh.D[e], sh.red);
    if (e == 0) {
        res->e_fermi = ef;
        res->e_band = eb;
        res->n_found = nf;
        res->entropy = s_kb;
        res->e_entropy = -kT * s_kb;
        res->n_target = n_target;
        res->iterations = it;
        res->status = (cap_err && *cap_err) ? -7 : 0;     // MALA_E_CAPACITY: neighbour lists were truncated
        res->density_from_window = 0;
        if (win) {
            const bool lo_ok = win->lo == 0 || e0 + win->lo * de <= ef - reach;
            const bool hi_ok = win->hi == n_e - 1 || e0 + win->hi * de >= ef + reach;
            win->covered = (win->valid && lo_ok && hi_ok) ? 1 : 0;
            res->density_from_window = win->covered;
        }
    }
}

// n(p) = prefix(p) + sum over the stored window of w_e d_e(p), when the
// window covers E_F +- 40 kT (outside it the Fermi weights equal the full
// trapezoid weights or vanish to within e^-40).
// n(p) = prefix(p) + sum over the window of w_e d_e(p).  A wave takes 64
// points at a time: their window rows are 64 W contiguous floats, read with
// consecutive lanes into LDS (row stride W: coalesced, where one lane per row
// strides W floats between the lanes of every load) and then summed by the
// row's lane in the fixed order of the energies (a tile's rows start on a
// 256 W-byte boundary, so the copy moves 16 bytes per lane).  The block's four waves
// move in step so that the staging area can be reused after a barrier.
// Windows wider than w_stage (the LDS the host gave, per point) are summed
// straight from memory.
__global__ __launch_bounds__(256) void k_density_window(const double* __restrict__ prefix,
                                                        const float* __restrict__ window, int64_t n_pts,
                                                        const WindowRec* __restrict__ win,
                                                        const ResultRec* __restrict__ res,
                                                        const double* __restrict__ w, double* __restrict__ dens,
                                                        int w_stage) {
    if (res->status != 0 || !win->covered) return;
    __shared__ double sw[kMlpMaxOut];
    extern __shared__ float srow[];                      // [4 waves][64 rows][w_stage]
    const int lo = win->lo, W = win->hi - win->lo + 1;
    for (int i = threadIdx.x; i < W; i += blockDim.x) sw[i] = w[lo + i];
    __syncthreads();
    if (W > w_stage) {
        for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pts;
             p += (int64_t)gridDim.x * blockDim.x) {
            double s = prefix[p];
            const float* row = window + p * W;
            for (int i = 0; i < W; ++i) s += sw[i] * (double)row[i];
            dens[p] = s;
        }
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float* rows = srow + wave * 64 * w_stage;
    for (int64_t t0 = (int64_t)blockIdx.x * 4; t0 * 64 < n_pts; t0 += (int64_t)gridDim.x * 4) {
        const int64_t p0 = (t0 + wave) * 64;
        const int np = p0 < n_pts ? (int)(n_pts - p0 < 64 ? n_pts - p0 : 64) : 0;
        // 64 W floats from 256 W-byte aligned rows: 16-byte loads, a few in flight
        const float* src = window + p0 * W;
        const int nf = np * W, n4 = nf >> 2;
        const float4* src4 = reinterpret_cast<const float4*>(src);
        float4* rows4 = reinterpret_cast<float4*>(rows);
#pragma unroll 4
        for (int i = lane; i < n4; i += 64) rows4[i] = src4[i];
        for (int i = (n4 << 2) + lane; i < nf; i += 64) rows[i] = src[i];
        __syncthreads();
        if (lane < np) {
            double s = prefix[p0 + lane];
            for (int i = 0; i < W; ++i) s += sw[i] * (double)rows[lane * W + i];
            dens[p0 + lane] = s;
        }
        __syncthreads();
    }
}

// Column sums of a stored LDOS [n][n_e] into FP64 partial rows, one per block
// over a fixed contiguous range of points.
__global__ __launch_bounds__(256) void k_ldos_colsum(const float* __restrict__ ldos, int64_t n_pts, int n_e,
                                                     double* __restrict__ partials, int n_blocks) {
    const int e = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t p_begin = n_pts * b / n_blocks, p_end = n_pts * (b + 1) / n_blocks;
    double s = 0.0;
    if (e < n_e)
        for (int64_t p = p_begin; p < p_end; ++p) s += (double)ldos[p * n_e + e];
    partials[b * kMlpMaxOut + e] = e < n_e ? s : 0.0;
}

// n(p) = sum_e w_e d_e(p), one wave per point (grid-stride).
__global__ __launch_bounds__(256) void k_density_ldos(const float* __restrict__ ldos, int64_t n_pts, int n_e,
                                                      const double* __restrict__ w,
                                                      const ResultRec* __restrict__ res,
                                                      double* __restrict__ dens) {
    if (res->status != 0) return;
    const int lane = threadIdx.x & 63;
    double wr[4];
    for (int q = 0; q < 4; ++q) wr[q] = (lane + 64 * q < n_e) ? w[lane + 64 * q] : 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); p < n_pts; p += (int64_t)gridDim.x * 4) {
        double s = 0.0;
        for (int q = 0; q < 4; ++q) {
            const int e = lane + 64 * q;
            if (e < n_e) s += wr[q] * (double)ldos[p * n_e + e];
        }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) dens[p] = s;
    }
}

hipError_t launch_fermi(hipStream_t s, const double* partials, int n_parts, int n_e, double dV, double e0,
                        double de, double kT, double n_target, double* dos_out, double* weights_out,
                        void* result, WindowRec* win, const double* li_coef, const int* cap_err) {
    hipLaunchKernelGGL(k_fermi, dim3(1), dim3(256), 0, s, partials, n_parts, n_e, dV, e0, de, kT, n_target,
                       dos_out, weights_out, static_cast<ResultRec*>(result), win, li_coef, 0, 0, 0.0, cap_err);
    return hipGetLastError();
}

hipError_t launch_fermi_estimate(hipStream_t s, const double* partials, int n_parts, int n_e, double dV,
                                 double e0, double de, double kT, double n_target, WindowRec* win,
                                 const double* li_coef, int w_max, double margin) {
    hipLaunchKernelGGL(k_fermi, dim3(1), dim3(256), 0, s, partials, n_parts, n_e, dV, e0, de, kT, n_target,
                       nullptr, nullptr, nullptr, win, li_coef, 1, w_max, margin, nullptr);
    return hipGetLastError();
}

hipError_t launch_density_window(hipStream_t s, const double* prefix, const float* window, int64_t n_pts,
                                 const WindowRec* win, const void* result, const double* weights,
                                 double* density, int w_max) {
    int64_t blocks = (n_pts + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) return hipSuccess;
    // stage up to 96 energies per point (96 KB of LDS per block); wider
    // windows (high temperatures on fine energy grids) take the direct path
    const int w_stage = w_max <= kDensityStageMax ? (w_max > 0 ? w_max : 1) : 0;
    const size_t lds = sizeof(float) * 256 * (size_t)w_stage;
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(attr_once, [] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_density_window),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(float) * 256 * kDensityStageMax));
    });
    if (attr_err != hipSuccess) return attr_err;
    hipLaunchKernelGGL(k_density_window, dim3((unsigned)blocks), dim3(256), lds, s, prefix, window, n_pts, win,
                       static_cast<const ResultRec*>(result), weights, density, w_stage);
    return hipGetLastError();
}

hipError_t launch_ldos_colsum(hipStream_t s, const float* ldos, int64_t n_pts, int n_e, double* partials,
                              int n_blocks) {
    hipLaunchKernelGGL(k_ldos_colsum, dim3(n_blocks), dim3(256), 0, s, ldos, n_pts, n_e, partials, n_blocks);
    return hipGetLastError();
}

hipError_t launch_density_from_ldos(hipStream_t s, const float* ldos, int64_t n_pts, int n_e,
                                    const double* weights, const void* result, double* density) {
    int64_t blocks = (n_pts + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(k_density_ldos, dim3((unsigned)blocks), dim3(256), 0, s, ldos, n_pts, n_e, weights,
                       static_cast<const ResultRec*>(result), density);
    return hipGetLastError();
}

// Taylor coefficients of Li_s(-e^t) about t = 0 for s = 2, 3, then the
// inverse powers 1/k^s used by the power series:
// c_{s,n} = Li_{s-n}(-1)/n! = -eta(s-n)/n!, with eta(1) = ln 2,
// eta(2) = pi^2/12, eta(3) = 3 zeta(3)/4 and, for m >= 0,
// eta(-m) = (2^(m+1) - 1) B_{m+1}/(m+1) (B_1 = +1/2; B_{2k} from zeta(2k)).
void polylog_coefficients(double* coef) {
    for (int si = 0; si < 2; ++si)
        for (int k = 0; k < kLiPow; ++k)
            coef[2 * kLiTerms + si * kLiPow + k] = k == 0 ? 0.0 : pow((double)k, -(double)(2 + si));
    auto zeta_even = [](int n) {     // zeta(n), n >= 2 even: sum plus integral tail
        if (n == 2) return kPi * kPi / 6.0;
        const int K = 2000;
        double s = pow((double)K, 1.0 - n) / (n - 1) - 0.5 * pow((double)K, -(double)n);
        for (int k = K - 1; k >= 1; --k) s += pow((double)k, -(double)n);
        return s;
    };
    auto bernoulli = [&](int n) {    // B_n with B_1 = +1/2
        if (n == 0) return 1.0;
        if (n == 1) return 0.5;
        if (n & 1) return 0.0;
        double f = 1.0;
        for (int k = 2; k <= n; ++k) f *= k;
        const double sign = ((n / 2) & 1) ? 1.0 : -1.0;      // (-1)^(n/2+1)
        return sign * 2.0 * f * zeta_even(n) / pow(2.0 * kPi, n);
    };
    auto eta = [&](int s) {
        if (s == 1) return log(2.0);
        if (s == 2) return kPi * kPi / 12.0;
        if (s == 3) return 0.75 * 1.2020569031595942854;   // zeta(3) (Apery's constant)
        const int m = -s;                                      // s <= 0
        return (pow(2.0, m + 1) - 1.0) * bernoulli(m + 1) / (m + 1);
    };
    for (int si = 0; si < 2; ++si) {
        const int s = 2 + si;
        double fact = 1.0;
        for (int n = 0; n < kLiTerms; ++n) {
            if (n > 0) fact *= n;
            coef[si * kLiTerms + n] = -eta(s - n) / fact;
        }
    }
}

}  // namespace mala
