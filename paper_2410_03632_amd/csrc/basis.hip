// Cosmology-independent basis (Eq. t_tilde), computed once per plan on the GPU in FP64:
//
//   Ttilde[a][b][t][l][n] = sum_q v_q f_t(k_q) T_n(x(k_q)) j_l(k_q chi_a) j_l(k_q R_b chi_a)
//
// The k-integral over [k_min, k_max] is a composite 16-point Gauss-Legendre rule.  For each
// chi_a the coarse panels are uniform in theta = arccos(x) (they resolve T_n near both ends
// of the ln-k range) and each is split into equal k sub-panels so that the Bessel phase
// (chi_a + R_b chi_a) dk across one sub-panel stays below `kq_phase` (8 by default, where
// 16-point Gauss-Legendre is accurate far below 1e-12 for a pure oscillation).  The nodes
// depend on a only, so j_l(k chi_a) is shared by every R_b.
//
// Per launch, up to G items (distinct a, one chunk of <= Qc nodes each) go through
//   tq_kernel      : T_n(x_q) (three-term recurrence), v_q f_t(k_q), k_q
//   bessel_kernel  : j_l(k_q chi) for chi in {chi_a, R_b chi_a} and the plan's multipoles
//   gemm_kernel    : Ttilde += sum_q [v f_t j j]_q,l * T_n(x_q)   (FP64 MFMA 16x16x4)
// and the chunk sums accumulate in the resident FP64 basis.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace blast {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kG = 4;        // items per launch
constexpr int kQc = 4096;    // nodes per item
constexpr int kMaxTypes = 3;

__constant__ double c_glx[16];
__constant__ double c_glw[16];

struct Items {
    int a[kG];
    int p0[kG];   // first sub-panel of the item
    int nq[kG];   // nodes in the item (<= kQc)
    int n;        // number of items
};

// ---------------------------------------------------------------------------------------------
// j_l(x) for increasing multipoles ell[0..nl) (all >= 2), x > 0.
//  x >= lmax : upward three-term recurrence from j_0, j_1 (stable below the turning point).
//  x <  lmax : upward to m = floor(x), then Miller's downward recurrence from a start L where
//              the Debye exponent nu (alpha - tanh alpha), cosh alpha = nu/x, reaches 100
//              (j_L / j_m ~ e^-100, so the start error is invisible and nothing overflows),
//              normalised to the upward value j_m(x) > 0 (x < m+1 lies before j_m's first zero).
// Orders above L are set to zero (they are below e^-70 of the turning-point amplitude).
// ---------------------------------------------------------------------------------------------
// Order nu > x at which the Debye exponent nu (alpha - tanh alpha), cosh alpha = nu / x, reaches
// 100: Newton from above (the exponent is convex in nu with derivative alpha).
__device__ double miller_start(double x) {
    double nu = x + 10.0 + 25.0 * cbrt(x + 8.0);
    for (int it = 0; it < 12; ++it) {
        const double al = acosh(nu / x);
        const double a2 = al * al;
        const double E = al < 0.1 ? nu * al * a2 * (1.0 / 3.0 - a2 * (2.0 / 15.0 - a2 * (17.0 / 315.0)))
                                  : nu * (al - tanh(al));
        const double d = (E - 100.0) / al;
        nu -= d;
        if (nu < x + 1e-3) nu = x + 1e-3;
        if (fabs(d) < 0.25) break;
    }
    return nu;
}

__device__ void bessel_list(double x, const int *__restrict__ ell, int nl, double *__restrict__ out) {
    const int lmax = ell[nl - 1];
    double sx, cx;
    sincos(x, &sx, &cx);
    const double inv = 1.0 / x;
    const double j0 = sx * inv;
    if (x >= (double)lmax) {
        double jm = j0, jc = (j0 - cx) * inv;  // j_0, j_1
        int il = 0, next = ell[0];
        for (int l = 1; il < nl; ++l) {
            const double jn = (2.0 * l + 1.0) * inv * jc - jm;
            jm = jc;
            jc = jn;
            if (l + 1 == next) {
                out[il] = jc;
                ++il;
                next = il < nl ? ell[il] : -1;
            }
        }
        return;
    }
    const int m = (int)x;
    int il = 0;
    double jmv;
    if (m == 0) {
        jmv = j0;
    } else {
        double a0 = j0, a1 = (j0 - cx) * inv;  // x >= 1 here
        int next = ell[0];
        for (int l = 1; l < m; ++l) {
            const double an = (2.0 * l + 1.0) * inv * a1 - a0;
            a0 = a1;
            a1 = an;
            if (l + 1 == next) {
                out[il] = a1;
                ++il;
                next = il < nl ? ell[il] : 1 << 30;
            }
        }
        jmv = a1;
    }
    int L = (int)ceil(miller_start(x)) + 2;
    if (L < m + 2) L = m + 2;
    int ih = nl - 1;
    while (ih >= il && ell[ih] > L) {
        out[ih] = 0.0;
        --ih;
    }
    double yp = 0.0, y = 1.0;  // y_{l+1}, y_l
    int nxt = ih >= il ? ell[ih] : -1;
    for (int l = L; l > m; --l) {
        if (l == nxt) {
            out[ih] = y;
            --ih;
            nxt = ih >= il ? ell[ih] : -1;
        }
        const double yn = (2.0 * l + 1.0) * inv * y - yp;
        yp = y;
        y = yn;
    }
    const double scale = jmv / y;  // y = y_m
    for (int q = il; q < nl && ell[q] <= L; ++q) out[q] *= scale;
}

// ---------------------------------------------------------------------------------------------
// j_nu(x) for real multipoles nu (not all integers), x > 0.  The multipoles are taken in runs of
// equal fractional part mu, members mu + n with increasing n (run r: ell[perm[runs[r] ..
// runs[r+1])]); one run is one recurrence over the orders mu + i, as for integer orders:
//  x >= kHankelX : j_mu and j_{mu+1} from Hankel's expansion for large argument (DLMF 10.17.3,
//                  cylindrical order a = mu + 1/2), then upward to m = floor(x - mu) and, for
//                  members above m, Miller's downward recurrence from the Debye start,
//                  normalised to the upward value at m (positive: x < mu + m + 1 lies before the
//                  first zero of j_{mu+m}).
//  x <  kHankelX : Miller's downward recurrence from the Debye start to order mu, normalised by
//                  Neumann's series (x/2)^a / Gamma(a) = sqrt(2x/pi) sum_k (a+2k) r_k j_{mu+2k}(x),
//                  r_k = Gamma(a+k) / (Gamma(a) k!) (DLMF 10.23), with the r_k generated downwards
//                  from an arbitrary top value and divided by the r_0 they reach.
// Orders above the Debye start are set to zero, as on the integer path.
// ---------------------------------------------------------------------------------------------
constexpr double kHankelX = 30.0;

// P and Q of Hankel's expansion of J_a(x): t_k = t_{k-1} (4a^2 - (2k-1)^2) / (8 k x),
// P = t_0 - t_2 + t_4 - ..., Q = t_1 - t_3 + ...; for x >= 30 and a < 2 the terms fall below
// 1e-17 before k = 40, well ahead of the smallest term (k ~ 2x).
__device__ void hankel_pq(double a, double x, double &P, double &Q) {
    const double a4 = 4.0 * a * a, i8x = 1.0 / (8.0 * x);
    double t = 1.0;
    P = 1.0;
    Q = 0.0;
    for (int k = 1; k < 48; ++k) {
        t *= (a4 - (2.0 * k - 1.0) * (2.0 * k - 1.0)) * i8x / k;
        const double s = ((k >> 1) & 1) ? -t : t;  // sign (-1)^floor(k/2)
        if (k & 1)
            Q += s;
        else
            P += s;
        if (fabs(t) < 1e-17) break;
    }
}

__device__ void bessel_run(double x, double sx, double cx, double Lnu, double mu, const double *__restrict__ ell,
                           const int *__restrict__ perm, int r0, int r1, double *__restrict__ out) {
    const double inv = 1.0 / x;
    const int itop0 = (int)ceil(Lnu - mu) + 2;
    int hi = r1 - 1;  // members above the start are zero
    while (hi >= r0 && (int)floor(ell[perm[hi]]) > itop0) {
        out[perm[hi]] = 0.0;
        --hi;
    }
    if (hi < r0) return;
    if (x < kHankelX) {
        const double a = mu + 0.5;
        int itop = itop0 + (itop0 & 1);  // even: the series terms sit on even i
        double yp = 0.0, y = 1.0, rk = 1.0, sum = 0.0;
        int q = hi;
        for (int i = itop; i >= 0; --i) {
            if (q >= r0 && (int)floor(ell[perm[q]]) == i) {
                out[perm[q]] = y;
                --q;
            }
            if (!(i & 1)) {
                const int k = i >> 1;
                sum += (a + 2.0 * k) * rk * y;
                if (k) rk *= k / (a + k - 1.0);
            }
            if (i) {
                const double yn = (2.0 * (mu + i) + 1.0) * inv * y - yp;
                yp = y;
                y = yn;
            }
        }
        const double scale = exp(a * log(0.5 * x) - lgamma(a)) / (sqrt(2.0 * x / M_PI) * (sum / rk));
        for (int u = r0; u <= hi; ++u) out[perm[u]] *= scale;
        return;
    }
    // seeds from Hankel's expansion: w = x - (mu + 1) pi / 2
    double sph, cph;
    sincos(0.5 * M_PI * (mu + 1.0), &sph, &cph);
    const double cw = cx * cph + sx * sph, sw = sx * cph - cx * sph;
    double P0, Q0, P1, Q1;
    hankel_pq(mu + 0.5, x, P0, Q0);
    hankel_pq(mu + 1.5, x, P1, Q1);
    double a0 = (P0 * cw - Q0 * sw) * inv;  // j_mu
    double a1 = (P1 * sw + Q1 * cw) * inv;  // j_{mu+1}
    const int m = (int)floor(x - mu);
    int q = r0;
    auto take = [&](int i, double v) {
        while (q <= hi && (int)floor(ell[perm[q]]) == i) {
            out[perm[q]] = v;
            ++q;
        }
    };
    take(0, a0);
    take(1, a1);
    const int nup = min((int)floor(ell[perm[hi]]), m);
    for (int i = 1; i < nup; ++i) {
        const double an = (2.0 * (mu + i) + 1.0) * inv * a1 - a0;
        a0 = a1;
        a1 = an;
        take(i + 1, a1);
    }
    if (q > hi) return;
    // members above m: Miller from the start down to m, normalised to j_{mu+m} from above
    const double jm = nup >= 1 ? a1 : a0;  // nup = m here (m >= 29)
    const int itop = max(itop0, m + 2);
    double yp = 0.0, y = 1.0;
    int u = hi;
    for (int i = itop; i > m; --i) {
        if (u >= q && (int)floor(ell[perm[u]]) == i) {
            out[perm[u]] = y;
            --u;
        }
        const double yn = (2.0 * (mu + i) + 1.0) * inv * y - yp;
        yp = y;
        y = yn;
    }
    const double scale = jm / y;
    for (int v = q; v <= hi; ++v) out[perm[v]] *= scale;
}

// J[g][s][q][ilp] for a plan with non-integer multipoles (layout as bessel_kernel)
__global__ __launch_bounds__(256) void bessel_real_kernel(Items it, const double *__restrict__ Kq,
                                                          const double *__restrict__ chi, const double *__restrict__ R,
                                                          int S, const double *__restrict__ ell,
                                                          const int *__restrict__ perm, const int *__restrict__ runs,
                                                          int nruns, int nl, int ilp, double *__restrict__ J) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y, g = blockIdx.z;
    if (q >= kQc || g >= it.n) return;
    double *out = J + (((size_t)g * S + s) * kQc + q) * ilp;
    const double k = Kq[(size_t)g * kQc + q];
    if (q >= it.nq[g] || k <= 0.0) {
        for (int il = 0; il < ilp; ++il) out[il] = 0.0;
        return;
    }
    const double x = k * chi[it.a[g]] * (s == 0 ? 1.0 : R[s - 1]);
    double sx, cx;
    sincos(x, &sx, &cx);
    const double Lnu = miller_start(x);
    for (int r = 0; r < nruns; ++r) {
        const double l0 = ell[perm[runs[r]]];
        bessel_run(x, sx, cx, Lnu, l0 - floor(l0), ell, perm, runs[r], runs[r + 1], out);
    }
    for (int il = nl; il < ilp; ++il) out[il] = 0.0;
}

// node tables of one launch: Tq[g][q][n], Fq[g][q][3], Kq[g][q]
__global__ __launch_bounds__(256) void tq_kernel(Items it, const double2 *__restrict__ panels, double lnkmin,
                                                 double span, int n_cheb, int ncp, int nt, int t0, int t1, int t2,
                                                 double *__restrict__ Tq, double *__restrict__ Fq,
                                                 double *__restrict__ Kq) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (q >= kQc || g >= it.n) return;
    double *T = Tq + ((size_t)g * kQc + q) * ncp;
    double *F = Fq + ((size_t)g * kQc + q) * kMaxTypes;
    if (q >= it.nq[g]) {
        for (int n = 0; n < ncp; ++n) T[n] = 0.0;
        F[0] = F[1] = F[2] = 0.0;
        Kq[(size_t)g * kQc + q] = 0.0;
        return;
    }
    const double2 pk = panels[it.p0[g] + q / 16];
    const int node = q % 16;
    const double mid = 0.5 * (pk.x + pk.y), half = 0.5 * (pk.y - pk.x);
    const double k = mid + half * c_glx[node];
    const double v = half * c_glw[node];
    const double x = 2.0 * (log(k) - lnkmin) / span - 1.0;
    double tm = 1.0, tc = x;
    T[0] = 1.0;
    if (n_cheb > 1) T[1] = x;
    for (int n = 2; n < n_cheb; ++n) {
        const double tn = 2.0 * x * tc - tm;
        tm = tc;
        tc = tn;
        T[n] = tn;
    }
    for (int n = n_cheb; n < ncp; ++n) T[n] = 0.0;
    const int tb[3] = {t0, t1, t2};
    for (int s = 0; s < kMaxTypes; ++s) {
        double f = 0.0;
        if (s < nt) f = tb[s] == BLAST_GG ? k * k : (tb[s] == BLAST_GS ? 1.0 : 1.0 / (k * k));
        F[s] = v * f;
    }
    Kq[(size_t)g * kQc + q] = k;
}

// J[g][s][q][ilp]: s = 0 -> chi_a, s = 1 + b -> R_b chi_a
__global__ __launch_bounds__(256) void bessel_kernel(Items it, const double *__restrict__ Kq,
                                                     const double *__restrict__ chi, const double *__restrict__ R,
                                                     int S, const int *__restrict__ ell, int nl, int ilp,
                                                     double *__restrict__ J) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y, g = blockIdx.z;
    if (q >= kQc || g >= it.n) return;
    double *out = J + (((size_t)g * S + s) * kQc + q) * ilp;
    const double k = Kq[(size_t)g * kQc + q];
    if (q >= it.nq[g] || k <= 0.0) {
        for (int il = 0; il < ilp; ++il) out[il] = 0.0;
        return;
    }
    const double c = chi[it.a[g]] * (s == 0 ? 1.0 : R[s - 1]);
    bessel_list(k * c, ell, nl, out);
    for (int il = nl; il < ilp; ++il) out[il] = 0.0;
}

// Ttilde[a][b][slot*n_ell + l][n] += sum_q (v f_slot j_l(k chi_a) j_l(k R_b chi_a))_q T_n(x_q)
// grid (ilp/32, n_R, items), 4 waves; wave w owns n-tiles w and w+4 for both 16-row l-tiles and
// every type slot: 12 FP64 16x16 accumulators.  v_mfma_f64_16x16x4f64 lane layout: A[i][k] and
// B[k][j] in lane i (or j) + 16k; D[i][j] in register r of lane j + 16*(i%4), r = i/4.
__global__ __launch_bounds__(256) void gemm_kernel(Items it, const double *__restrict__ J,
                                                   const double *__restrict__ Tq, const double *__restrict__ Fq,
                                                   int S, int ilp, int ncp, int n_ell, int nt, int nR, int rows_pad,
                                                   double *__restrict__ basis) {
    const int g = blockIdx.z, b = blockIdx.y, il0 = blockIdx.x * 32;
    if (g >= it.n) return;
    const int a = it.a[g], nq = it.nq[g];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int ntiles = ncp >> 4;
    d4 acc[kMaxTypes][2][2];
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[t][m][j] = d4{0.0, 0.0, 0.0, 0.0};
    const double *J0 = J + ((size_t)g * S) * kQc * ilp;
    const double *Jb = J + ((size_t)g * S + 1 + b) * kQc * ilp;
    const double *T = Tq + (size_t)g * kQc * ncp;
    const double *F = Fq + (size_t)g * kQc * kMaxTypes;
    const bool has0 = w < ntiles, has1 = w + 4 < ntiles;
    const int nsteps = (nq + 3) >> 2;
    for (int st = 0; st < nsteps; ++st) {
        const int q = 4 * st + lk;
        double p0 = 0.0, p1 = 0.0, f[kMaxTypes] = {0.0, 0.0, 0.0}, tv0 = 0.0, tv1 = 0.0;
        if (q < nq) {
            const double *j0 = J0 + (size_t)q * ilp + il0;
            const double *jb = Jb + (size_t)q * ilp + il0;
            p0 = j0[lr] * jb[lr];
            p1 = j0[16 + lr] * jb[16 + lr];
#pragma unroll
            for (int t = 0; t < kMaxTypes; ++t) f[t] = F[(size_t)q * kMaxTypes + t];
            if (has0) tv0 = T[(size_t)q * ncp + 16 * w + lr];
            if (has1) tv1 = T[(size_t)q * ncp + 16 * (w + 4) + lr];
        }
#pragma unroll
        for (int t = 0; t < kMaxTypes; ++t) {
            if (t < nt) {
                const double a0 = p0 * f[t], a1 = p1 * f[t];
                acc[t][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, tv0, acc[t][0][0], 0, 0, 0);
                acc[t][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, tv0, acc[t][1][0], 0, 0, 0);
                if (ntiles > 4) {
                    acc[t][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, tv1, acc[t][0][1], 0, 0, 0);
                    acc[t][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, tv1, acc[t][1][1], 0, 0, 0);
                }
            }
        }
    }
    const size_t base = ((size_t)a * nR + b) * rows_pad;
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t) {
        if (t >= nt) continue;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const bool ok = j == 0 ? has0 : has1;
                if (!ok) continue;
                const int n = 16 * (w + 4 * j) + lr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int il = il0 + 16 * m + lk + 4 * r;  // FP64 16x16 output: row lane/16 + 4r
                    if (il < n_ell) basis[(base + (size_t)t * n_ell + il) * ncp + n] += acc[t][m][j][r];
                }
            }
    }
}

// FP32 copy in the tiled layout (src row-major [point][rows_pad][ncp])
__global__ void to_f32_kernel(const double *__restrict__ src, float *__restrict__ dst, size_t n, int rows_pad,
                              int ncp) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t blk = (size_t)rows_pad * ncp;
    const size_t pt = i / blk, rem = i % blk;
    const int row = (int)(rem / ncp), col = (int)(rem % ncp);
    dst[pt * blk + tiled_off(row, col, ncp / 16, 4)] = (float)src[i];
}

// FP32 copy of the transposed basis per point (Ttilde^T: n the row, the basis row the column) in the
// tiled layout, the A operand of the transposed contraction of the adjoint
__global__ void to_f32t_kernel(const double *__restrict__ src, float *__restrict__ dst, size_t n, int rows_pad,
                               int ncp) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t blk = (size_t)rows_pad * ncp;
    const size_t pt = i / blk, rem = i % blk;
    const int row = (int)(rem / ncp), col = (int)(rem % ncp);
    dst[pt * blk + tiled_off(col, row, rows_pad / 16, 4)] = (float)src[i];
}

__device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// one wave per basis row: power-of-two scale, BF16 hi and (optionally) lo parts, tiled layout
__global__ __launch_bounds__(256) void to_bf16_kernel(const double *__restrict__ src, size_t nrows, int rows_pad,
                                                      int ncp, uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                                                      float *__restrict__ scale) {
    const size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;
    const double *r = src + row * ncp;
    double mx = 0.0;
    for (int n = lane; n < ncp; n += 64) mx = fmax(mx, fabs(r[n]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    const double sc = mx > 0.0 ? ldexp(1.0, ilogb(mx) + 1) : 1.0;  // |value / sc| < 1
    if (lane == 0) scale[row] = (float)sc;
    const size_t base = (row / rows_pad) * (size_t)rows_pad * ncp;
    const int rr = (int)(row % rows_pad);
    for (int n = lane; n < ncp; n += 64) {
        const double v = r[n] / sc;
        const uint16_t h = f32_to_bf16_rne((float)v);
        const size_t o = base + tiled_off(rr, n, ncp / 32, 8);
        hi[o] = h;
        if (lo) lo[o] = f32_to_bf16_rne((float)(v - (double)bf16_to_f32(h)));
    }
}

// one wave per basis row: a power-of-two scale that puts the row's largest magnitude in
// [2^14, 2^15) (FP16's normal range, below its largest finite value), then FP16 hi = fp16(v) and
// lo = fp16(v - hi) of v = value / scale, tiled layout
__global__ __launch_bounds__(256) void to_fp16_kernel(const double *__restrict__ src, size_t nrows, int rows_pad,
                                                      int ncp, uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                                                      float *__restrict__ scale) {
    const size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;
    const double *r = src + row * ncp;
    double mx = 0.0;
    for (int n = lane; n < ncp; n += 64) mx = fmax(mx, fabs(r[n]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    const double sc = mx > 0.0 ? ldexp(1.0, ilogb(mx) - 14) : 1.0;
    if (lane == 0) scale[row] = (float)sc;
    const size_t base = (row / rows_pad) * (size_t)rows_pad * ncp;
    const int rr = (int)(row % rows_pad);
    for (int n = lane; n < ncp; n += 64) {
        const double v = r[n] / sc;
        const _Float16 h = (_Float16)(float)v;
        const size_t o = base + tiled_off(rr, n, ncp / 32, 8);
        hi[o] = __builtin_bit_cast(uint16_t, h);
        lo[o] = __builtin_bit_cast(uint16_t, (_Float16)(float)(v - (double)(float)h));
    }
}

__device__ inline double readlane_f64(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The nodal basis: B[row][j] = sum_n Ttilde[row][n] D[n][j] with D the DCT-II matrix of Eq. dft
// (c_n = sum_j D[n][j] P_j), so that sum_j B[row][j] P_j = sum_n Ttilde[row][n] c_n (Eq. pmd): the
// projection applied once to the basis instead of to every P.  FP64 sums in n order, then
// (OUT 16) the FP16 hi + lo split of to_fp16_kernel (row scale, tiled layout), (OUT 32) the FP32
// copy of to_f32_kernel, (OUT 33) the FP32 transpose of to_f32t_kernel (B^T, for the adjoint) or
// (OUT 64) FP64 in the FP64 basis' row-major layout; column j = k node j, zero past n_cheb.  D sits in LDS; one wave per basis row (grid-stride over all rows of all
// points), lane L making columns L and L + 64, the row's Ttilde values broadcast one per step
// from the lane that loaded them.
template <int OUT>
__global__ __launch_bounds__(256) void to_nodal_kernel(const double *__restrict__ src, const double *__restrict__ dctn,
                                                       size_t nrows, int rows_pad, int ncp, int N,
                                                       uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                                                       float *__restrict__ scale, float *__restrict__ f32,
                                                       double *__restrict__ f64) {
    __shared__ double Dl[kMaxCheb * kMaxCheb];  // [n][j], ncp x ncp
    for (int i = threadIdx.x; i < ncp * ncp; i += blockDim.x) {
        const int n = i / ncp, j = i % ncp;
        Dl[i] = (n < N && j < N) ? dctn[(size_t)n * N + j] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const bool c0 = lane < ncp, c1 = lane + 64 < ncp;
    for (size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < nrows; row += (size_t)gridDim.x * 4) {
        const double *r = src + row * ncp;
        const double t0 = c0 ? r[lane] : 0.0, t1 = c1 ? r[lane + 64] : 0.0;
        double a0 = 0.0, a1 = 0.0;
        for (int n = 0; n < ncp; ++n) {
            const double tn = readlane_f64(n < 64 ? t0 : t1, n & 63);
            if (c0) a0 = fma(tn, Dl[n * ncp + lane], a0);
            if (c1) a1 = fma(tn, Dl[n * ncp + lane + 64], a1);
        }
        const size_t base = (row / rows_pad) * (size_t)rows_pad * ncp;
        const int rr = (int)(row % rows_pad);
        if constexpr (OUT == 32) {
            if (c0) f32[base + tiled_off(rr, lane, ncp / 16, 4)] = (float)a0;
            if (c1) f32[base + tiled_off(rr, lane + 64, ncp / 16, 4)] = (float)a1;
            continue;
        }
        if constexpr (OUT == 33) {
            if (c0) f32[base + tiled_off(lane, rr, rows_pad / 16, 4)] = (float)a0;
            if (c1) f32[base + tiled_off(lane + 64, rr, rows_pad / 16, 4)] = (float)a1;
            continue;
        }
        if constexpr (OUT == 64) {
            if (c0) f64[row * ncp + lane] = a0;
            if (c1) f64[row * ncp + lane + 64] = a1;
            continue;
        }
        double mx = fmax(fabs(a0), fabs(a1));
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
        const double sc = mx > 0.0 ? ldexp(1.0, ilogb(mx) - 14) : 1.0;
        if (lane == 0) scale[row] = (float)sc;
        for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * h;
            if (j >= ncp) continue;
            const double v = (h ? a1 : a0) / sc;
            const _Float16 x = (_Float16)(float)v;
            const size_t o = base + tiled_off(rr, j, ncp / 32, 8);
            hi[o] = __builtin_bit_cast(uint16_t, x);
            lo[o] = __builtin_bit_cast(uint16_t, (_Float16)(float)(v - (double)(float)x));
        }
    }
}

// the FP16X3 projection's operand table (layout: dct16_off), one thread per 8-half entry
__global__ __launch_bounds__(256) void to_dct16_kernel(const double *__restrict__ dctn, int N, int NT, int NK, int g,
                                                       uint16_t *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 2 * NT * NK * 2 * 64) return;
    const int lane = i % 64, hl = (i / 64) % 2, k = (i / 128) % NK, t = (i / (128 * NK)) % NT, par = i / (128 * NK * NT);
    const int n = 2 * (16 * t + lane % 16) + par;
    for (int e = 0; e < 8; ++e) {
        const int j = 32 * k + 8 * (lane / 16) + e;
        const double v = (n < N && j < N / 2) ? ldexp(dctn[(size_t)n * N + j], g) : 0.0;
        const _Float16 h = (_Float16)(float)v;
        const _Float16 x = hl ? (_Float16)(float)(v - (double)(float)h) : h;
        out[dct16_off(par, t, k, hl, lane, NT, NK) + e] = __builtin_bit_cast(uint16_t, x);
    }
}

void gauss_legendre16(double *x, double *w) {
    const int n = 16;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 60; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            dp = n * (z * p1 - p2) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

blast_status build_basis(blast_plan *p, hipStream_t s) {
    const int M = p->kq_panels;
    const double phase = p->kq_phase;
    const double lnkmin = std::log(p->kmin), span = std::log(p->kmax) - std::log(p->kmin);
    const double Rmax = *std::max_element(p->R.begin(), p->R.end());
    // sub-panels per chi node
    std::vector<double2> panels;
    std::vector<int> pstart(p->n_chi + 1, 0);
    for (int a = 0; a < p->n_chi; ++a) {
        pstart[a] = (int)panels.size();
        const double omega = p->chi[a] * (1.0 + Rmax);
        for (int i = 0; i < M; ++i) {
            const double xa = -std::cos(M_PI * i / M), xb = -std::cos(M_PI * (i + 1) / M);
            const double ka = i == 0 ? p->kmin : std::exp(lnkmin + 0.5 * (xa + 1.0) * span);
            const double kb = i == M - 1 ? p->kmax : std::exp(lnkmin + 0.5 * (xb + 1.0) * span);
            const int ns = std::max(1, (int)std::ceil(omega * (kb - ka) / phase));
            const double h = (kb - ka) / ns;
            for (int u = 0; u < ns; ++u)
                panels.push_back(make_double2(ka + u * h, u == ns - 1 ? kb : ka + (u + 1) * h));
        }
    }
    pstart[p->n_chi] = (int)panels.size();
    p->kq_nodes = (int64_t)panels.size() * 16;

    double glx[16], glw[16];
    gauss_legendre16(glx, glw);
    BLAST_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_glx), glx, sizeof(glx)));
    BLAST_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_glw), glw, sizeof(glw)));

    const int S = p->n_R + 1;
    const int ilp = round_up(p->n_ell, 32);
    const int ncp = p->nc_pad;
    const size_t nb = (size_t)p->NP * p->rows_pad * ncp;
    hipError_t e = hipMalloc(&p->basis.f64, nb * sizeof(double));
    if (e != hipSuccess) {
        p->basis.f64 = nullptr;
        set_error("basis allocation of %zu bytes failed: %s", nb * sizeof(double), hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP;
    }
    BLAST_HIP_TRY(hipMemsetAsync(p->basis.f64, 0, nb * sizeof(double), s));

    double2 *d_panels = nullptr;
    double *d_Tq = nullptr, *d_Fq = nullptr, *d_Kq = nullptr, *d_J = nullptr, *d_R = nullptr;
    int *d_perm = nullptr, *d_runs = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        if (d_panels) (void)hipFree(d_panels);
        if (d_Tq) (void)hipFree(d_Tq);
        if (d_Fq) (void)hipFree(d_Fq);
        if (d_Kq) (void)hipFree(d_Kq);
        if (d_J) (void)hipFree(d_J);
        if (d_R) (void)hipFree(d_R);
        if (d_perm) (void)hipFree(d_perm);
        if (d_runs) (void)hipFree(d_runs);
    };
    auto alloc = [&](void **q, size_t bytes) {
        hipError_t r = hipMalloc(q, bytes);
        if (r != hipSuccess) *q = nullptr;
        return r;
    };
    e = alloc((void **)&d_panels, panels.size() * sizeof(double2));
    if (e == hipSuccess) e = alloc((void **)&d_Tq, (size_t)kG * kQc * ncp * sizeof(double));
    if (e == hipSuccess) e = alloc((void **)&d_Fq, (size_t)kG * kQc * kMaxTypes * sizeof(double));
    if (e == hipSuccess) e = alloc((void **)&d_Kq, (size_t)kG * kQc * sizeof(double));
    if (e == hipSuccess) e = alloc((void **)&d_J, (size_t)kG * S * kQc * ilp * sizeof(double));
    if (e == hipSuccess) e = alloc((void **)&d_R, p->n_R * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(d_panels, panels.data(), panels.size() * sizeof(double2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_R, p->R.data(), p->n_R * sizeof(double), hipMemcpyHostToDevice);
    // non-integer multipoles: runs of equal fractional part (each in increasing order)
    int nruns = 0;
    if (e == hipSuccess && !p->int_ell) {
        std::vector<int> perm(p->n_ell), runs;
        std::vector<char> done(p->n_ell, 0);
        int np = 0;
        for (int i = 0; i < p->n_ell; ++i) {
            if (done[i]) continue;
            const double mu = p->ell[i] - std::floor(p->ell[i]);
            runs.push_back(np);
            for (int j = i; j < p->n_ell; ++j)
                if (!done[j] && p->ell[j] - std::floor(p->ell[j]) == mu) {
                    done[j] = 1;
                    perm[np++] = j;
                }
        }
        runs.push_back(np);
        nruns = (int)runs.size() - 1;
        e = alloc((void **)&d_perm, perm.size() * sizeof(int));
        if (e == hipSuccess) e = alloc((void **)&d_runs, runs.size() * sizeof(int));
        if (e == hipSuccess) e = hipMemcpy(d_perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_runs, runs.data(), runs.size() * sizeof(int), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        set_error("basis workspace: %s", hipGetErrorString(e));
        cleanup();
        return e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP;
    }

    // items: groups of kG consecutive chi nodes, chunk c of each
    const int t0 = p->tslot_type[0], t1 = p->tslot_type[1], t2 = p->tslot_type[2];
    for (int ag = 0; ag < p->n_chi; ag += kG) {
        int maxch = 0;
        for (int a = ag; a < std::min(ag + kG, p->n_chi); ++a)
            maxch = std::max(maxch, ((pstart[a + 1] - pstart[a]) * 16 + kQc - 1) / kQc);
        for (int c = 0; c < maxch; ++c) {
            Items it{};
            it.n = 0;
            for (int a = ag; a < std::min(ag + kG, p->n_chi); ++a) {
                const int nq_a = (pstart[a + 1] - pstart[a]) * 16;
                if (c * kQc >= nq_a) continue;
                it.a[it.n] = a;
                it.p0[it.n] = pstart[a] + c * (kQc / 16);
                it.nq[it.n] = std::min(kQc, nq_a - c * kQc);
                it.n++;
            }
            if (!it.n) continue;
            hipLaunchKernelGGL(tq_kernel, dim3(kQc / 256, it.n), dim3(256), 0, s, it, d_panels, lnkmin, span,
                               p->n_cheb, ncp, p->nt, t0, t1, t2, d_Tq, d_Fq, d_Kq);
            if (p->int_ell)
                hipLaunchKernelGGL(bessel_kernel, dim3(kQc / 256, S, it.n), dim3(256), 0, s, it, d_Kq, p->d_chi, d_R,
                                   S, p->d_elli, p->n_ell, ilp, d_J);
            else
                hipLaunchKernelGGL(bessel_real_kernel, dim3(kQc / 256, S, it.n), dim3(256), 0, s, it, d_Kq, p->d_chi,
                                   d_R, S, p->d_ell, d_perm, d_runs, nruns, p->n_ell, ilp, d_J);
            hipLaunchKernelGGL(gemm_kernel, dim3(ilp / 32, p->n_R, it.n), dim3(256), 0, s, it, d_J, d_Tq, d_Fq, S, ilp,
                               ncp, p->n_ell, p->nt, p->n_R, p->rows_pad, p->basis.f64);
            e = hipGetLastError();
            if (e != hipSuccess) {
                set_error("basis kernels: %s", hipGetErrorString(e));
                cleanup();
                return BLAST_E_HIP;
            }
        }
    }
    cleanup();
    return BLAST_OK;
}

blast_status ensure_f32t(blast_plan *p, hipStream_t s) {
    if (p->basis.f32t) return BLAST_OK;
    const size_t n = (size_t)p->NP * p->rows_pad * p->nc_pad;
    hipError_t e = hipMalloc(&p->basis.f32t, n * sizeof(float));
    if (e != hipSuccess) {
        p->basis.f32t = nullptr;
        set_error("transposed FP32 basis: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP;
    }
    hipLaunchKernelGGL(to_f32t_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p->basis.f64, p->basis.f32t,
                       n, p->rows_pad, p->nc_pad);
    BLAST_HIP_TRY(hipGetLastError());
    // once per plan: finished before any call on another stream can see the pointer
    BLAST_HIP_TRY(hipStreamSynchronize(s));
    return BLAST_OK;
}

blast_status ensure_nf32t(blast_plan *p, hipStream_t s) {
    if (p->basis.nf32t) return BLAST_OK;
    const size_t n = (size_t)p->NP * p->rows_pad * p->nc_pad, nrows = (size_t)p->NP * p->rows_pad;
    hipError_t e = hipMalloc(&p->basis.nf32t, n * sizeof(float));
    if (e != hipSuccess) {
        p->basis.nf32t = nullptr;
        set_error("transposed FP32 nodal basis: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP;
    }
    const unsigned g = (unsigned)std::min<size_t>((nrows + 3) / 4, 2048);
    hipLaunchKernelGGL(to_nodal_kernel<33>, dim3(g), dim3(256), 0, s, p->basis.f64, p->d_dctn64, nrows, p->rows_pad,
                       p->nc_pad, p->n_cheb, nullptr, nullptr, nullptr, p->basis.nf32t, nullptr);
    BLAST_HIP_TRY(hipGetLastError());
    // once per plan: finished before any call on another stream can see the pointer
    BLAST_HIP_TRY(hipStreamSynchronize(s));
    return BLAST_OK;
}

blast_status derive_precisions(blast_plan *p, hipStream_t s) {
    const size_t n = (size_t)p->NP * p->rows_pad * p->nc_pad;
    const size_t nrows = (size_t)p->NP * p->rows_pad;
    auto fail = [&](hipError_t e, const char *what) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP;
    };
    if (p->precisions & (1u << BLAST_FP32)) {
        hipError_t e = hipMalloc(&p->basis.f32, n * sizeof(float));
        if (e != hipSuccess) return p->basis.f32 = nullptr, fail(e, "FP32 basis");
        hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p->basis.f64,
                           p->basis.f32, n, p->rows_pad, p->nc_pad);
        if (p->n_cheb % 4 == 0) {  // P rows of whole 16-byte granules, read in place of c rows
            e = hipMalloc(&p->basis.nf32, n * sizeof(float));
            if (e != hipSuccess) return p->basis.nf32 = nullptr, fail(e, "FP32 nodal basis");
            const unsigned g = (unsigned)std::min<size_t>((nrows + 3) / 4, 2048);
            hipLaunchKernelGGL(to_nodal_kernel<32>, dim3(g), dim3(256), 0, s, p->basis.f64, p->d_dctn64, nrows,
                               p->rows_pad, p->nc_pad, p->n_cheb, nullptr, nullptr, nullptr, p->basis.nf32, nullptr);
        }
    }
    if ((p->precisions & (1u << BLAST_FP64)) && p->n_cheb == p->nc_pad) {  // FP64 nodal P read as c
        hipError_t e = hipMalloc(&p->basis.nf64, n * sizeof(double));
        if (e != hipSuccess) return p->basis.nf64 = nullptr, fail(e, "FP64 nodal basis");
        const unsigned g = (unsigned)std::min<size_t>((nrows + 3) / 4, 2048);
        hipLaunchKernelGGL(to_nodal_kernel<64>, dim3(g), dim3(256), 0, s, p->basis.f64, p->d_dctn64, nrows,
                           p->rows_pad, p->nc_pad, p->n_cheb, nullptr, nullptr, nullptr, nullptr, p->basis.nf64);
    }
    const bool want_hi = p->precisions & ((1u << BLAST_BF16) | (1u << BLAST_BF16X3));
    const bool want_lo = p->precisions & (1u << BLAST_BF16X3);
    if (want_hi) {
        hipError_t e = hipMalloc(&p->basis.hi, n * sizeof(uint16_t));
        if (e != hipSuccess) return p->basis.hi = nullptr, fail(e, "BF16 basis");
        e = hipMalloc(&p->basis.scale, nrows * sizeof(float));
        if (e != hipSuccess) return p->basis.scale = nullptr, fail(e, "basis scales");
        if (want_lo) {
            e = hipMalloc(&p->basis.lo, n * sizeof(uint16_t));
            if (e != hipSuccess) return p->basis.lo = nullptr, fail(e, "BF16 lo basis");
        }
        hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((nrows + 3) / 4)), dim3(256), 0, s, p->basis.f64, nrows,
                           p->rows_pad, p->nc_pad, p->basis.hi, p->basis.lo, p->basis.scale);
    }
    if (p->precisions & (1u << BLAST_FP16X3)) {
        hipError_t e = hipMalloc(&p->basis.h16, n * sizeof(uint16_t));
        if (e != hipSuccess) return p->basis.h16 = nullptr, fail(e, "FP16 basis");
        e = hipMalloc(&p->basis.l16, n * sizeof(uint16_t));
        if (e != hipSuccess) return p->basis.l16 = nullptr, fail(e, "FP16 lo basis");
        e = hipMalloc(&p->basis.scale16, nrows * sizeof(float));
        if (e != hipSuccess) return p->basis.scale16 = nullptr, fail(e, "FP16 basis scales");
        hipLaunchKernelGGL(to_fp16_kernel, dim3((unsigned)((nrows + 3) / 4)), dim3(256), 0, s, p->basis.f64, nrows,
                           p->rows_pad, p->nc_pad, p->basis.h16, p->basis.l16, p->basis.scale16);
        const int NT = p->nc_pad / 32, NK = (NT + 1) / 2, nent = 2 * NT * NK * 2 * 64;
        e = hipMalloc(&p->d_dct16, (size_t)nent * 8 * sizeof(uint16_t));
        if (e != hipSuccess) return p->d_dct16 = nullptr, fail(e, "FP16 projection table");
        hipLaunchKernelGGL(to_dct16_kernel, dim3((unsigned)((nent + 255) / 256)), dim3(256), 0, s, p->d_dctn64,
                           p->n_cheb, NT, NK, dct16_exp(p->n_cheb), p->d_dct16);
        if (p->n_cheb % 4 == 0) {  // P rows of whole 16-byte granules, loaded as such by the FP16X3 nodal kernel
            e = hipMalloc(&p->basis.n16, n * sizeof(uint16_t));
            if (e != hipSuccess) return p->basis.n16 = nullptr, fail(e, "FP16 nodal basis");
            e = hipMalloc(&p->basis.nl16, n * sizeof(uint16_t));
            if (e != hipSuccess) return p->basis.nl16 = nullptr, fail(e, "FP16 lo nodal basis");
            e = hipMalloc(&p->basis.nscale16, nrows * sizeof(float));
            if (e != hipSuccess) return p->basis.nscale16 = nullptr, fail(e, "FP16 nodal basis scales");
            const unsigned g = (unsigned)std::min<size_t>((nrows + 3) / 4, 2048);
            hipLaunchKernelGGL(to_nodal_kernel<16>, dim3(g), dim3(256), 0, s, p->basis.f64, p->d_dctn64, nrows,
                               p->rows_pad, p->nc_pad, p->n_cheb, p->basis.n16, p->basis.nl16, p->basis.nscale16,
                               nullptr, nullptr);
        }
    }
    BLAST_HIP_TRY(hipGetLastError());
    return BLAST_OK;
}

}  // namespace blast
