// Limber approximations (first order and extended) and the non-linear correction.
//
//   C_ij(l) = N_t(l) (pi/2) sum_a wchi_a f_t(k)/k^2 dP[l][a] / chi_a^2 E_ij(l, a),  k = (l+1/2)/chi_a
//   E = K_i K_j                                      (order 1)
//   E = K_i K_j - nu^-2 (A_i K_j + K_i A_j),  A = sqrt(chi) (chi^2/2 Kt'' + chi^3/6 Kt''')   (order 2)
// with Kt = K / sqrt(chi) and nu = l + 1/2 (Sec. 2.2; the sign of the correction is the one of
// the Bessel expansion, see the header).  dP = P - P_sub is the caller's spectrum (or the
// difference non-linear minus linear of Sec. 3.2) at the Limber points.  FP64 throughout: the
// whole path is a few hundred MFLOP per batch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"

namespace blast {
namespace {

constexpr int kLimbChunk = 128;   // chi nodes staged in LDS per pass

struct LimbSel {
    int n_out;
    int16_t idx[kMaxEll];
};

// (K, A) for every (cosmology, bin, chi node); A only for order 2
__global__ __launch_bounds__(256) void limber_ka_kernel(const double *__restrict__ Kchi, const double *__restrict__ chi,
                                                        const double *__restrict__ fd, const int *__restrict__ fds,
                                                        int n_chi, long total, int order, double2 *__restrict__ KA) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int a = (int)(i % n_chi);
    const double *row = Kchi + (i - a);
    const double K = row[a];
    double A = 0.0;
    if (order == 2) {
        const int s0 = fds[a];
        double d2 = 0.0, d3 = 0.0;
        for (int q = 0; q < 5; ++q) {
            const double kt = row[s0 + q] / sqrt(chi[s0 + q]);
            d2 += fd[((size_t)a * 2 + 0) * 5 + q] * kt;
            d3 += fd[((size_t)a * 2 + 1) * 5 + q] * kt;
        }
        const double x = chi[a];
        A = sqrt(x) * (0.5 * x * x * d2 + x * x * x / 6.0 * d3);
    }
    KA[i] = make_double2(K, A);
}

__device__ inline void pair_decode(int p, int ng, int ns, uint32_t types, int &t, int &i, int &j) {
    const int ngg = (types & BLAST_GG) ? ng * (ng + 1) / 2 : 0;
    const int ngs = (types & BLAST_GS) ? ng * ns : 0;
    int q;
    int n, base;
    if (p < ngg) {
        t = BLAST_GG, q = p, n = ng, base = 0;
    } else if (p < ngg + ngs) {
        t = BLAST_GS, q = p - ngg;
        i = q / ns;
        j = ng + q % ns;
        return;
    } else {
        t = BLAST_SS, q = p - ngg - ngs, n = ns, base = ng;
    }
    int r = 0;
    while (q >= n - r) {
        q -= n - r;
        ++r;
    }
    i = base + r;
    j = base + r + q;
}

// One work-group per (16 output multipoles, cosmology); threads over bin pairs, each keeping the
// sums of its pair for the 16 multipoles; the chi loop runs over chunks with the weighted
// spectra of the 16 multipoles and every bin's (K, A) of the chunk staged in LDS (rows padded by
// one entry so that the bins read at one node fall in different banks).  Per chi node a thread
// forms K_i K_j and A_i K_j + K_i A_j once and uses them for all 16 multipoles.
constexpr int kLimbEll = 16;

template <typename PT>
__global__ __launch_bounds__(256) void limber_kernel(const PT *__restrict__ P, const PT *__restrict__ Psub,
                                                     const double2 *__restrict__ KA, const double *__restrict__ chi,
                                                     const double *__restrict__ wchi, const double *__restrict__ pref,
                                                     const double *__restrict__ ell, int slot_gg, int slot_gs,
                                                     int slot_ss, int n_chi, int n_ell, int ng, int ns, uint32_t types,
                                                     int npairs, LimbSel sel, int order, int accumulate,
                                                     double *__restrict__ C) {
    extern __shared__ __align__(16) double smem_l[];
    constexpr int KST = kLimbChunk + 1, LE = kLimbEll;
    double *u = smem_l;                                  // [LE][kLimbChunk]: wchi dP / chi^2
    double *c2 = smem_l + LE * kLimbChunk;               // [kLimbChunk]: chi^2
    double2 *kas = (double2 *)(c2 + kLimbChunk);         // [nbins][KST]: (K, A)
    const int io0 = blockIdx.x * LE, beta = blockIdx.y;
    const int nio = min(LE, sel.n_out - io0);
    const int nbins = ng + ns;
    const double2 *ka = KA + (size_t)beta * nbins * n_chi;
    double inu2[LE];
#pragma unroll
    for (int e = 0; e < LE; ++e) {
        const double nu = ell[sel.idx[io0 + (e < nio ? e : 0)]] + 0.5;
        inu2[e] = 1.0 / (nu * nu);
    }
    for (int p0 = 0; p0 < npairs; p0 += blockDim.x) {
        const int p = p0 + threadIdx.x;
        int t = 0, pi = 0, pj = 0;
        if (p < npairs) pair_decode(p, ng, ns, types, t, pi, pj);
        double s0[LE], s1[LE];
#pragma unroll
        for (int e = 0; e < LE; ++e) s0[e] = s1[e] = 0.0;
        for (int a0 = 0; a0 < n_chi; a0 += kLimbChunk) {
            const int na = min(kLimbChunk, n_chi - a0);
            __syncthreads();
            for (int i = threadIdx.x; i < LE * na; i += blockDim.x) {
                const int e = i / na, a = i % na;
                double d = 0.0;
                if (e < nio) {
                    const size_t o = ((size_t)beta * n_ell + sel.idx[io0 + e]) * n_chi + a0 + a;
                    d = (double)P[o];
                    if (Psub) d -= (double)Psub[o];
                }
                const double x = chi[a0 + a];
                u[e * kLimbChunk + a] = wchi[a0 + a] * d / (x * x);
            }
            for (int a = threadIdx.x; a < na; a += blockDim.x) c2[a] = chi[a0 + a] * chi[a0 + a];
            for (int i = threadIdx.x; i < nbins * na; i += blockDim.x) {
                const int bin = i / na, a = i % na;
                kas[bin * KST + a] = ka[(size_t)bin * n_chi + a0 + a];
            }
            __syncthreads();
            if (p >= npairs) continue;
            const double2 *ki = kas + pi * KST, *kj = kas + pj * KST;
            for (int a = 0; a < na; ++a) {
                const double2 vi = ki[a], vj = kj[a];
                const double e0 = vi.x * vj.x, e1 = vi.y * vj.x + vi.x * vj.y;
                const double x2 = c2[a];
#pragma unroll
                for (int e = 0; e < LE; ++e) {
                    // f_t / k^2 = 1, 1/k^2, 1/k^4 with 1/k^2 = chi^2 / nu^2
                    const double k2i = x2 * inu2[e];
                    const double g = t == BLAST_GG ? 1.0 : (t == BLAST_GS ? k2i : k2i * k2i);
                    const double wv = u[e * kLimbChunk + a] * g;
                    s0[e] += wv * e0;
                    s1[e] += wv * e1;
                }
            }
        }
        if (p >= npairs) continue;
        const int slot = t == BLAST_GG ? slot_gg : (t == BLAST_GS ? slot_gs : slot_ss);
#pragma unroll
        for (int e = 0; e < LE; ++e) {
            if (e >= nio) break;
            const int l = sel.idx[io0 + e];
            const double sum = order == 2 ? s0[e] - inu2[e] * s1[e] : s0[e];
            const double v = pref[slot * n_ell + l] * (0.5 * M_PI) * sum;
            double *o = C + ((size_t)beta * npairs + p) * sel.n_out + io0 + e;
            *o = accumulate ? *o + v : v;
        }
    }
}

int npairs_for(int ng, int ns, uint32_t types) {
    return ((types & BLAST_GG) ? ng * (ng + 1) / 2 : 0) + ((types & BLAST_GS) ? ng * ns : 0) +
           ((types & BLAST_SS) ? ns * (ns + 1) / 2 : 0);
}

}  // namespace

blast_status limber(blast_plan *p, const blast_limber_args *a, hipStream_t s) {
    if (a->batch < 1) return set_error("batch must be >= 1"), BLAST_E_INVALID;
    if (a->p_dtype != 0 && a->p_dtype != 1) return set_error("p_dtype must be 0 (FP64) or 1 (FP32)"), BLAST_E_INVALID;
    if (!a->P || !a->K_chi || !a->C) return set_error("P, K_chi and C are required"), BLAST_E_INVALID;
    if (a->order != 1 && a->order != 2) return set_error("order must be 1 or 2"), BLAST_E_INVALID;
    if (a->order == 2 && !p->d_fd)
        return set_error("the extended Limber approximation needs at least 5 chi nodes"), BLAST_E_INVALID;
    const int ng = a->n_g, ns = a->n_s, nbins = ng + ns;
    if (ng < 0 || ns < 0 || nbins < 1 || nbins > kMaxBins)
        return set_error("need n_g, n_s >= 0 and 1 <= n_g + n_s <= %d", kMaxBins), BLAST_E_INVALID;
    if (a->types == 0 || (a->types & ~p->types))
        return set_error("types 0x%x not a non-empty subset of the plan's 0x%x", a->types, p->types), BLAST_E_INVALID;
    const int npairs = npairs_for(ng, ns, a->types);
    if (npairs < 1) return set_error("no bin pairs for these types and bins"), BLAST_E_INVALID;
    LimbSel sel{};
    if (a->n_ell_out == 0) {
        sel.n_out = p->n_ell;
        for (int i = 0; i < p->n_ell; ++i) sel.idx[i] = (int16_t)i;
    } else {
        if (a->n_ell_out < 0 || a->n_ell_out > p->n_ell || !a->ell_idx)
            return set_error("bad n_ell_out / ell_idx"), BLAST_E_INVALID;
        sel.n_out = a->n_ell_out;
        for (int i = 0; i < a->n_ell_out; ++i) {
            const int v = a->ell_idx[i];
            if (v < 0 || v >= p->n_ell || (i && v <= a->ell_idx[i - 1]))
                return set_error("ell_idx must be increasing indices into the plan's ell"), BLAST_E_INVALID;
            sel.idx[i] = (int16_t)v;
        }
    }
    // (K, A) table in the plan's Limber scratch
    const size_t need = (size_t)a->batch * nbins * p->n_chi * sizeof(double2);
    void *ws;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        if (p->limb_ws_bytes < need) {
            (void)hipDeviceSynchronize();
            if (p->limb_ws) (void)hipFree(p->limb_ws);
            p->limb_ws = nullptr;
            p->limb_ws_bytes = 0;
            hipError_t e = hipMalloc(&p->limb_ws, need);
            if (e != hipSuccess) {
                p->limb_ws = nullptr;
                return set_error("Limber scratch of %zu bytes: %s", need, hipGetErrorString(e)), BLAST_E_OOM;
            }
            p->limb_ws_bytes = need;
        }
        ws = p->limb_ws;
    }
    const long total = (long)a->batch * nbins * p->n_chi;
    hipLaunchKernelGGL(limber_ka_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a->K_chi, p->d_chi,
                       p->d_fd, p->d_fds, p->n_chi, total, a->order, (double2 *)ws);
    dim3 grid((unsigned)((sel.n_out + kLimbEll - 1) / kLimbEll), (unsigned)a->batch);
    const size_t lds = ((kLimbEll + 1) * kLimbChunk + 2 * (size_t)nbins * (kLimbChunk + 1)) * sizeof(double);  // <= 83 KB
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute((const void *)limber_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipFuncSetAttribute((const void *)limber_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
    });
    if (a->p_dtype == 0)
        hipLaunchKernelGGL(limber_kernel<double>, grid, dim3(256), lds, s, (const double *)a->P, (const double *)a->P_sub,
                           (const double2 *)ws, p->d_chi, p->d_wchi, p->d_pref, p->d_ell, p->slot[0], p->slot[1], p->slot[2],
                           p->n_chi, p->n_ell,
                           ng, ns, a->types, npairs, sel, a->order, a->accumulate, a->C);
    else
        hipLaunchKernelGGL(limber_kernel<float>, grid, dim3(256), lds, s, (const float *)a->P, (const float *)a->P_sub,
                           (const double2 *)ws, p->d_chi, p->d_wchi, p->d_pref, p->d_ell, p->slot[0], p->slot[1], p->slot[2],
                           p->n_chi, p->n_ell,
                           ng, ns, a->types, npairs, sel, a->order, a->accumulate, a->C);
    BLAST_HIP_TRY(hipGetLastError());
    return BLAST_OK;
}

}  // namespace blast
