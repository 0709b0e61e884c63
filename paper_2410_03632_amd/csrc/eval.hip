// Per-cosmology evaluation: projection -> contraction -> quadrature.
//
//  project   c[beta][ab][n] = sum_j D[n][j] P[beta][ab][j]                      (Eq. dft, as a DCT-II)
//  contract  w[beta][ab][row] = sum_n Ttilde[ab][row][n] c[beta][ab][n]          (Eq. pmd)
//  quad_y    Y[beta][a][row][bin] = sum_b wR_b K_bin(R_b chi_a) w[beta][ab][row]
//  quad_c    C[beta][p][l] = N_t(l) sum_a wchi_a chi_a [K_i(chi_a) Y[..][j] + K_j(chi_a) Y[..][i]]
//                                                                              (Eq. final_cls)
// ab = a * n_R + b is the (chi_a, R_b) point; row = slot(t) * n_ell + l.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "internal.h"

namespace blast {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct alignas(16) U4 {
    uint32_t x, y, z, w;
};

// ---------------------------------------------------------------------------------------------
// projection
// ---------------------------------------------------------------------------------------------
constexpr int kProjRows = 32;

__device__ inline uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_val(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// OUT: 0 -> double c, 1 -> float c, 2 -> BF16 hi (+ lo when c_lo != nullptr)
template <typename PT, typename AT, int OUT>
__global__ __launch_bounds__(256) void project_kernel(const PT *__restrict__ P, const AT *__restrict__ Dt, int N,
                                                      int ncp, long nrows, void *__restrict__ c_out,
                                                      uint16_t *__restrict__ c_lo) {
    __shared__ AT Ps[kProjRows][kMaxCheb];
    const long r0 = (long)blockIdx.x * kProjRows;
    for (int i = threadIdx.x; i < kProjRows * N; i += blockDim.x) {
        const int r = i / N, j = i % N;
        Ps[r][j] = (r0 + r < nrows) ? (AT)P[(r0 + r) * N + j] : (AT)0;
    }
    __syncthreads();
    const int groups = 256 / ncp;  // ncp in {32, 64, 128}
    const int n = threadIdx.x % ncp, grp = threadIdx.x / ncp;
    if (grp >= groups) return;
    constexpr int kMaxAcc = kProjRows / 2;
    AT acc[kMaxAcc];
#pragma unroll
    for (int i = 0; i < kMaxAcc; ++i) acc[i] = (AT)0;
    const int per = kProjRows / groups;
    for (int j = 0; j < N; ++j) {
        const AT d = Dt[(size_t)j * ncp + n];
#pragma unroll
        for (int i = 0; i < kMaxAcc; ++i)
            if (i < per) acc[i] += d * Ps[grp + i * groups][j];
    }
#pragma unroll
    for (int i = 0; i < kMaxAcc; ++i) {
        if (i >= per) break;
        const long row = r0 + grp + i * groups;
        if (row >= nrows) continue;
        const size_t o = (size_t)row * ncp + n;
        if (OUT == 0) {
            ((double *)c_out)[o] = (double)acc[i];
        } else if (OUT == 1) {
            ((float *)c_out)[o] = (float)acc[i];
        } else {
            const float v = (float)acc[i];
            const uint16_t h = bf16_rne(v);
            ((uint16_t *)c_out)[o] = h;
            if (c_lo) c_lo[o] = bf16_rne(v - bf16_val(h));
        }
    }
}

// ---------------------------------------------------------------------------------------------
// contraction: per (chi_a, R_b) point a [rows x n] x [n x batch] product on MFMA.
// Lane layout of the 16x16 tiles: A[i][k] lane = i + 16*(k-group), B[k][j] lane = j + 16*(k-group),
// D[i][j] in register r of lane j + 16*(i/4), r = i%4 (f32 results), or r = i/4 of lane
// j + 16*(i%4) (f64 results).  The k order inside a tile is a free
// permutation shared by A and B: lane group g at load s supplies k = KSTEP*s + VEC*g + u.
// ---------------------------------------------------------------------------------------------
constexpr int kRowTilesPerWave = 5;

template <int PREC>
struct Cfg;
template <>
struct Cfg<BLAST_FP64> {
    using E = double;   // storage element
    using Acc = d4;
    static constexpr int VEC = 2, BT = 32;
};
template <>
struct Cfg<BLAST_FP32> {
    using E = float;
    using Acc = f4;
    static constexpr int VEC = 4, BT = 64;
};
template <>
struct Cfg<BLAST_BF16> {
    using E = uint16_t;
    using Acc = f4;
    static constexpr int VEC = 8, BT = 64;
};
template <>
struct Cfg<BLAST_BF16X3> {
    using E = uint16_t;
    using Acc = f4;
    static constexpr int VEC = 8, BT = 64;
};

template <int PREC>
__device__ inline void mma(typename Cfg<PREC>::Acc &acc, const U4 &a, const U4 &b) {
    if constexpr (PREC == BLAST_FP64) {
        double2 av, bv;
        memcpy(&av, &a, 16);
        memcpy(&bv, &b, 16);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.y, acc, 0, 0, 0);
    } else if constexpr (PREC == BLAST_FP32) {
        float4 av, bv;
        memcpy(&av, &a, 16);
        memcpy(&bv, &b, 16);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, acc, 0, 0, 0);
    } else {
        bf8 av, bv;
        memcpy(&av, &a, 16);
        memcpy(&bv, &b, 16);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
}

template <int PREC>
__global__ __launch_bounds__(256) void contract_kernel(const typename Cfg<PREC>::E *__restrict__ basis,
                                                       const uint16_t *__restrict__ basis_lo,
                                                       const float *__restrict__ scale,
                                                       const typename Cfg<PREC>::E *__restrict__ c,
                                                       const uint16_t *__restrict__ c_lo, int batch, int NP,
                                                       int rows_pad, int ncp, void *__restrict__ w_out) {
    using C = Cfg<PREC>;
    using E = typename C::E;
    using Acc = typename C::Acc;
    constexpr int VEC = C::VEC, BT = C::BT, BTN = BT / 16;
    constexpr bool X3 = PREC == BLAST_BF16X3;
    constexpr int KSTEP = 4 * VEC;
    // c tile of BT cosmologies: [BT][ncp] (+ lo part)
    // rows padded by 16 bytes so that the 16 rows read by one ds_read_b128 fall in distinct banks
    extern __shared__ __align__(16) unsigned char smem[];
    const int cst = ncp + 16 / (int)sizeof(E);
    E *cs = (E *)smem;
    uint16_t *cls = (uint16_t *)(smem + (size_t)BT * cst * sizeof(E));

    const int ab = blockIdx.x;
    const int beta0 = blockIdx.y * BT;
    const int nb = min(BT, batch - beta0);
    const int vec_per_row = ncp / VEC;
    for (int i = threadIdx.x; i < BT * vec_per_row; i += blockDim.x) {
        const int bb = i / vec_per_row, v = i % vec_per_row;
        U4 val = {0, 0, 0, 0}, vlo = {0, 0, 0, 0};
        if (bb < nb) {
            const size_t off = ((size_t)(beta0 + bb) * NP + ab) * ncp + (size_t)v * VEC;
            val = *(const U4 *)(c + off);
            if (X3) vlo = *(const U4 *)(c_lo + off);
        }
        *(U4 *)(cs + (size_t)bb * cst + v * VEC) = val;
        if (X3) *(U4 *)(cls + (size_t)bb * cst + v * VEC) = vlo;
    }
    __syncthreads();

    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int RT = rows_pad / 16;
    const E *brow = basis + (size_t)ab * rows_pad * ncp;
    const uint16_t *blo = X3 ? basis_lo + (size_t)ab * rows_pad * ncp : nullptr;
    const int nsteps = ncp / KSTEP;

    for (int pass = 0; pass * 4 * kRowTilesPerWave < RT; ++pass) {
        Acc acc[kRowTilesPerWave][BTN];
#pragma unroll
        for (int i = 0; i < kRowTilesPerWave; ++i)
#pragma unroll
            for (int j = 0; j < BTN; ++j) acc[i][j] = Acc{0, 0, 0, 0};
        int rt[kRowTilesPerWave];
#pragma unroll
        for (int i = 0; i < kRowTilesPerWave; ++i) rt[i] = pass * 4 * kRowTilesPerWave + w + 4 * i;

        for (int s = 0; s < nsteps; ++s) {
            const int kof = s * KSTEP + lk * VEC;
            U4 bv[BTN], bvl[BTN];
#pragma unroll
            for (int j = 0; j < BTN; ++j) {
                bv[j] = *(const U4 *)(cs + (size_t)(16 * j + lr) * cst + kof);
                if (X3) bvl[j] = *(const U4 *)(cls + (size_t)(16 * j + lr) * cst + kof);
            }
#pragma unroll
            for (int i = 0; i < kRowTilesPerWave; ++i) {
                if (rt[i] >= RT) continue;
                const size_t off = (size_t)(16 * rt[i] + lr) * ncp + kof;
                const U4 av = *(const U4 *)(brow + off);
                U4 avl;
                if (X3) avl = *(const U4 *)(blo + off);
#pragma unroll
                for (int j = 0; j < BTN; ++j) {
                    if (16 * j >= nb) continue;
                    mma<PREC>(acc[i][j], av, bv[j]);
                    if (X3) {
                        mma<PREC>(acc[i][j], av, bvl[j]);
                        mma<PREC>(acc[i][j], avl, bv[j]);
                    }
                }
            }
        }
        // epilogue: lane holds rows 16*rt + 4*lk + r for cosmology 16*j + lr
#pragma unroll
        for (int i = 0; i < kRowTilesPerWave; ++i) {
            if (rt[i] >= RT) continue;
            const int row0 = 16 * rt[i] + 4 * lk;
            float sc[4] = {1.f, 1.f, 1.f, 1.f};
            if (PREC == BLAST_BF16 || PREC == BLAST_BF16X3) {
#pragma unroll
                for (int r = 0; r < 4; ++r) sc[r] = scale[(size_t)ab * rows_pad + row0 + r];
            }
#pragma unroll
            for (int j = 0; j < BTN; ++j) {
                const int bb = 16 * j + lr;
                if (bb >= nb) continue;
                const size_t o = ((size_t)(beta0 + bb) * NP + ab) * rows_pad + row0;
                if (PREC == BLAST_FP64) {
                    // FP64 16x16 output: lane holds rows 16*rt + lk + 4r
                    double *wo = (double *)w_out + o - 4 * lk + lk;
#pragma unroll
                    for (int r = 0; r < 4; ++r) wo[4 * r] = acc[i][j][r];
                } else {
                    float4 v;
                    v.x = acc[i][j][0] * sc[0];
                    v.y = acc[i][j][1] * sc[1];
                    v.z = acc[i][j][2] * sc[2];
                    v.w = acc[i][j][3] * sc[3];
                    *(float4 *)((float *)w_out + o) = v;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// quadrature
// ---------------------------------------------------------------------------------------------
struct TypeInfo {
    int nt;
    int type[3];   // type bit of each resident slot
};

template <typename WT, int NB>
__global__ __launch_bounds__(256) void quad_y_kernel(const WT *__restrict__ w, const double *__restrict__ Kchi2,
                                                     const double *__restrict__ wR, int NP, int nR, int n_chi,
                                                     int rows, int rows_pad, int n_ell, TypeInfo ti, int ng, int ns,
                                                     double *__restrict__ Y) {
    extern __shared__ double Kt[];  // [nbins][nR]
    const int a = blockIdx.x, beta = blockIdx.y;
    const int nbins = ng + ns;
    for (int i = threadIdx.x; i < nbins * nR; i += blockDim.x) {
        const int bin = i / nR, b = i % nR;
        Kt[i] = wR[b] * Kchi2[(((size_t)beta * nbins + bin) * n_chi + a) * nR + b];
    }
    __syncthreads();
    const WT *wa = w + ((size_t)beta * NP + (size_t)a * nR) * rows_pad;
    for (int row = threadIdx.x; row < rows; row += blockDim.x) {
        const int t = ti.type[row / n_ell];
        const int lo = t == BLAST_SS ? ng : 0;
        const int hi = t == BLAST_GG ? ng : nbins;
        double acc[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] = 0.0;
        for (int b = 0; b < nR; ++b) {
            const double wv = (double)wa[(size_t)b * rows_pad + row];
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q >= lo && q < hi) acc[q] += Kt[q * nR + b] * wv;
        }
        double *y = Y + (((size_t)beta * n_chi + a) * rows_pad + row) * nbins;
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (q < nbins) y[q] = acc[q];
    }
}

struct Slots {
    int s[3];
};

struct EllSel {
    int n_out;
    int16_t idx[kMaxEll];
};

__device__ inline void decode_pair(int p, int ng, int ns, uint32_t types, int &t, int &i, int &j) {
    if (types & BLAST_GG) {
        const int n = ng * (ng + 1) / 2;
        if (p < n) {
            int r = 0;
            while (p >= ng - r) {
                p -= ng - r;
                ++r;
            }
            t = BLAST_GG;
            i = r;
            j = r + p;
            return;
        }
        p -= n;
    }
    if (types & BLAST_GS) {
        const int n = ng * ns;
        if (p < n) {
            t = BLAST_GS;
            i = p / ns;
            j = ng + p % ns;
            return;
        }
        p -= n;
    }
    int r = 0;
    while (p >= ns - r) {
        p -= ns - r;
        ++r;
    }
    t = BLAST_SS;
    i = ng + r;
    j = ng + r + p;
}

__global__ __launch_bounds__(256) void quad_c_kernel(const double *__restrict__ Y, const double *__restrict__ Kchi,
                                                     const double *__restrict__ wchi, const double *__restrict__ chi,
                                                     const double *__restrict__ pref, int n_chi, int rows_pad,
                                                     int n_ell, Slots slot_of, int ng, int ns,
                                                     uint32_t types, int npairs, EllSel sel, int batch,
                                                     double *__restrict__ C) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)batch * npairs * sel.n_out;
    if (gid >= total) return;
    const int io = gid % sel.n_out;
    const int p = (gid / sel.n_out) % npairs;
    const int beta = gid / ((long)sel.n_out * npairs);
    int t, i, j;
    decode_pair(p, ng, ns, types, t, i, j);
    const int sl = slot_of.s[t == BLAST_GG ? 0 : (t == BLAST_GS ? 1 : 2)];
    const int row = sl * n_ell + sel.idx[io];
    const int nbins = ng + ns;
    const double *Kb = Kchi + (size_t)beta * nbins * n_chi;
    double s = 0.0;
    for (int a = 0; a < n_chi; ++a) {
        const double *y = Y + (((size_t)beta * n_chi + a) * rows_pad + row) * nbins;
        s += wchi[a] * chi[a] * (Kb[(size_t)i * n_chi + a] * y[j] + Kb[(size_t)j * n_chi + a] * y[i]);
    }
    C[gid] = pref[row] * s;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
    size_t c, clo, w, y, total;
};

Layout layout_of(const blast_plan *p, int batch, int prec, int nbins, bool need_w) {
    Layout L{};
    const size_t nc = (size_t)batch * p->NP * p->nc_pad;
    const size_t ce = prec == BLAST_FP64 ? 8 : (prec == BLAST_FP32 ? 4 : 2);
    size_t off = 0;
    L.c = off;
    off += align256(nc * ce);
    L.clo = off;
    if (prec == BLAST_BF16X3) off += align256(nc * 2);
    L.w = off;
    if (need_w) off += align256((size_t)batch * p->NP * p->rows_pad * (prec == BLAST_FP64 ? 8 : 4));
    L.y = off;
    off += align256((size_t)batch * p->n_chi * p->rows_pad * nbins * 8);
    L.total = off;
    return L;
}

}  // namespace

size_t workspace_bytes(const blast_plan *p, int batch, int prec, int n_bins) {
    return layout_of(p, batch, prec, n_bins, true).total;
}

static int npairs_of(int ng, int ns, uint32_t types) {
    int n = 0;
    if (types & BLAST_GG) n += ng * (ng + 1) / 2;
    if (types & BLAST_GS) n += ng * ns;
    if (types & BLAST_SS) n += ns * (ns + 1) / 2;
    return n;
}

blast_status forward(blast_plan *p, const blast_cl_args *a, hipStream_t s) {
    if (a->batch < 1) return set_error("batch must be >= 1"), BLAST_E_INVALID;
    if (a->precision < 0 || a->precision > 3) return set_error("unknown precision %d", a->precision), BLAST_E_INVALID;
    const int prec = a->precision;
    const bool resident = (prec == BLAST_FP64 && p->basis.f64) || (prec == BLAST_FP32 && p->basis.f32) ||
                          (prec == BLAST_BF16 && p->basis.hi) || (prec == BLAST_BF16X3 && p->basis.lo);
    if (!resident) return set_error("precision %d is not resident in this plan", prec), BLAST_E_INVALID;
    if (a->p_dtype != 0 && a->p_dtype != 1) return set_error("p_dtype must be 0 (FP64) or 1 (FP32)"), BLAST_E_INVALID;
    if (!a->P || !a->K_chi || !a->K_chi2 || !a->C) return set_error("P, K_chi, K_chi2 and C are required"), BLAST_E_INVALID;
    const int ng = a->n_g, ns = a->n_s, nbins = ng + ns;
    if (ng < 0 || ns < 0 || nbins < 1 || nbins > kMaxBins)
        return set_error("need n_g, n_s >= 0 and 1 <= n_g + n_s <= %d", kMaxBins), BLAST_E_INVALID;
    if (a->types == 0 || (a->types & ~p->types))
        return set_error("types 0x%x not a non-empty subset of the plan's 0x%x", a->types, p->types), BLAST_E_INVALID;
    const int npairs = npairs_of(ng, ns, a->types);
    if (npairs < 1) return set_error("no bin pairs for these types and bins"), BLAST_E_INVALID;
    EllSel sel{};
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
    if ((size_t)nbins * p->n_R * sizeof(double) > 64 * 1024)
        return set_error("n_bins * n_R too large for the quadrature tile"), BLAST_E_UNSUPPORTED;

    const bool need_w = a->w_save == nullptr;
    Layout L = layout_of(p, a->batch, prec, nbins, need_w);
    unsigned char *ws = (unsigned char *)a->workspace;
    if (ws) {
        if (a->workspace_bytes < L.total)
            return set_error("workspace of %zu bytes is smaller than the %zu needed", a->workspace_bytes, L.total),
                   BLAST_E_INVALID;
    } else {
        std::lock_guard<std::mutex> lk(p->mu);
        if (p->scratch_bytes < L.total) {
            (void)hipDeviceSynchronize();
            if (p->scratch) (void)hipFree(p->scratch);
            p->scratch = nullptr;
            p->scratch_bytes = 0;
            hipError_t e = hipMalloc(&p->scratch, L.total);
            if (e != hipSuccess) {
                p->scratch = nullptr;
                return set_error("plan scratch of %zu bytes: %s", L.total, hipGetErrorString(e)), BLAST_E_OOM;
            }
            p->scratch_bytes = L.total;
        }
        ws = (unsigned char *)p->scratch;
    }
    void *c = ws + L.c;
    uint16_t *clo = prec == BLAST_BF16X3 ? (uint16_t *)(ws + L.clo) : nullptr;
    void *w = need_w ? (void *)(ws + L.w) : a->w_save;
    double *Y = (double *)(ws + L.y);
    const long nrows = (long)a->batch * p->NP;
    const int N = p->n_cheb, ncp = p->nc_pad;

    // 1. projection
    {
        dim3 grid((unsigned)((nrows + kProjRows - 1) / kProjRows));
        if (prec == BLAST_FP64) {
            if (a->p_dtype == 0)
                hipLaunchKernelGGL((project_kernel<double, double, 0>), grid, dim3(256), 0, s, (const double *)a->P,
                                   p->d_dct64, N, ncp, nrows, c, nullptr);
            else
                hipLaunchKernelGGL((project_kernel<float, double, 0>), grid, dim3(256), 0, s, (const float *)a->P,
                                   p->d_dct64, N, ncp, nrows, c, nullptr);
        } else {
            if (a->p_dtype == 0) {
                if (prec == BLAST_FP32)
                    hipLaunchKernelGGL((project_kernel<double, float, 1>), grid, dim3(256), 0, s, (const double *)a->P,
                                       p->d_dct32, N, ncp, nrows, c, nullptr);
                else
                    hipLaunchKernelGGL((project_kernel<double, float, 2>), grid, dim3(256), 0, s, (const double *)a->P,
                                       p->d_dct32, N, ncp, nrows, c, clo);
            } else {
                if (prec == BLAST_FP32)
                    hipLaunchKernelGGL((project_kernel<float, float, 1>), grid, dim3(256), 0, s, (const float *)a->P,
                                       p->d_dct32, N, ncp, nrows, c, nullptr);
                else
                    hipLaunchKernelGGL((project_kernel<float, float, 2>), grid, dim3(256), 0, s, (const float *)a->P,
                                       p->d_dct32, N, ncp, nrows, c, clo);
            }
        }
    }
    // 2. contraction
    {
        auto launch = [&](auto tag) {
            constexpr int PR = decltype(tag)::value;
            using E = typename Cfg<PR>::E;
            const int BT = Cfg<PR>::BT;
            const size_t cst = ncp + 16 / sizeof(E);
            const size_t sh = (size_t)BT * cst * sizeof(E) + (PR == BLAST_BF16X3 ? (size_t)BT * cst * 2 : 0);
            dim3 grid(p->NP, (a->batch + BT - 1) / BT);
            const E *bas = PR == BLAST_FP64 ? (const E *)p->basis.f64
                                            : (PR == BLAST_FP32 ? (const E *)p->basis.f32 : (const E *)p->basis.hi);
            hipLaunchKernelGGL((contract_kernel<PR>), grid, dim3(256), sh, s, bas, p->basis.lo, p->basis.scale,
                               (const E *)c, clo, a->batch, p->NP, p->rows_pad, ncp, w);
        };
        if (prec == BLAST_FP64) launch(std::integral_constant<int, BLAST_FP64>());
        if (prec == BLAST_FP32) launch(std::integral_constant<int, BLAST_FP32>());
        if (prec == BLAST_BF16) launch(std::integral_constant<int, BLAST_BF16>());
        if (prec == BLAST_BF16X3) launch(std::integral_constant<int, BLAST_BF16X3>());
    }
    // 3. quadrature
    {
        TypeInfo ti{};
        ti.nt = p->nt;
        for (int i = 0; i < 3; ++i) ti.type[i] = p->tslot_type[i];
        dim3 grid(p->n_chi, a->batch);
        auto qy = [&](auto nbtag) {
            constexpr int NB = decltype(nbtag)::value;
            const size_t sh = (size_t)nbins * p->n_R * sizeof(double);
            if (prec == BLAST_FP64)
                hipLaunchKernelGGL((quad_y_kernel<double, NB>), grid, dim3(256), sh, s, (const double *)w, a->K_chi2,
                                   p->d_wR, p->NP, p->n_R, p->n_chi, p->rows, p->rows_pad, p->n_ell, ti, ng, ns, Y);
            else
                hipLaunchKernelGGL((quad_y_kernel<float, NB>), grid, dim3(256), sh, s, (const float *)w, a->K_chi2,
                                   p->d_wR, p->NP, p->n_R, p->n_chi, p->rows, p->rows_pad, p->n_ell, ti, ng, ns, Y);
        };
        if (nbins <= 4)
            qy(std::integral_constant<int, 4>());
        else if (nbins <= 8)
            qy(std::integral_constant<int, 8>());
        else if (nbins <= 16)
            qy(std::integral_constant<int, 16>());
        else
            qy(std::integral_constant<int, 32>());
        Slots slots{{p->slot[0], p->slot[1], p->slot[2]}};
        const long total = (long)a->batch * npairs * sel.n_out;
        hipLaunchKernelGGL(quad_c_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Y, a->K_chi,
                           p->d_wchi, p->d_chi, p->d_pref, p->n_chi, p->rows_pad, p->n_ell, slots, ng, ns, a->types,
                           npairs, sel, a->batch, a->C);
    }
    BLAST_HIP_TRY(hipGetLastError());
    return BLAST_OK;
}

}  // namespace blast
