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
#include <mutex>
#include <type_traits>

#include "internal.h"

namespace blast {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

typedef uint32_t U4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

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

// MFMA projection: c[row][n] = sum_j P[row][j] D[n][j], 256 rows per work-group (wave w owns row
// tiles 4w..4w+3) and every n tile.  FP32: D staged in LDS (rows padded by 16 bytes so the 16
// rows of one ds_read_b128 fall in distinct banks).  FP64: D read through L1/L2.  The k order
// inside a tile is a permutation shared by A and B (lane group g supplies j = KSTEP*s + VEC*g + u).
// Needs N % (4*VEC) == 0.
template <typename PT, bool F64, int OUT>
__global__ __launch_bounds__(256) void project_mfma_kernel(const PT *__restrict__ P,
                                                           const typename std::conditional<F64, double, float>::type
                                                               *__restrict__ Dn,
                                                           int N, int ncp, long nrows, void *__restrict__ c_out,
                                                           uint16_t *__restrict__ c_lo) {
    using T = typename std::conditional<F64, double, float>::type;
    using Acc = typename std::conditional<F64, d4, f4>::type;
    constexpr int VEC = F64 ? 2 : 4;
    constexpr int KSTEP = 4 * VEC;
    constexpr int MAXNT = kMaxCheb / 16;
    constexpr int RT = 4;
    extern __shared__ __align__(16) unsigned char smem_p[];
    const int dst = N + 16 / (int)sizeof(T);
    const T *D = Dn;
    if constexpr (!F64) {
        T *Ds = (T *)smem_p;
        for (int i = threadIdx.x; i < ncp * (N / 4); i += blockDim.x) {
            const int n = i / (N / 4), q = i % (N / 4);
            *(float4 *)(Ds + (size_t)n * dst + 4 * q) = *(const float4 *)(Dn + (size_t)n * N + 4 * q);
        }
        __syncthreads();
        D = Ds;
    }
    const int ldd = F64 ? N : dst;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int nt = ncp >> 4;
    const long row0 = (long)blockIdx.x * 256 + 64 * w;
    Acc acc[RT][MAXNT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < MAXNT; ++t) acc[r][t] = Acc{0, 0, 0, 0};
    for (int s = 0; s < N / KSTEP; ++s) {
        const int j0 = s * KSTEP + lk * VEC;
        T av[RT][VEC];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const long row = row0 + 16 * r + lr;
            if (row < nrows) {
                const PT *pr = P + row * (long)N + j0;
                if constexpr (sizeof(PT) == 4 && VEC == 4) {
                    const float4 v = *(const float4 *)pr;
                    av[r][0] = v.x, av[r][1] = v.y, av[r][2] = v.z, av[r][3] = v.w;
                } else if constexpr (sizeof(PT) == 8 && VEC == 4) {
                    const double2 v0 = *(const double2 *)pr, v1 = *(const double2 *)(pr + 2);
                    av[r][0] = (T)v0.x, av[r][1] = (T)v0.y, av[r][2] = (T)v1.x, av[r][3] = (T)v1.y;
                } else if constexpr (sizeof(PT) == 8) {
                    const double2 v = *(const double2 *)pr;
                    av[r][0] = v.x, av[r][1] = v.y;
                } else {
                    const float2 v = *(const float2 *)pr;
                    av[r][0] = v.x, av[r][1] = v.y;
                }
            } else {
#pragma unroll
                for (int u = 0; u < VEC; ++u) av[r][u] = (T)0;
            }
        }
#pragma unroll
        for (int t = 0; t < MAXNT; ++t) {
            if (t >= nt) break;
            T bv[VEC];
            const T *dr = D + (size_t)(16 * t + lr) * ldd + j0;
            if constexpr (VEC == 4) {
                const float4 v = *(const float4 *)dr;
                bv[0] = v.x, bv[1] = v.y, bv[2] = v.z, bv[3] = v.w;
            } else {
                const double2 v = *(const double2 *)dr;
                bv[0] = v.x, bv[1] = v.y;
            }
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    if constexpr (F64)
                        acc[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r][u], bv[u], acc[r][t], 0, 0, 0);
                    else
                        acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][u], bv[u], acc[r][t], 0, 0, 0);
                }
        }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < MAXNT; ++t) {
            if (t >= nt) break;
            const int n = 16 * t + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long row = row0 + 16 * r + (F64 ? lk + 4 * q : 4 * lk + q);
                if (row >= nrows) continue;
                const size_t o = (size_t)row * ncp + n;
                if (OUT == 0) {
                    ((double *)c_out)[o] = (double)acc[r][t][q];
                } else if (OUT == 1) {
                    ((float *)c_out)[o] = (float)acc[r][t][q];
                } else {
                    const float v = (float)acc[r][t][q];
                    const uint16_t h = bf16_rne(v);
                    ((uint16_t *)c_out)[o] = h;
                    if (c_lo) c_lo[o] = bf16_rne(v - bf16_val(h));
                }
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
        U4 val = {0u, 0u, 0u, 0u}, vlo = {0u, 0u, 0u, 0u};
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
            U4 av[kRowTilesPerWave], avl[kRowTilesPerWave];
#pragma unroll
            for (int i = 0; i < kRowTilesPerWave; ++i) {
                if (rt[i] >= RT) continue;
                const size_t off = (size_t)(16 * rt[i] + lr) * ncp + kof;
                av[i] = *(const U4 *)(brow + off);
                if (X3) avl[i] = *(const U4 *)(blo + off);
            }
            // consecutive MFMAs target different accumulators
            if constexpr (PREC == BLAST_FP64) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < kRowTilesPerWave; ++i) {
                        if (rt[i] >= RT) continue;
                        const double a = __builtin_bit_cast(d2v, av[i])[u];
#pragma unroll
                        for (int j = 0; j < BTN; ++j) {
                            if (16 * j >= nb) continue;
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, __builtin_bit_cast(d2v, bv[j])[u],
                                                                             acc[i][j], 0, 0, 0);
                        }
                    }
            } else if constexpr (PREC == BLAST_FP32) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int i = 0; i < kRowTilesPerWave; ++i) {
                        if (rt[i] >= RT) continue;
                        const float a = __builtin_bit_cast(f4v, av[i])[u];
#pragma unroll
                        for (int j = 0; j < BTN; ++j) {
                            if (16 * j >= nb) continue;
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, __builtin_bit_cast(f4v, bv[j])[u],
                                                                             acc[i][j], 0, 0, 0);
                        }
                    }
            } else {
#pragma unroll
                for (int i = 0; i < kRowTilesPerWave; ++i) {
                    if (rt[i] >= RT) continue;
                    const bf8 a = __builtin_bit_cast(bf8, av[i]);
#pragma unroll
                    for (int j = 0; j < BTN; ++j) {
                        if (16 * j >= nb) continue;
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf8, bv[j]),
                                                                            acc[i][j], 0, 0, 0);
                    }
                }
                if constexpr (X3) {
#pragma unroll
                    for (int i = 0; i < kRowTilesPerWave; ++i) {
                        if (rt[i] >= RT) continue;
                        const bf8 a = __builtin_bit_cast(bf8, av[i]), al = __builtin_bit_cast(bf8, avl[i]);
#pragma unroll
                        for (int j = 0; j < BTN; ++j) {
                            if (16 * j >= nb) continue;
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf8, bvl[j]),
                                                                                acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, __builtin_bit_cast(bf8, bv[j]),
                                                                                acc[i][j], 0, 0, 0);
                        }
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
// R-quadrature on MFMA: per (chi_a, cosmology) the product Y[row][bin] = sum_b w[b][row] Khat[b][bin]
// with Khat[b][bin] = wR_b K_bin(R_b chi_a).  M = rows (wave w owns row tiles w, w+4, ...),
// N = bins (one or two 16-wide tiles), K = b, staged through LDS 16 b at a time with 16-byte
// loads.  Y layout [beta][row][a][NBP] (contiguous per row for the chi-quadrature).
template <bool F64, int NBT>
__global__ __launch_bounds__(256) void quad_y_mfma_kernel(const typename std::conditional<F64, double, float>::type
                                                              *__restrict__ w,
                                                          const double *__restrict__ Kchi2,
                                                          const double *__restrict__ wR, int NP, int nR, int n_chi,
                                                          int rows_pad, int nbins,
                                                          typename std::conditional<F64, double, float>::type
                                                              *__restrict__ Y) {
    using T = typename std::conditional<F64, double, float>::type;
    using Acc = typename std::conditional<F64, d4, f4>::type;
    constexpr int NBP = 16 * NBT;
    constexpr int RTW = 5;
    constexpr int BCH = 16;  // b per LDS chunk
    extern __shared__ __align__(16) unsigned char smem_q[];
    const int a = blockIdx.x, beta = blockIdx.y;
    const int nRc = (nR + BCH - 1) / BCH * BCH;
    T *Kh = (T *)smem_q;                       // [nRc][NBP]
    T *Ws = Kh + (size_t)nRc * NBP;            // [BCH][rows_pad]
    for (int i = threadIdx.x; i < nRc * NBP; i += blockDim.x) {
        const int b = i / NBP, bin = i % NBP;
        double v = 0.0;
        if (b < nR && bin < nbins) v = wR[b] * Kchi2[(((size_t)beta * nbins + bin) * n_chi + a) * nR + b];
        Kh[i] = (T)v;
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int RT = rows_pad >> 4;
    const T *wa = w + ((size_t)beta * NP + (size_t)a * nR) * rows_pad;
    constexpr int V = 16 / sizeof(T);
    for (int pass = 0; pass * 4 * RTW < RT; ++pass) {
        Acc acc[RTW][NBT];
#pragma unroll
        for (int i = 0; i < RTW; ++i)
#pragma unroll
            for (int j = 0; j < NBT; ++j) acc[i][j] = Acc{0, 0, 0, 0};
        for (int b0 = 0; b0 < nRc; b0 += BCH) {
            __syncthreads();
            const int nvec = BCH * rows_pad / V;
            for (int i = threadIdx.x; i < nvec; i += blockDim.x) {
                const int bb = (i * V) / rows_pad, rr = (i * V) % rows_pad;
                U4 v = {0u, 0u, 0u, 0u};
                if (b0 + bb < nR) v = *(const U4 *)(wa + (size_t)(b0 + bb) * rows_pad + rr);
                *(U4 *)(Ws + (size_t)bb * rows_pad + rr) = v;
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < BCH / 4; ++s) {
                const int b = 4 * s + lk;
                T bv[NBT];
#pragma unroll
                for (int j = 0; j < NBT; ++j) bv[j] = Kh[(size_t)(b0 + b) * NBP + 16 * j + lr];
#pragma unroll
                for (int i = 0; i < RTW; ++i) {
                    const int rt = pass * 4 * RTW + wv + 4 * i;
                    if (rt >= RT) continue;
                    const T av = Ws[(size_t)b * rows_pad + 16 * rt + lr];
#pragma unroll
                    for (int j = 0; j < NBT; ++j) {
                        if constexpr (F64)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[j], acc[i][j], 0, 0, 0);
                        else
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[j], acc[i][j], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RTW; ++i) {
            const int rt = pass * 4 * RTW + wv + 4 * i;
            if (rt >= RT) continue;
#pragma unroll
            for (int j = 0; j < NBT; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * rt + (F64 ? lk + 4 * r : 4 * lk + r);
                    Y[(((size_t)beta * rows_pad + row) * n_chi + a) * NBP + 16 * j + lr] = acc[i][j][r];
                }
        }
    }
}

struct Slots {
    int s[3];
};

struct EllSel {
    int n_out;
    int16_t idx[kMaxEll];
};

// chi-quadrature and pair assembly, one work-group per (type slot x output multipole, cosmology):
//   C[beta][p][io] = N_t(l) sum_a wchi_a chi_a [K_i(chi_a) Y[a][row][j] + K_j(chi_a) Y[a][row][i]]
// The row's Y[a][bin] and the weighted kernels are staged in LDS; each wave reduces pairs over a.
template <typename YT>
__global__ __launch_bounds__(256) void quad_c_row_kernel(const YT *__restrict__ Y, int nbp,
                                                         const double *__restrict__ Kchi,
                                                         const double *__restrict__ wchi,
                                                         const double *__restrict__ chi,
                                                         const double *__restrict__ pref, int n_chi, int rows_pad,
                                                         int n_ell, Slots slot_type, int ng, int ns, uint32_t types,
                                                         int npairs, EllSel sel, double *__restrict__ C) {
    extern __shared__ double smem_c[];
    const int nbins = ng + ns;
    double *Ys = smem_c;                         // [nbins][n_chi]
    double *Ks = smem_c + (size_t)nbins * n_chi; // [nbins][n_chi], weighted
    const int slot = blockIdx.x / sel.n_out, io = blockIdx.x % sel.n_out;
    const int beta = blockIdx.y;
    const int t = slot_type.s[slot];
    if (!(t & types)) return;
    const int row = slot * n_ell + sel.idx[io];
    for (int i = threadIdx.x; i < nbins * n_chi; i += blockDim.x) {
        const int a = i / nbins, bin = i % nbins;
        Ys[bin * n_chi + a] = (double)Y[(((size_t)beta * rows_pad + row) * n_chi + a) * nbp + bin];
        const int bin2 = i / n_chi, a2 = i % n_chi;
        Ks[bin2 * n_chi + a2] = wchi[a2] * chi[a2] * Kchi[((size_t)beta * nbins + bin2) * n_chi + a2];
    }
    __syncthreads();
    // pairs of this type and their position in the output
    int off = 0, ntp, ni, nj;
    if (t == BLAST_GG) {
        ntp = ng * (ng + 1) / 2;
    } else if (t == BLAST_GS) {
        off = (types & BLAST_GG) ? ng * (ng + 1) / 2 : 0;
        ntp = ng * ns;
    } else {
        off = ((types & BLAST_GG) ? ng * (ng + 1) / 2 : 0) + ((types & BLAST_GS) ? ng * ns : 0);
        ntp = ns * (ns + 1) / 2;
    }
    (void)ni;
    (void)nj;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double pf = pref[row];
    for (int q = wv; q < ntp; q += 4) {
        int i, j;
        if (t == BLAST_GS) {
            i = q / ns;
            j = ng + q % ns;
        } else {
            const int n = t == BLAST_GG ? ng : ns, base = t == BLAST_GG ? 0 : ng;
            int r = 0, p = q;
            while (p >= n - r) {
                p -= n - r;
                ++r;
            }
            i = base + r;
            j = base + r + p;
        }
        double acc = 0.0;
        for (int a = lane; a < n_chi; a += 64)
            acc += Ks[i * n_chi + a] * Ys[j * n_chi + a] + Ks[j * n_chi + a] * Ys[i * n_chi + a];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) C[((size_t)beta * npairs + off + q) * sel.n_out + io] = pf * acc;
    }
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
    const int nbp = nbins <= 16 ? 16 : 32;
    off += align256((size_t)batch * p->n_chi * p->rows_pad * nbp * (prec == BLAST_FP64 ? 8 : 4));
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

// gfx950 has 160 KB of LDS per CU; kernels whose tiles exceed HIP's default 64 KB dynamic limit
// are allowed the full amount once per process.
hipError_t allow_large_lds() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        const int lim = 160 * 1024;
        const void *fns[] = {
            (const void *)project_mfma_kernel<float, false, 1>, (const void *)project_mfma_kernel<float, false, 2>,
            (const void *)project_mfma_kernel<double, false, 1>, (const void *)project_mfma_kernel<double, false, 2>,
            (const void *)quad_y_mfma_kernel<true, 1>, (const void *)quad_y_mfma_kernel<true, 2>,
            (const void *)quad_y_mfma_kernel<false, 1>, (const void *)quad_y_mfma_kernel<false, 2>,
        };
        for (const void *f : fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
            if (e != hipSuccess) err = e;
        }
    });
    return err;
}

template <typename Mark>
blast_status forward_impl(blast_plan *p, const blast_cl_args *a, hipStream_t s, Mark &mark) {
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
    if ((size_t)nbins * p->n_chi * 2 * sizeof(double) > 64 * 1024)
        return set_error("(n_g + n_s) * n_chi must be <= 4096"), BLAST_E_UNSUPPORTED;

    BLAST_HIP_TRY(allow_large_lds());
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
    void *Y = ws + L.y;
    const int nbp = nbins <= 16 ? 16 : 32;
    const long nrows = (long)a->batch * p->NP;
    const int N = p->n_cheb, ncp = p->nc_pad;

    // 1. projection
    mark(0);
    {
        const bool f64 = prec == BLAST_FP64;
        const bool p64 = a->p_dtype == 0;
        const int out = f64 ? 0 : (prec == BLAST_FP32 ? 1 : 2);
        if (N % (f64 ? 8 : 16) == 0) {
            dim3 grid((unsigned)((nrows + 255) / 256));
            const size_t shp = f64 ? 0 : (size_t)ncp * (N + 4) * sizeof(float);
#define BLAST_PROJ(PT, F, O, D)                                                                                  \
    hipLaunchKernelGGL((project_mfma_kernel<PT, F, O>), grid, dim3(256), shp, s, (const PT *)a->P, D, N, ncp, nrows, \
                       c, clo)
            if (f64 && p64) BLAST_PROJ(double, true, 0, p->d_dctn64);
            if (f64 && !p64) BLAST_PROJ(float, true, 0, p->d_dctn64);
            if (!f64 && p64 && out == 1) BLAST_PROJ(double, false, 1, p->d_dctn32);
            if (!f64 && p64 && out == 2) BLAST_PROJ(double, false, 2, p->d_dctn32);
            if (!f64 && !p64 && out == 1) BLAST_PROJ(float, false, 1, p->d_dctn32);
            if (!f64 && !p64 && out == 2) BLAST_PROJ(float, false, 2, p->d_dctn32);
#undef BLAST_PROJ
        } else {
            dim3 grid((unsigned)((nrows + kProjRows - 1) / kProjRows));
#define BLAST_PROJ(PT, AT, O, D) \
    hipLaunchKernelGGL((project_kernel<PT, AT, O>), grid, dim3(256), 0, s, (const PT *)a->P, D, N, ncp, nrows, c, clo)
            if (f64 && p64) BLAST_PROJ(double, double, 0, p->d_dct64);
            if (f64 && !p64) BLAST_PROJ(float, double, 0, p->d_dct64);
            if (!f64 && p64 && out == 1) BLAST_PROJ(double, float, 1, p->d_dct32);
            if (!f64 && p64 && out == 2) BLAST_PROJ(double, float, 2, p->d_dct32);
            if (!f64 && !p64 && out == 1) BLAST_PROJ(float, float, 1, p->d_dct32);
            if (!f64 && !p64 && out == 2) BLAST_PROJ(float, float, 2, p->d_dct32);
#undef BLAST_PROJ
        }
    }
    // 2. contraction
    mark(1);
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
    mark(2);
    {
        dim3 grid(p->n_chi, a->batch);
        const int nRc = (p->n_R + 15) / 16 * 16;
        if (prec == BLAST_FP64) {
            const size_t sh = ((size_t)nRc * nbp + 16 * (size_t)p->rows_pad) * sizeof(double);
            if (nbp == 16)
                hipLaunchKernelGGL((quad_y_mfma_kernel<true, 1>), grid, dim3(256), sh, s, (const double *)w, a->K_chi2,
                                   p->d_wR, p->NP, p->n_R, p->n_chi, p->rows_pad, nbins, (double *)Y);
            else
                hipLaunchKernelGGL((quad_y_mfma_kernel<true, 2>), grid, dim3(256), sh, s, (const double *)w, a->K_chi2,
                                   p->d_wR, p->NP, p->n_R, p->n_chi, p->rows_pad, nbins, (double *)Y);
        } else {
            const size_t sh = ((size_t)nRc * nbp + 16 * (size_t)p->rows_pad) * sizeof(float);
            if (nbp == 16)
                hipLaunchKernelGGL((quad_y_mfma_kernel<false, 1>), grid, dim3(256), sh, s, (const float *)w, a->K_chi2,
                                   p->d_wR, p->NP, p->n_R, p->n_chi, p->rows_pad, nbins, (float *)Y);
            else
                hipLaunchKernelGGL((quad_y_mfma_kernel<false, 2>), grid, dim3(256), sh, s, (const float *)w, a->K_chi2,
                                   p->d_wR, p->NP, p->n_R, p->n_chi, p->rows_pad, nbins, (float *)Y);
        }
        mark(3);
        Slots st{{p->tslot_type[0], p->tslot_type[1], p->tslot_type[2]}};
        dim3 g2((unsigned)(p->nt * sel.n_out), a->batch);
        const size_t sh2 = (size_t)nbins * p->n_chi * 2 * sizeof(double);
        if (prec == BLAST_FP64)
            hipLaunchKernelGGL((quad_c_row_kernel<double>), g2, dim3(256), sh2, s, (const double *)Y, nbp, a->K_chi,
                               p->d_wchi, p->d_chi, p->d_pref, p->n_chi, p->rows_pad, p->n_ell, st, ng, ns, a->types,
                               npairs, sel, a->C);
        else
            hipLaunchKernelGGL((quad_c_row_kernel<float>), g2, dim3(256), sh2, s, (const float *)Y, nbp, a->K_chi,
                               p->d_wchi, p->d_chi, p->d_pref, p->n_chi, p->rows_pad, p->n_ell, st, ng, ns, a->types,
                               npairs, sel, a->C);
        mark(4);
    }
    BLAST_HIP_TRY(hipGetLastError());
    return BLAST_OK;
}

blast_status forward(blast_plan *p, const blast_cl_args *a, hipStream_t s) {
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool prof = false;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        prof = p->profile;
    }
    if (prof) {
        for (int i = 0; i < 5; ++i)
            if (hipEventCreate(&ev[i]) != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
                return set_error("hipEventCreate failed"), BLAST_E_HIP;
            }
    }
    auto mark = [&](int i) {
        if (prof) (void)hipEventRecord(ev[i], s);
    };
    blast_status st = forward_impl(p, a, s, mark);
    if (prof) {
        if (st == BLAST_OK) {
            std::lock_guard<std::mutex> lk(p->mu);
            for (int i = 0; i < 5; ++i) p->prof_events.push_back(ev[i]);
        } else {
            for (int i = 0; i < 5; ++i) (void)hipEventDestroy(ev[i]);
        }
    }
    return st;
}

}  // namespace blast
