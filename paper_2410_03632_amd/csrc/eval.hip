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
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

typedef uint32_t U4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct TypeTag {
    using type = T;
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

// FP32 projection for N % 8 == 0, with the even/odd split of the DCT-II.
// With u_j = P_j + P_{N-1-j} and v_j = P_j - P_{N-1-j} (j < N/2), and D[n][N-1-j] = (-1)^n D[n][j],
//     c_{2m} = sum_{j<N/2} D[2m][j] u_j,      c_{2m+1} = sum_{j<N/2} D[2m+1][j] v_j,
// two [rows x N/2] x [N/2 x N/2] products: half the MFMA work of the plain product.  N/2 is padded
// to Hp (a multiple of 16) with zero weights, so the nc_pad = 2 Hp outputs of a row come out with
// exact zeros past N.  Each wave owns split_rt() row tiles and every even and odd output tile; the
// P values of step s+1 are loaded while step s runs.  A lane stores (c_{2m}, c_{2m+1}) as one
// 8-byte pair.
constexpr int split_rt() { return 2; }
// the FP16X3 projection's launch order: the cosmology blocks of kProjPG consecutive 16-point blocks
// next to each other (measured 2.5 % faster than the point blocks of one cosmology block)
constexpr long kProjPG = 8;
constexpr int kProjPasses = 8;  // passes of 4 cosmologies per work-group of the FP16X3 projection

// NT = Hp / 16 output tiles per parity (1..4) and as many K steps: with both known at compile time
// the step loop unrolls and every load is unconditional (rows past the end read the last row and
// are never stored), so the compiler can wait for exactly the loads a step needs and the next
// step's loads stay in flight under the current step's MFMAs.
// OUT: 1 -> float c, 2 -> BF16 hi (+ lo when c_lo != nullptr); the FP16X3 output has a kernel of its
// own (project_h16_kernel).
template <typename PT, int OUT, int NT>
__global__ __launch_bounds__(256) void project_split_kernel(const PT *__restrict__ P, const float *__restrict__ Dn,
                                                            int N, int ncp, long nrows, void *__restrict__ c_out,
                                                            uint16_t *__restrict__ c_lo) {
    constexpr int RT = split_rt(), VEC = 4, KSTEP = 16;
    extern __shared__ __align__(16) unsigned char smem_s[];
    const int H = N / 2;
    constexpr int Hp = 16 * NT, hs = Hp + 4;  // LDS row stride: 16 bytes of padding
    float *De = (float *)smem_s, *Do = De + (size_t)Hp * hs;
    for (int i = threadIdx.x; i < Hp * (Hp / 4); i += blockDim.x) {
        const int m = i / (Hp / 4), q = i % (Hp / 4);
        float4 e = make_float4(0.f, 0.f, 0.f, 0.f), o = e;
        if (m < H && 4 * q < H) {
            e = *(const float4 *)(Dn + (size_t)(2 * m) * N + 4 * q);
            o = *(const float4 *)(Dn + (size_t)(2 * m + 1) * N + 4 * q);
        }
        *(float4 *)(De + (size_t)m * hs + 4 * q) = e;
        *(float4 *)(Do + (size_t)m * hs + 4 * q) = o;
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const long row0 = (long)blockIdx.x * (64 * RT) + 16 * RT * w;
    const PT *prow[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) prow[r] = P + min(row0 + 16 * r + lr, nrows - 1) * (long)N;
    f4 ae[RT][NT], ao[RT][NT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) ae[r][t] = ao[r][t] = f4{0, 0, 0, 0};

    // raw P values of one step: front[r] = P[j0 .. j0+3], back[r] = P[N-4-j0 .. N-1-j0]
    // past N/2 the weights are zero, so any finite P values will do: the loads are clamped to the
    // row's last 4-vector below N/2 (H % 4 == 0)
    auto load = [&](int st, float4 (&front)[RT], float4 (&back)[RT]) {
        const int j0 = min(st * KSTEP + lk * VEC, H - 4);
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const PT *pr = prow[r];
            if constexpr (sizeof(PT) == 4) {
                front[r] = *(const float4 *)(pr + j0);
                back[r] = *(const float4 *)(pr + N - 4 - j0);
            } else {
                const double2 f0 = *(const double2 *)(pr + j0), f1 = *(const double2 *)(pr + j0 + 2);
                const double2 b0 = *(const double2 *)(pr + N - 4 - j0), b1 = *(const double2 *)(pr + N - 2 - j0);
                front[r] = make_float4((float)f0.x, (float)f0.y, (float)f1.x, (float)f1.y);
                back[r] = make_float4((float)b0.x, (float)b0.y, (float)b1.x, (float)b1.y);
            }
        }
    };
    auto compute = [&](int st, const float4 (&front)[RT], const float4 (&back)[RT]) {
        const int j0 = st * KSTEP + lk * VEC;
        float u[RT][VEC], v[RT][VEC];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            // mirror of j0 + e is N-1-j0-e = (N-4-j0) + (3-e)
            u[r][0] = front[r].x + back[r].w, v[r][0] = front[r].x - back[r].w;
            u[r][1] = front[r].y + back[r].z, v[r][1] = front[r].y - back[r].z;
            u[r][2] = front[r].z + back[r].y, v[r][2] = front[r].z - back[r].y;
            u[r][3] = front[r].w + back[r].x, v[r][3] = front[r].w - back[r].x;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float4 de = *(const float4 *)(De + (size_t)(16 * t + lr) * hs + j0);
            const float4 dd = *(const float4 *)(Do + (size_t)(16 * t + lr) * hs + j0);
            const float dev[4] = {de.x, de.y, de.z, de.w}, dov[4] = {dd.x, dd.y, dd.z, dd.w};
#pragma unroll
            for (int e = 0; e < VEC; ++e)
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    ae[r][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(u[r][e], dev[e], ae[r][t], 0, 0, 0);
                    ao[r][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[r][e], dov[e], ao[r][t], 0, 0, 0);
                }
        }
    };
    float4 fr[2][RT], bk[2][RT];
    load(0, fr[0], bk[0]);
#pragma unroll
    for (int st = 0; st < NT; ++st) {
        if (st + 1 < NT) load(st + 1, fr[(st + 1) & 1], bk[(st + 1) & 1]);
        compute(st, fr[st & 1], bk[st & 1]);
    }
    // lane holds rows 16r + 4lk + q of output m = 16t + lr, i.e. n = 2m and 2m + 1
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = 2 * (16 * t + lr);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long row = row0 + 16 * r + 4 * lk + q;
                if (row >= nrows) continue;
                const size_t o = (size_t)row * ncp + n;
                const float ce = ae[r][t][q], co = ao[r][t][q];
                if (OUT == 1) {
                    *(float2 *)((float *)c_out + o) = make_float2(ce, co);
                } else {
                    const uint16_t he = bf16_rne(ce), ho = bf16_rne(co);
                    *(uint32_t *)((uint16_t *)c_out + o) = (uint32_t)he | ((uint32_t)ho << 16);
                    if (c_lo)
                        *(uint32_t *)(c_lo + o) = (uint32_t)bf16_rne(ce - bf16_val(he)) |
                                                   ((uint32_t)bf16_rne(co - bf16_val(ho)) << 16);
                }
            }
        }
}

// FP64 projection for N % 8 == 0 with the same even/odd split (FP64 path): v_mfma_f64_16x16x4f64,
// one 16-row tile per wave, the D halves in LDS as doubles.  The f64 result layout puts row
// 4 r + lk of the tile in register r of lane (m % 16) + 16 lk, so a lane stores rows 4 r + lk.
template <typename PT, int NT>
__global__ __launch_bounds__(256) void project_split64_kernel(const PT *__restrict__ P, const double *__restrict__ Dn,
                                                              int N, int ncp, long nrows, double *__restrict__ c_out) {
    constexpr int KSTEP = 16;
    extern __shared__ __align__(16) unsigned char smem_d[];
    const int H = N / 2;
    constexpr int Hp = 16 * NT, hs = Hp + 2;  // doubles per LDS row: 16 bytes of padding
    double *De = (double *)smem_d, *Do = De + (size_t)Hp * hs;
    {
        // the halves of D in pairs of doubles: all loads of a thread first (clamped, masked)
        constexpr int TOT = Hp * (Hp / 2), PER = (TOT + 255) / 256;
        double2 e[PER], o[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = min((int)threadIdx.x + 256 * u, TOT - 1);
            const int m = min(i / (Hp / 2), H - 1), q = min(i % (Hp / 2), H / 2 - 1);
            e[u] = *(const double2 *)(Dn + (size_t)(2 * m) * N + 2 * q);
            o[u] = *(const double2 *)(Dn + (size_t)(2 * m + 1) * N + 2 * q);
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + 256 * u;
            const int m = i / (Hp / 2), q = i % (Hp / 2);
            if (i < TOT) {
                const bool in = m < H && 2 * q < H;  // per component: a struct select went through scratch
                *(double2 *)(De + (size_t)m * hs + 2 * q) = make_double2(in ? e[u].x : 0.0, in ? e[u].y : 0.0);
                *(double2 *)(Do + (size_t)m * hs + 2 * q) = make_double2(in ? o[u].x : 0.0, in ? o[u].y : 0.0);
            }
        }
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const long row0 = (long)blockIdx.x * 64 + 16 * w;
    const PT *pr = P + min(row0 + lr, nrows - 1) * (long)N;
    d4 ae[NT], ao[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) ae[t] = ao[t] = d4{0, 0, 0, 0};
    // raw P values of one step: front = P[j0 .. j0+3], back = P[N-4-j0 .. N-1-j0] (clamped as in
    // the FP32 kernel: past N/2 the weights are zero)
    auto load = [&](int st, double (&front)[4], double (&back)[4]) {
        const int j0 = min(st * KSTEP + lk * 4, H - 4);
        if constexpr (sizeof(PT) == 8) {
            const double2 f0 = *(const double2 *)(pr + j0), f1 = *(const double2 *)(pr + j0 + 2);
            const double2 b0 = *(const double2 *)(pr + N - 4 - j0), b1 = *(const double2 *)(pr + N - 2 - j0);
            front[0] = f0.x, front[1] = f0.y, front[2] = f1.x, front[3] = f1.y;
            back[0] = b0.x, back[1] = b0.y, back[2] = b1.x, back[3] = b1.y;
        } else {
            const float4 f = *(const float4 *)(pr + j0), b = *(const float4 *)(pr + N - 4 - j0);
            front[0] = f.x, front[1] = f.y, front[2] = f.z, front[3] = f.w;
            back[0] = b.x, back[1] = b.y, back[2] = b.z, back[3] = b.w;
        }
    };
    auto compute = [&](int st, const double (&front)[4], const double (&back)[4]) {
        const int j0 = st * KSTEP + lk * 4;
        double u[4], v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {  // mirror of j0 + e is (N-4-j0) + (3-e)
            u[e] = front[e] + back[3 - e];
            v[e] = front[e] - back[3 - e];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double *de = De + (size_t)(16 * t + lr) * hs + j0, *dd = Do + (size_t)(16 * t + lr) * hs + j0;
            const double2 e0 = *(const double2 *)de, e1 = *(const double2 *)(de + 2);
            const double2 o0 = *(const double2 *)dd, o1 = *(const double2 *)(dd + 2);
            const double dev[4] = {e0.x, e0.y, e1.x, e1.y}, dov[4] = {o0.x, o0.y, o1.x, o1.y};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ae[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(u[e], dev[e], ae[t], 0, 0, 0);
                ao[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[e], dov[e], ao[t], 0, 0, 0);
            }
        }
    };
    double fr[2][4], bk[2][4];
    load(0, fr[0], bk[0]);
#pragma unroll
    for (int st = 0; st < NT; ++st) {
        if (st + 1 < NT) {
            load(st + 1, fr[(st + 1) & 1], bk[(st + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);  // keep the next step's loads ahead of these MFMAs
        }
        compute(st, fr[st & 1], bk[st & 1]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = 2 * (16 * t + lr);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long row = row0 + 4 * r + lk;
            if (row < nrows) *(double2 *)(c_out + (size_t)row * ncp + n) = make_double2(ae[t][r], ao[t][r]);
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

// Work-group -> (point ab, cosmology tile bt) for the per-point contractions over a 1-D grid of
// point_tile_grid(NP, nBT) work-groups.  Work-groups are dealt round-robin over the 8 XCDs; the
// numbering gives each XCD a contiguous range of points with all their tiles in a row, so that a
// point's basis rows come from HBM once and from that XCD's L2 for its other tiles.  Spare
// work-groups (the grid is rounded up to a multiple of 8) return false.
__device__ inline bool point_tile(int NP, int nBT, int &ab, int &bt) {
    const int units = NP * nBT, per = (units + 7) / 8;
    const int u = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (u >= units) return false;
    ab = u / nBT;
    bt = u % nBT;
    return true;
}
inline dim3 point_tile_grid(int NP, int nBT) { return dim3((unsigned)((NP * nBT + 7) / 8 * 8)); }

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
template <>
struct Cfg<BLAST_FP16X3> {
    using E = uint16_t;
    using Acc = f4;
    static constexpr int VEC = 8, BT = 64;
};

// one 16x16x32 MFMA on 16-bit operands held as bit patterns: FP16 for FP16X3, BF16 otherwise
template <int PREC>
__device__ inline f4 mfma16(U4 a, U4 b, f4 c) {
    if constexpr (PREC == BLAST_FP16X3)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                       0);
}

// FP16X3 projection on FP16 MFMA.  The even/odd split of project_split_kernel (c_2m from
// u_j = P_j + P_{N-1-j}, c_2m+1 from v_j = P_j - P_{N-1-j}, j < N/2), with u, v and the matrix
// halves as FP16 hi + lo pairs and the three products hi*hi + hi*lo + lo*hi of each 32-column step
// on v_mfma_f32_16x16x32_f16 (FP32 accumulate): a fifth of the MFMA cycles of the FP32 products,
// which the FP32 form could not hide under its HBM traffic.  Each row is scaled by s = 2^(13 - e),
// e = floor(log2 max|P_j|), before the split, so |u s|, |v s| < 2^15 stay in FP16's normal range;
// then c s (the scaled output, cs = 1 / s) comes straight out of the products, whose matrix factor
// 2^g (dct16_exp) is taken off exactly.  u and v carry 22 significant bits through the split, the
// matrix 22, and the dropped lo*lo term is 2^-22 of a product.
// A work-group takes 16 points x 4 npass cosmologies, in npass passes of 4 (one per wave), and
// writes c point-major, c[(point * batch + beta) * ncp + n], each point's 4 rows of a pass side by
// side; the operand table (32 KB at 128 nodes) is copied to LDS once per work-group (measured at
// full 3x2pt, batch 256: 1.48 ms with one pass, 1.31 with 4, 1.29 with 8).
template <typename PT, int NT>
__global__ __launch_bounds__(256) void project_h16_kernel(const PT *__restrict__ P, const uint16_t *__restrict__ Dh,
                                                          int N, int ncp, int g, long NP, int batch,
                                                          uint16_t *__restrict__ c_hi, uint16_t *__restrict__ c_lo,
                                                          float *__restrict__ cs, int npass) {
    constexpr int NK = (NT + 1) / 2, TAB = 2 * NT * NK * 2 * 64;
    __shared__ U4 tab[TAB];
    for (int i = threadIdx.x; i < TAB; i += 256) tab[i] = ((const U4 *)Dh)[i];
    __syncthreads();
    const long NPB = (NP + 15) / 16, NBB = (batch + 4 * npass - 1) / (4 * npass), L = blockIdx.x;
    const long grp = L / (kProjPG * NBB), rem = L % (kProjPG * NBB);
    const long pbk = grp * kProjPG + rem % kProjPG, bbk = rem / kProjPG;
    if (pbk >= NPB) return;  // uniform over the work-group (no barrier follows)
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const long pt0 = 16L * pbk;
    for (int it = 0; it < npass; ++it) {
        if (4 * npass * bbk + 4 * it >= batch) break;  // uniform over the work-group
        const int beta = 4 * npass * (int)bbk + 4 * it + w;
        const int H = N / 2;
        const PT *prow = P + ((long)min(beta, batch - 1) * NP + min(pt0 + lr, NP - 1)) * N;
        // the lane's columns of each step: j0 = 32 k + 8 lk + 4 h (h = 0, 1) and the mirrored ones;
        // chunks past N/2 (zero weights) read the row's last chunk below N/2 instead (H % 4 == 0)
        float4 fr[NK][2], bk[NK][2];
#pragma unroll
        for (int k = 0; k < NK; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                int j0 = 32 * k + 8 * lk + 4 * h;
                j0 = j0 < H ? j0 : H - 4;
                if constexpr (sizeof(PT) == 4) {
                    fr[k][h] = *(const float4 *)(prow + j0);
                    bk[k][h] = *(const float4 *)(prow + N - 4 - j0);
                } else {
                    const double2 f0 = *(const double2 *)(prow + j0), f1 = *(const double2 *)(prow + j0 + 2);
                    const double2 b0 = *(const double2 *)(prow + N - 4 - j0), b1 = *(const double2 *)(prow + N - 2 - j0);
                    fr[k][h] = make_float4((float)f0.x, (float)f0.y, (float)f1.x, (float)f1.y);
                    bk[k][h] = make_float4((float)b0.x, (float)b0.y, (float)b1.x, (float)b1.y);
                }
            }
        // the row's largest |P_j| (its four lanes together load every P_j of the row)
        float pm = 0.f;
#pragma unroll
        for (int k = 0; k < NK; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                pm = fmaxf(pm, fmaxf(fmaxf(fmaxf(fabsf(fr[k][h].x), fabsf(fr[k][h].y)),
                                           fmaxf(fabsf(fr[k][h].z), fabsf(fr[k][h].w))),
                                     fmaxf(fmaxf(fabsf(bk[k][h].x), fabsf(bk[k][h].y)),
                                           fmaxf(fabsf(bk[k][h].z), fabsf(bk[k][h].w)))));
        pm = fmaxf(pm, __shfl_xor(pm, 16));
        pm = fmaxf(pm, __shfl_xor(pm, 32));
        // e kept where 2^(13 - e) is a finite float; rows of zeros get s = 1
        const int e = pm > 0.f ? min(max(ilogbf(pm), -100), 127) : 13;
        const float mul = ldexpf(1.f, 13 - e);
        // A operands: lane (row lr, lk) holds columns 32 k + 8 lk .. + 7 of u s and v s, hi and lo
        U4 uh[NK], ul[NK], vh[NK], vl[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            h8 a, b, c, d;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // the mirror of column j0 + q is N - 1 - j0 - q = (N - 4 - j0) + (3 - q)
                const float f[4] = {fr[k][h].x, fr[k][h].y, fr[k][h].z, fr[k][h].w};
                const float r[4] = {bk[k][h].w, bk[k][h].z, bk[k][h].y, bk[k][h].x};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float u = (f[q] + r[q]) * mul, v = (f[q] - r[q]) * mul;  // exact scaling
                    const _Float16 uhi = (_Float16)u, vhi = (_Float16)v;
                    a[4 * h + q] = uhi;
                    b[4 * h + q] = (_Float16)(u - (float)uhi);
                    c[4 * h + q] = vhi;
                    d[4 * h + q] = (_Float16)(v - (float)vhi);
                }
            }
            uh[k] = __builtin_bit_cast(U4, a), ul[k] = __builtin_bit_cast(U4, b);
            vh[k] = __builtin_bit_cast(U4, c), vl[k] = __builtin_bit_cast(U4, d);
        }
        f4 ae[NT], ao[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            ae[t] = ao[t] = f4{0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const U4 *te = tab + dct16_off(0, t, k, 0, lane, NT, NK) / 8;
                const U4 *to = tab + dct16_off(1, t, k, 0, lane, NT, NK) / 8;
                const U4 eh = te[0], el = te[64], oh = to[0], ol = to[64];
                ae[t] = mfma16<BLAST_FP16X3>(uh[k], eh, ae[t]);
                ao[t] = mfma16<BLAST_FP16X3>(vh[k], oh, ao[t]);
                ae[t] = mfma16<BLAST_FP16X3>(uh[k], el, ae[t]);
                ao[t] = mfma16<BLAST_FP16X3>(vh[k], ol, ao[t]);
                ae[t] = mfma16<BLAST_FP16X3>(ul[k], eh, ae[t]);
                ao[t] = mfma16<BLAST_FP16X3>(vl[k], oh, ao[t]);
            }
        }
        // lane holds rows 4 lk + q (points pt0 + 4 lk + q) of output m = 16 t + lr, i.e. n = 2m, 2m + 1
        const float og = ldexpf(1.f, -g);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const long pt = pt0 + 4 * lk + q;
            const int eq = __shfl(e, 4 * lk + q);  // the scale exponent of that row
            if (pt >= NP || beta >= batch) continue;
            if (lr == 0) cs[(long)beta * NP + pt] = ldexpf(1.f, eq - 13);
            const size_t o = ((size_t)pt * batch + beta) * ncp;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int n = 2 * (16 * t + lr);
                const float ve = ae[t][q] * og, vo = ao[t][q] * og;  // exact: powers of two
                const _Float16 he = (_Float16)ve, ho = (_Float16)vo;
                const _Float16 le = (_Float16)(ve - (float)he), lo = (_Float16)(vo - (float)ho);
                *(uint32_t *)(c_hi + o + n) = (uint32_t)__builtin_bit_cast(uint16_t, he) |
                                              ((uint32_t)__builtin_bit_cast(uint16_t, ho) << 16);
                *(uint32_t *)(c_lo + o + n) = (uint32_t)__builtin_bit_cast(uint16_t, le) |
                                              ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
            }
        }
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

    int ab, tile;
    if (!point_tile(NP, (batch + BT - 1) / BT, ab, tile)) return;  // uniform over the work-group
    const int beta0 = tile * BT;
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

        // basis tiles of step s+1 are in flight while step s runs on the MFMA units
        auto loadA = [&](int st, U4(&dst)[kRowTilesPerWave], U4(&dstl)[kRowTilesPerWave]) {
            const int kof = st * KSTEP + lk * VEC;
#pragma unroll
            for (int i = 0; i < kRowTilesPerWave; ++i) {
                const int r = rt[i] < RT ? rt[i] : RT - 1;
                const size_t off = (size_t)(16 * r + lr) * ncp + kof;
                dst[i] = *(const U4 *)(brow + off);
                if (X3) dstl[i] = *(const U4 *)(blo + off);
            }
        };
        auto compute = [&](int st, const U4(&av)[kRowTilesPerWave], const U4(&avl)[kRowTilesPerWave]) {
            const int kof = st * KSTEP + lk * VEC;
            U4 bv[BTN], bvl[BTN];
#pragma unroll
            for (int j = 0; j < BTN; ++j) {
                bv[j] = *(const U4 *)(cs + (size_t)(16 * j + lr) * cst + kof);
                if (X3) bvl[j] = *(const U4 *)(cls + (size_t)(16 * j + lr) * cst + kof);
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
        };
        U4 a0[kRowTilesPerWave], a0l[kRowTilesPerWave];
        if constexpr (X3) {
            // hi and lo tiles together already fill the registers: no second buffer
            for (int st = 0; st < nsteps; ++st) {
                loadA(st, a0, a0l);
                compute(st, a0, a0l);
            }
        } else {
            U4 a1[kRowTilesPerWave], a1l[kRowTilesPerWave];
            loadA(0, a0, a0l);
            for (int st = 0; st < nsteps; st += 2) {
                if (st + 1 < nsteps) loadA(st + 1, a1, a1l);
                compute(st, a0, a0l);
                if (st + 1 < nsteps) {
                    if (st + 2 < nsteps) loadA(st + 2, a0, a0l);
                    compute(st + 1, a1, a1l);
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

// Mixed-precision contraction on the tiled basis copies (FP32, BF16, BF16x3).  One work-group per
// (point, batch tile of 64 cosmologies); its W = blockDim/64 waves each own kTilesPerWave adjacent
// 16-row tiles per pass, so that e.g. 18 row tiles split evenly over 6 waves.  Every basis load is
// a contiguous 1 KB (tiled layout); the c tile sits in LDS; the loads of step s+1 are in flight
// while step s runs on the MFMA units.
constexpr int kTilesPerWave = 3;

template <int PREC, int WPE = (PREC == BLAST_BF16X3 ? 2 : 4), int BTT = Cfg<PREC>::BT, int TPWT = kTilesPerWave>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WPE))) void contract_tiled_kernel(const typename Cfg<PREC>::E *__restrict__ basis,
                                                             const uint16_t *__restrict__ basis_lo,
                                                             const float *__restrict__ scale,
                                                             const typename Cfg<PREC>::E *__restrict__ c,
                                                             const uint16_t *__restrict__ c_lo, int batch, int NP,
                                                             int rows_pad, int ncp, float *__restrict__ w_out,
                                                             int cld) {
    using C = Cfg<PREC>;
    using E = typename C::E;
    constexpr int VEC = C::VEC, BT = BTT, BTN = BT / 16, TPW = TPWT;
    constexpr bool X3 = PREC == BLAST_BF16X3;
    constexpr int KSTEP = 4 * VEC;
    extern __shared__ __align__(16) unsigned char smem[];
    const int cst = ncp + 16 / (int)sizeof(E);
    E *cs = (E *)smem;
    uint16_t *cls = (uint16_t *)(smem + (size_t)BT * cst * sizeof(E));

    int ab, tile;
    if (!point_tile(NP, (batch + BT - 1) / BT, ab, tile)) return;  // uniform over the work-group
    const int beta0 = tile * BT;
    const int nb = min(BT, batch - beta0);
    const int vec_per_row = ncp / VEC;
    for (int i = threadIdx.x; i < BT * vec_per_row; i += blockDim.x) {
        const int bb = i / vec_per_row, v = i % vec_per_row;
        U4 val = {0u, 0u, 0u, 0u}, vlo = {0u, 0u, 0u, 0u};
        if (bb < nb) {
            // c rows of cld elements (ncp for the library's own c; n_cheb for a caller's nodal P,
            // whose granules past its end repeat the last one: their basis columns are zero)
            const size_t off = ((size_t)(beta0 + bb) * NP + ab) * cld + (size_t)min(v, cld / VEC - 1) * VEC;
            val = *(const U4 *)(c + off);
            if (X3) vlo = *(const U4 *)(c_lo + off);
        }
        *(U4 *)(cs + (size_t)bb * cst + v * VEC) = val;
        if (X3) *(U4 *)(cls + (size_t)bb * cst + v * VEC) = vlo;
    }
    __syncthreads();

    const int W = blockDim.x >> 6;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int RT = rows_pad / 16;
    const int nsteps = ncp / KSTEP;
    const size_t blk = (size_t)ab * rows_pad * ncp;
    const U4 *bt = (const U4 *)(basis + blk) + lane;
    const U4 *btl = X3 ? (const U4 *)(basis_lo + blk) + lane : nullptr;

    for (int pass = 0; pass * W * TPW < RT; ++pass) {
        const int rt0 = (pass * W + w) * TPW;
        if (rt0 >= RT) break;
        f4 acc[TPW][BTN];
#pragma unroll
        for (int i = 0; i < TPW; ++i)
#pragma unroll
            for (int j = 0; j < BTN; ++j) acc[i][j] = f4{0, 0, 0, 0};
        bool on[TPW];
#pragma unroll
        for (int i = 0; i < TPW; ++i) on[i] = rt0 + i < RT;

        auto loadA = [&](int st, U4(&dst)[TPW], U4(&dstl)[TPW]) {
#pragma unroll
            for (int i = 0; i < TPW; ++i) {
                const int r = on[i] ? rt0 + i : rt0;
                const size_t o = ((size_t)r * nsteps + st) * 64;
                dst[i] = bt[o];
                if (X3) dstl[i] = btl[o];
            }
        };
        auto compute = [&](int st, const U4(&av)[TPW], const U4(&avl)[TPW]) {
            const int kof = st * KSTEP + lk * VEC;
            U4 bv[BTN], bvl[BTN];
#pragma unroll
            for (int j = 0; j < BTN; ++j) {
                bv[j] = *(const U4 *)(cs + (size_t)(16 * j + lr) * cst + kof);
                if (X3) bvl[j] = *(const U4 *)(cls + (size_t)(16 * j + lr) * cst + kof);
            }
            if constexpr (PREC == BLAST_FP32) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int i = 0; i < TPW; ++i) {
                        if (!on[i]) continue;
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
                for (int i = 0; i < TPW; ++i) {
                    if (!on[i]) continue;
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
                    for (int i = 0; i < TPW; ++i) {
                        if (!on[i]) continue;
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
        };
        // basis steps PD - 1 ahead of the MFMAs (a ring of PD register sets; deeper with one row
        // tile per wave, whose step has the fewest MFMAs to cover a load)
        // Loads past the last step repeat it (unconditional, so that the compiler waits for exactly
        // the loads a step needs); the last nsteps % PD steps run after the loop.
        constexpr int PD = TPW == 1 ? 4 : 2;
        U4 ar[PD][TPW], arl[PD][TPW];
#pragma unroll
        for (int u = 0; u < PD - 1; ++u) loadA(min(u, nsteps - 1), ar[u], arl[u]);
        int st = 0;
        for (; st + PD <= nsteps; st += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                loadA(min(st + u + PD - 1, nsteps - 1), ar[(u + PD - 1) % PD], arl[(u + PD - 1) % PD]);
                compute(st + u, ar[u], arl[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < PD - 1; ++u)
            if (st + u < nsteps) compute(st + u, ar[u], arl[u]);
        // lane holds rows 16*rt + 4*lk + r for cosmology 16*j + lr
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (!on[i]) continue;
            const int row0 = 16 * (rt0 + i) + 4 * lk;
            float sc[4] = {1.f, 1.f, 1.f, 1.f};
            if (PREC != BLAST_FP32) {
#pragma unroll
                for (int r = 0; r < 4; ++r) sc[r] = scale[(size_t)ab * rows_pad + row0 + r];
            }
#pragma unroll
            for (int j = 0; j < BTN; ++j) {
                const int bb = 16 * j + lr;
                if (bb >= nb) continue;
                const size_t o = ((size_t)(beta0 + bb) * NP + ab) * rows_pad + row0;
                float4 v;
                v.x = acc[i][j][0] * sc[0];
                v.y = acc[i][j][1] * sc[1];
                v.z = acc[i][j][2] * sc[2];
                v.w = acc[i][j][3] * sc[3];
                *(float4 *)(w_out + o) = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// quadrature
// ---------------------------------------------------------------------------------------------
// R-quadrature: Y[beta][row][a][bin] = sum_b wR_b K_bin(R_b chi_a) w[beta][a][b][row].
// One thread owns V consecutive rows (one 16-byte load of w per b) of one chi_a and all NB
// (padded) bins; consecutive threads own consecutive row groups, so every load instruction of
// a wave reads a contiguous 1 KB.  The weighted kernels of the work-group's chi_a values sit in
// LDS.  Y layout [beta][row][a][NB] (contiguous per row for the chi-quadrature).
template <typename T, int NB>
__global__ __launch_bounds__(256) void quad_y_kernel(const T *__restrict__ w, const double *__restrict__ Kchi2,
                                                     const double *__restrict__ wR, int NP, int nR, int n_chi,
                                                     int rows_pad, int nbins, T *__restrict__ Y) {
    constexpr int V = 16 / sizeof(T);
    extern __shared__ __align__(16) unsigned char smem_q[];
    T *Kh = (T *)smem_q;  // [a - a_lo][b][NB]
    const int RQ = rows_pad / V;
    const int beta = blockIdx.y;
    const long g0 = (long)blockIdx.x * blockDim.x;
    const int a_lo = (int)(g0 / RQ);
    const int a_hi = min(n_chi - 1, (int)((g0 + blockDim.x - 1) / RQ));
    const int na = a_hi - a_lo + 1;
    for (int i = threadIdx.x; i < na * nR * NB; i += blockDim.x) {
        const int al = i / (nR * NB), b = (i / NB) % nR, bin = i % NB;
        double v = 0.0;
        if (bin < nbins) v = wR[b] * Kchi2[(((size_t)beta * nbins + bin) * n_chi + a_lo + al) * nR + b];
        Kh[i] = (T)v;
    }
    __syncthreads();
    const long g = g0 + threadIdx.x;
    const int a = (int)(g / RQ), rq = (int)(g % RQ);
    if (a >= n_chi) return;
    const T *kh = Kh + (size_t)(a - a_lo) * nR * NB;
    const T *wp = w + ((size_t)beta * NP + (size_t)a * nR) * rows_pad + (size_t)rq * V;
    T acc[V][NB];
#pragma unroll
    for (int r = 0; r < V; ++r)
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[r][q] = (T)0;
    // UB loads of w in flight; the weights of a b read 16 bytes at a time (NB is a multiple of 4)
    constexpr int UB = sizeof(T) == 8 ? 8 : 4, KV = 16 / sizeof(T);
    int b = 0;
    for (; b + UB <= nR; b += UB) {
        U4 v[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) v[u] = *(const U4 *)(wp + (size_t)(b + u) * rows_pad);
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const T *wv = (const T *)&v[u];
#pragma unroll
            for (int q0 = 0; q0 < NB; q0 += KV) {
                const U4 kk = *(const U4 *)(kh + (b + u) * NB + q0);
                const T *k = (const T *)&kk;
#pragma unroll
                for (int q = 0; q < KV; ++q)
#pragma unroll
                    for (int r = 0; r < V; ++r) acc[r][q0 + q] += wv[r] * k[q];
            }
        }
    }
    for (; b < nR; ++b) {
        const U4 v = *(const U4 *)(wp + (size_t)b * rows_pad);
        const T *wv = (const T *)&v;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const T k = kh[b * NB + q];
#pragma unroll
            for (int r = 0; r < V; ++r) acc[r][q] += wv[r] * k;
        }
    }
#pragma unroll
    for (int r = 0; r < V; ++r) {
        T *y = Y + (((size_t)beta * rows_pad + (size_t)rq * V + r) * n_chi + a) * NB;
#pragma unroll
        for (int q = 0; q < NB; q += 16 / sizeof(T)) {
            U4 o;
            T *op = (T *)&o;
#pragma unroll
            for (int e = 0; e < (int)(16 / sizeof(T)); ++e) op[e] = acc[r][q + e];
            *(U4 *)(y + q) = o;
        }
    }
}

// Fused contraction and R-quadrature (mixed precisions, no w_save): w never leaves the registers
// of the wave that makes it.
//   w[row][beta]          = sum_n Ttilde[a, b][row][n] c[beta][a, b][n]        (MFMA, per b)
//   Y[beta][row][a][bin] += w[row][beta] * Kt[a, b][beta][bin]               (VALU, per b)
// with Kt = wR_b K_bin(R_b chi_a).  Work-group = (chi_a, batch tile of 64, group of TR row
// tiles), 4*TR waves: wave (i, k) makes the 16 x 16 tile (row tile i, cosmologies 16k..16k+15)
// for every b and keeps Y for its 4 rows x NB bins.  Per b the TR basis tiles (tiled layout:
// contiguous 1 KB register images) and the 64 c rows are moved straight from global memory to
// LDS (global_load_lds_dwordx4, no registers), shared by the 4 waves of a row tile and the TR
// waves of a cosmology sub-tile.  Basis tiles run two b ahead (3 LDS buffers), c rows one b
// ahead (2 buffers); one barrier per b.  The c rows sit in LDS with their 16-byte granules
// permuted (granule v of row r at v ^ (r & 7)) so that the 16 rows read by one instruction
// spread over the banks.  Work-groups are numbered so that the row groups and batch tiles of
// one chi_a run together on one XCD (work-groups go round-robin over the 8 XCDs) and share c
// rows and basis tiles in its L2.  Y rows are written with stride NBP (zero padding), the layout
// of the chi-quadrature.
constexpr int kFusedTR = 3;

template <int PREC, int NS>
struct FusedShape {
    using E = typename Cfg<PREC>::E;
    static constexpr int VEC = Cfg<PREC>::VEC, KSTEP = 4 * VEC, ncp = NS * KSTEP;
    static constexpr int NPART = PREC == BLAST_BF16X3 || PREC == BLAST_FP16X3 ? 2 : 1;
    static constexpr int ROWB = ncp * (int)sizeof(E);                  // bytes of one c row
    static constexpr int A_CH = kFusedTR * NS * NPART;                 // 1 KB chunks of basis per b
    static constexpr int C_CH = 64 * ROWB * NPART / 1024;              // 1 KB chunks of c per b
    static constexpr int NW = 4 * kFusedTR;                            // waves
    static constexpr int A_PW = (A_CH + NW - 1) / NW, C_PW = (C_CH + NW - 1) / NW;  // per wave
    static constexpr size_t A_BUF = (size_t)A_CH * 1024, C_BUF = (size_t)C_CH * 1024;
    // per b also: kernel weights of the 64 cosmologies (<= 20 bins: <= 5 KB) and row scales
    static constexpr size_t X_BUF = 6 * 1024;
    static constexpr size_t LDS = 3 * A_BUF + 2 * (C_BUF + X_BUF);
};

__device__ inline void lds_dma16(const void *g, void *l) {
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)g,
                                     (void __attribute__((address_space(3))) *)l, 16, 0, 0);
}

// LDS reads of DMA-filled buffers.  Written as asm so that the compiler, which cannot always tell
// which buffer an LDS DMA in flight writes, adds no wait for the DMAs (the kernel orders them
// itself with explicit counts and barriers); each block waits for its own reads before it ends.
__device__ inline uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}
// f(integral_constant<I>) for I = B..N-1
template <int I, int N, typename F>
__device__ inline void static_for(F &f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>());
        static_for<I + 1, N>(f);
    }
}

// two (or four) 16-byte reads at base + compile-time offset, then a wait for them
template <int O0, int O1>
__device__ inline void lds_read2(uint32_t b0, uint32_t b1, U4 &r0, U4 &r1) {
    asm volatile("ds_read_b128 %0, %2 offset:%4\n\tds_read_b128 %1, %3 offset:%5\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(r0), "=&v"(r1)
                 : "v"(b0), "v"(b1), "i"(O0), "i"(O1)
                 : "memory");
}
template <int O0, int O1, int O2, int O3>
__device__ inline void lds_read4(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3, U4 &r0, U4 &r1, U4 &r2,
                                 U4 &r3) {
    asm volatile(
        "ds_read_b128 %0, %4 offset:%8\n\tds_read_b128 %1, %5 offset:%9\n\t"
        "ds_read_b128 %2, %6 offset:%10\n\tds_read_b128 %3, %7 offset:%11\n\ts_waitcnt lgkmcnt(0)"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
        : "v"(b0), "v"(b1), "v"(b2), "v"(b3), "i"(O0), "i"(O1), "i"(O2), "i"(O3)
        : "memory");
}

// six 16-byte reads (three at base a, three at base c, compile-time offsets), then a wait for them
template <int A0, int A1, int C0, int C1, int C2, int C3>
__device__ inline void lds_read6(uint32_t a, uint32_t c, U4 &r0, U4 &r1, U4 &r2, U4 &r3, U4 &r4, U4 &r5) {
    asm volatile(
        "ds_read_b128 %0, %6 offset:%8\n\tds_read_b128 %1, %6 offset:%9\n\t"
        "ds_read_b128 %2, %7 offset:%10\n\tds_read_b128 %3, %7 offset:%11\n\t"
        "ds_read_b128 %4, %7 offset:%12\n\tds_read_b128 %5, %7 offset:%13\n\ts_waitcnt lgkmcnt(0)"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5)
        : "v"(a), "v"(c), "i"(A0), "i"(A1), "i"(C0), "i"(C1), "i"(C2), "i"(C3)
        : "memory");
}

// FP32 contraction steps of the fused kernel, software-pipelined.  Each block issues the LDS reads
// of the next step, then the four v_mfma_f32_16x16x4_f32 of the current step (operand a[e], b[e]
// holds the K slice e of the step) into two accumulator chains (each MFMA one instruction behind
// the one it depends on, an exact overlap of SrcC and the previous result, which the hardware
// orders), and waits for its own reads before it ends, so no read is in flight outside the block.  The leading s_nop keeps the MFMAs two wait states clear of any VALU
// write of their operands.  The first block also reads the four 16-byte groups of kernel weights
// and starts the accumulators from zero; the last one reads nothing and ends with 32 wait states,
// so that the VALU may read the accumulators right after it.  From the first block's MFMAs to the
// end of the last one the wave runs at raised priority (s_setprio 3), so that the waves feeding
// the MFMA unit issue ahead of those doing address arithmetic or the R-sum.
#define BLAST_MFMA4_ACC                                                                               \
    "v_mfma_f32_16x16x4_f32 %[c0], %[a0], %[b0], %[c0]\n\t"                                        \
    "v_mfma_f32_16x16x4_f32 %[c1], %[a1], %[b1], %[c1]\n\t"                                        \
    "v_mfma_f32_16x16x4_f32 %[c0], %[a2], %[b2], %[c0]\n\t"                                        \
    "v_mfma_f32_16x16x4_f32 %[c1], %[a3], %[b3], %[c1]\n\t"
#define BLAST_AB_IN(av, bv)                                                                           \
    [a0] "v"(av[0]), [a1] "v"(av[1]), [a2] "v"(av[2]), [a3] "v"(av[3]), [b0] "v"(bv[0]), [b1] "v"(bv[1]), \
        [b2] "v"(bv[2]), [b3] "v"(bv[3])

template <int AO, int CO>
__device__ inline void mfma_first(uint32_t an, uint32_t cn, const uint32_t (&kq)[4], f4v av, f4v bv, U4 &ua, U4 &ub,
                                  U4 (&q)[4], f4 &c0, f4 &c1) {
    asm volatile(
        "ds_read_b128 %[na], %[ab] offset:%[ao]\n\t"
        "ds_read_b128 %[nb], %[cb] offset:%[co]\n\t"
        "ds_read_b128 %[q0], %[k0]\n\t"
        "ds_read_b128 %[q1], %[k1]\n\t"
        "ds_read_b128 %[q2], %[k2]\n\t"
        "ds_read_b128 %[q3], %[k3]\n\t"
        "s_setprio 3\n\t"
        "s_nop 1\n\t"
        "v_mfma_f32_16x16x4_f32 %[c0], %[a0], %[b0], 0\n\t"
        "v_mfma_f32_16x16x4_f32 %[c1], %[a1], %[b1], 0\n\t"
        "v_mfma_f32_16x16x4_f32 %[c0], %[a2], %[b2], %[c0]\n\t"
        "v_mfma_f32_16x16x4_f32 %[c1], %[a3], %[b3], %[c1]\n\t"
        "s_waitcnt lgkmcnt(0)"
        : [na] "=&v"(ua), [nb] "=&v"(ub), [q0] "=&v"(q[0]), [q1] "=&v"(q[1]), [q2] "=&v"(q[2]), [q3] "=&v"(q[3]),
          [c0] "=&v"(c0), [c1] "=&v"(c1)
        : [ab] "v"(an), [cb] "v"(cn), [ao] "i"(AO), [co] "i"(CO), [k0] "v"(kq[0]), [k1] "v"(kq[1]), [k2] "v"(kq[2]),
          [k3] "v"(kq[3]), BLAST_AB_IN(av, bv)
        : "memory");
}
template <int AO, int CO>
__device__ inline void mfma_mid(uint32_t an, uint32_t cn, f4v av, f4v bv, U4 &ua, U4 &ub, f4 &c0, f4 &c1) {
    asm volatile(
        "ds_read_b128 %[na], %[ab] offset:%[ao]\n\t"
        "ds_read_b128 %[nb], %[cb] offset:%[co]\n\t"
        "s_nop 1\n\t"
        BLAST_MFMA4_ACC
        "s_waitcnt lgkmcnt(0)"
        : [na] "=&v"(ua), [nb] "=&v"(ub), [c0] "+v"(c0), [c1] "+v"(c1)
        : [ab] "v"(an), [cb] "v"(cn), [ao] "i"(AO), [co] "i"(CO), BLAST_AB_IN(av, bv)
        : "memory");
}
__device__ inline void mfma_last(f4v av, f4v bv, f4 &c0, f4 &c1) {
    asm volatile(
        "s_nop 1\n\t"
        BLAST_MFMA4_ACC
        "s_setprio 0\n\t"
        "s_nop 15\n\t"
        "s_nop 15"
        : [c0] "+v"(c0), [c1] "+v"(c1)
        : BLAST_AB_IN(av, bv)
        : "memory");
}

// Split 16-bit contraction steps of the fused kernel (FP16X3, BF16X3), pipelined like the FP32
// steps: a block issues the four LDS reads of the next step (basis hi and lo, c hi and lo), runs the
// current step's hi*hi, hi*lo and lo*hi products into three accumulator chains (consecutive MFMAs
// never depend on each other) and waits for its reads.  The first block also reads the weight
// groups and the row scales and starts the accumulators from zero; the last one reads nothing and
// ends with 32 wait states before the VALU reads the accumulators.
#define BLAST_X3_STEP(OP, Z0, Z1, Z2)                                                                 \
    OP " %[c0], %[a], %[b], " Z0 "\n\t" OP " %[c1], %[a], %[bl], " Z1 "\n\t" OP " %[c2], %[al], %[b], " Z2 "\n\t"
#define BLAST_X3_READ4                                                                                \
    "ds_read_b128 %[na], %[ab] offset:%[ao]\n\t"                                                      \
    "ds_read_b128 %[nb], %[cb] offset:%[co]\n\t"                                                      \
    "ds_read_b128 %[nal], %[ab] offset:%[alo]\n\t"                                                    \
    "ds_read_b128 %[nbl], %[cb] offset:%[clo]\n\t"
template <int PREC, int AO, int ALO, int CO, int CLO>
__device__ inline void x3_first(uint32_t an, uint32_t cn, const uint32_t (&kq)[4], uint32_t sa, U4 a, U4 al, U4 b,
                                U4 bl, U4 &na, U4 &nb, U4 &nal, U4 &nbl, U4 (&q)[4], U4 &qs, f4 &c0, f4 &c1, f4 &c2) {
#define BLAST_X3_FIRST(OP)                                                                               \
    asm volatile(BLAST_X3_READ4                                                                          \
                 "ds_read_b128 %[q0], %[k0]\n\t"                                                         \
                 "ds_read_b128 %[q1], %[k1]\n\t"                                                         \
                 "ds_read_b128 %[q2], %[k2]\n\t"                                                         \
                 "ds_read_b128 %[q3], %[k3]\n\t"                                                         \
                 "ds_read_b128 %[qs], %[sa]\n\t"                                                         \
                 "s_setprio 3\n\t"                                                                      \
                 "s_nop 1\n\t" BLAST_X3_STEP(OP, "0", "0", "0") "s_waitcnt lgkmcnt(0)"                    \
                 : [na] "=&v"(na), [nb] "=&v"(nb), [nal] "=&v"(nal), [nbl] "=&v"(nbl), [q0] "=&v"(q[0]),       \
                   [q1] "=&v"(q[1]), [q2] "=&v"(q[2]), [q3] "=&v"(q[3]), [qs] "=&v"(qs), [c0] "=&v"(c0),       \
                   [c1] "=&v"(c1), [c2] "=&v"(c2)                                                        \
                 : [ab] "v"(an), [cb] "v"(cn), [ao] "i"(AO), [alo] "i"(ALO), [co] "i"(CO), [clo] "i"(CLO),     \
                   [k0] "v"(kq[0]), [k1] "v"(kq[1]), [k2] "v"(kq[2]), [k3] "v"(kq[3]), [sa] "v"(sa), [a] "v"(a), \
                   [al] "v"(al), [b] "v"(b), [bl] "v"(bl)                                                \
                 : "memory")
    if constexpr (PREC == BLAST_FP16X3)
        BLAST_X3_FIRST("v_mfma_f32_16x16x32_f16");
    else
        BLAST_X3_FIRST("v_mfma_f32_16x16x32_bf16");
#undef BLAST_X3_FIRST
}
template <int PREC, int AO, int ALO, int CO, int CLO>
__device__ inline void x3_mid(uint32_t an, uint32_t cn, U4 a, U4 al, U4 b, U4 bl, U4 &na, U4 &nb, U4 &nal, U4 &nbl,
                              f4 &c0, f4 &c1, f4 &c2) {
#define BLAST_X3_MID(OP)                                                                                 \
    asm volatile(BLAST_X3_READ4 "s_nop 1\n\t" BLAST_X3_STEP(OP, "%[c0]", "%[c1]", "%[c2]") "s_waitcnt lgkmcnt(0)" \
                 : [na] "=&v"(na), [nb] "=&v"(nb), [nal] "=&v"(nal), [nbl] "=&v"(nbl), [c0] "+v"(c0),         \
                   [c1] "+v"(c1), [c2] "+v"(c2)                                                          \
                 : [ab] "v"(an), [cb] "v"(cn), [ao] "i"(AO), [alo] "i"(ALO), [co] "i"(CO), [clo] "i"(CLO),     \
                   [a] "v"(a), [al] "v"(al), [b] "v"(b), [bl] "v"(bl)                                     \
                 : "memory")
    if constexpr (PREC == BLAST_FP16X3)
        BLAST_X3_MID("v_mfma_f32_16x16x32_f16");
    else
        BLAST_X3_MID("v_mfma_f32_16x16x32_bf16");
#undef BLAST_X3_MID
}
template <int PREC>
__device__ inline void x3_last(U4 a, U4 al, U4 b, U4 bl, f4 &c0, f4 &c1, f4 &c2) {
#define BLAST_X3_LAST(OP)                                                                                \
    asm volatile("s_nop 1\n\t" BLAST_X3_STEP(OP, "%[c0]", "%[c1]", "%[c2]") "s_setprio 0\n\t"            \
                 "s_nop 15\n\t"                                                                          \
                 "s_nop 15"                                                                              \
                 : [c0] "+v"(c0), [c1] "+v"(c1), [c2] "+v"(c2)                                           \
                 : [a] "v"(a), [al] "v"(al), [b] "v"(b), [bl] "v"(bl)                                    \
                 : "memory")
    if constexpr (PREC == BLAST_FP16X3)
        BLAST_X3_LAST("v_mfma_f32_16x16x32_f16");
    else
        BLAST_X3_LAST("v_mfma_f32_16x16x32_bf16");
#undef BLAST_X3_LAST
}

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding)
template <int N>
__device__ inline void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt out of range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

template <int PREC, int NB, int NBP, int NS>
__global__ __launch_bounds__(256 * kFusedTR) void contract_quad_kernel(
    const typename Cfg<PREC>::E *__restrict__ basis, const uint16_t *__restrict__ basis_lo,
    const float *__restrict__ scale, const typename Cfg<PREC>::E *__restrict__ c, const uint16_t *__restrict__ c_lo,
    const float *__restrict__ Kt, int batch, int n_chi, int n_R, int rows_pad, int nBT, int units, int n_ell,
    int nslots, int granges, float *__restrict__ Y, float *__restrict__ w_out, int cld) {
    using S = FusedShape<PREC, NS>;
    using E = typename S::E;
    constexpr int TR = kFusedTR, VEC = S::VEC, ncp = S::ncp, NPART = S::NPART;
    constexpr bool X3 = PREC == BLAST_BF16X3 || PREC == BLAST_FP16X3;
    constexpr int GPR = S::ROWB / 16;            // granules per c row
    // granule permutation mask: XOR by up to SWZ stays inside the row when SWZ + 1 divides GPR;
    // with 16 the 16 rows read by one instruction hit 16 distinct 16-byte bank groups
    constexpr int SWZ = GPR % 16 == 0 ? 15 : (GPR % 8 == 0 ? 7 : (GPR % 4 == 0 ? 3 : (GPR % 2 == 0 ? 1 : 0)));
    // the weights block [64 cosmologies][NB] is stored with the 4 granules of each row rotated by
    // (row >> 2) & 3 when NB = 16, so that the 16 rows read together fall in distinct bank groups
    constexpr bool KROT = NB == 16;
    // five distinct LDS objects, so that the compiler can tell the buffer a DMA writes from the
    // buffers the MFMA loop reads (and does not wait for the DMAs in flight)
    static_assert(S::LDS <= 160 * 1024, "LDS of the fused kernel");
    __shared__ __align__(1024) unsigned char A0[S::A_BUF], A1[S::A_BUF], A2[S::A_BUF];
    __shared__ __align__(1024) unsigned char C0[S::C_BUF + S::X_BUF], C1[S::C_BUF + S::X_BUF];

    const int groups = (rows_pad / 16 + TR - 1) / TR;
    const int per = (units + 7) / 8;
    const int unit = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (unit >= units) return;  // uniform over the work-group
    const int RT = rows_pad / 16;
    // the cosmology tiles of a row group next to each other (they read the same basis tiles): the
    // same time as row groups next to each other, with fewer HBM reads
    const int bt = unit % nBT, g = (unit / nBT) % groups, a = unit / (groups * nBT);
    const int rt0 = g * TR;
    const int ntile = min(TR, RT - rt0);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int ti = w >> 2, tk = w & 3;         // row tile, 16-cosmology sub-tile
    const int beta = bt * 64 + 16 * tk + lr;
    const int nb = min(64, batch - bt * 64);
    const size_t NP = (size_t)n_chi * n_R;
    const size_t pt_u4 = (size_t)RT * NS * 64;  // U4s per point in the tiled layout
    // waves whose row tile or cosmologies lie past the end only move data (small batches,
    // the last row group)
    const bool busy = ti < ntile && bt * 64 + 16 * tk < batch;
    // 4-bin groups the R-sum keeps for this wave's rows: a gg row pairs clustering bins only and
    // an ss row shear bins only (granges: per type slot s, first group in bits 6s..6s+2 and end in
    // bits 6s+3..6s+5); a tile that straddles slots keeps the union.  The other columns of Y stay
    // zero and are never read by the chi-quadrature.
    int gq0 = NB / 4, gq1 = 0;
    {
        const int r0 = 16 * (rt0 + min(ti, TR - 1));
        const int s0 = min(r0 / n_ell, nslots - 1), s1 = min((r0 + 15) / n_ell, nslots - 1);
        for (int sl = s0; sl <= s1; ++sl) {
            gq0 = min(gq0, (granges >> (6 * sl)) & 7);
            gq1 = max(gq1, (granges >> (6 * sl + 3)) & 7);
        }
    }
    // bit g set: group g is kept (a scalar mask, so the per-group tests stay off the VALU)
    const int gmask = __builtin_amdgcn_readfirstlane(gq1 > gq0 ? ((1 << gq1) - 1) & ~((1 << gq0) - 1) : 0);

    // every wave issues exactly A_PW basis and C_PW c DMA instructions per b, the basis ones last
    // (chunk indices past the end are clamped to the last chunk, which is then written more than once
    // with identical data), so the wait counts below are constants
    // Source addresses: a part that depends on b only (uniform, scalar registers) plus a per-lane
    // part that does not depend on b (computed once, before the loop).
    const U4 *srcA[S::A_PW];
#pragma unroll
    for (int k = 0; k < S::A_PW; ++k) {
        const int ch = min(w + k * S::NW, S::A_CH - 1);
        const int part = ch / (TR * NS), tl = (ch / NS) % TR, st = ch % NS;
        const int rt = min(rt0 + tl, RT - 1);
        srcA[k] = (const U4 *)(part ? (const void *)basis_lo : (const void *)basis) + ((size_t)rt * NS + st) * 64 + lane;
    }
    auto dma_A = [&](int b, unsigned char *__restrict__ buf) {
        const size_t ab = (size_t)a * n_R + (b < n_R ? b : n_R - 1);
#pragma unroll
        for (int k = 0; k < S::A_PW; ++k)
            lds_dma16(srcA[k] + ab * pt_u4, buf + (size_t)min(w + k * S::NW, S::A_CH - 1) * 1024);
    };
    // kernel weights Kt[ab][64 cosmologies][NB] (contiguous) and the row scales of the group, one
    // DMA per wave: waves 0..KCH-1 move weight chunks, wave KCH the scales (see dma_X for the others)
    constexpr int KCH = 64 * NB * 4 / 1024;
    static_assert(KCH + 1 <= S::NW && TR * 16 * 4 <= 1024 && KCH * 1024 + 1024 <= (int)S::X_BUF, "extra region");
    const int chX = min(w, KCH);
    const float *srcX;  // b-independent part: weights of (tile cosmology, bin), or the scales of the group's rows
    {
        int f = chX * 256 + lane * 4;                        // float index of the LDS position
        if (KROT) {                                          // position 4r + ((q + (r >> 2)) & 3) holds granule q
            const int r = f / 16, sp = (f / 4) & 3;
            f = r * 16 + ((sp - (r >> 2)) & 3) * 4;
        }
        const int bl = f / NB;
        // cosmologies past the batch read the tile's first weight instead (never used)
        srcX = chX < KCH ? Kt + (size_t)(bt * 64 + (bl < nb ? bl : 0)) * NB + (bl < nb ? f % NB : 0)
                         : (PREC != BLAST_FP32 ? scale + min(16 * rt0 + 4 * lane, rows_pad - 4) : Kt);
    }
    // per b: the weights advance by batch * NB floats per point, the scales by rows_pad
    const size_t strideX = chX < KCH ? (size_t)batch * NB : (PREC != BLAST_FP32 ? (size_t)rows_pad : 0);
    // waves past KCH repeat the scales on the FP32 path; on the 16-bit paths they move nothing (the
    // wait counts only keep the last A_PW DMAs, issued after this one, in flight).  Measured: the
    // FP32 path runs 3 % faster with the repeats, the split 16-bit path 3 % faster without.
    auto dma_X = [&](int b, unsigned char *__restrict__ buf) {
        if (PREC != BLAST_FP32 && w > KCH) return;
        const size_t ab = (size_t)a * n_R + (b < n_R ? b : n_R - 1);
        lds_dma16(srcX + ab * strideX, buf + S::C_BUF + (size_t)chX * 1024);
    };
    // FP16X3 coefficients are point-major ([point][beta][n]), the others cosmology-major with rows
    // of cld elements (ncp, or n_cheb for a caller's nodal P: granules past its end repeat the last
    // one, whose basis columns are zero)
    constexpr bool PM = PREC == BLAST_FP16X3;
    const size_t cstride = PM ? (size_t)batch * ncp : (size_t)cld;  // per point
    const void *srcC[S::C_PW];
#pragma unroll
    for (int k = 0; k < S::C_PW; ++k) {
        const int ch = min(w + k * S::NW, S::C_CH - 1);
        const int part = ch / (S::C_CH / NPART), chp = ch % (S::C_CH / NPART);
        // the lane's 16 bytes land at byte pos of the part's rows (a row need not divide 1 KB)
        const int pos = chp * 1024 + lane * 16;
        const int row = pos / S::ROWB, gp = (pos % S::ROWB) / 16;
        const int v = gp ^ (row & SWZ);          // granule stored at position gp
        const int bb = bt * 64 + (row < nb ? row : 0);
        srcC[k] = (part ? (const E *)c_lo : c) + (size_t)bb * (PM ? (size_t)ncp : (size_t)NP * cld) +
                  (PM ? v : min(v, cld / VEC - 1)) * VEC;
    }
    auto dma_C = [&](int b, unsigned char *__restrict__ buf) {
        const size_t ab = (size_t)a * n_R + (b < n_R ? b : n_R - 1);
#pragma unroll
        for (int k = 0; k < S::C_PW; ++k)
            lds_dma16((const E *)srcC[k] + ab * cstride, buf + (size_t)min(w + k * S::NW, S::C_CH - 1) * 1024);
    };

    float y[4][NB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < NB; ++j) y[r][j] = 0.f;
    const int crow = 16 * tk + lr;
    const int arow = min(ti, TR - 1) * NS * 64 + lane;  // U4 offset of the wave's basis tile

    // one b: buffers fixed at compile time (b mod 3 for the basis, b mod 2 for c)
    // (restrict: the compiler tags the LDS accesses with alias scopes, which its wait-count logic
    // needs before it will tell a DMA's target buffer from the buffers being read)
    auto step = [&](int b, const unsigned char *__restrict__ Ab, const unsigned char *__restrict__ Cb,
                    unsigned char *__restrict__ Cnext, unsigned char *__restrict__ Anext2) {
        // c(b), weights(b) and A(b) have landed once only A(b+1) may still be in flight; the
        // barrier is a plain s_barrier (a fence would drain every outstanding load)
        wait_vmcnt<S::A_PW>();
        __builtin_amdgcn_s_barrier();
        // the DMAs for b+1 and b+2 go out before any LDS read of b: the compiler then sees that
        // they write other buffers than the ones read here and adds no wait for them
        __builtin_amdgcn_sched_barrier(0);
        dma_C(b + 1, Cnext);
        dma_X(b + 1, Cnext);
        dma_A(b + 2, Anext2);
        __builtin_amdgcn_sched_barrier(0);
        if (!busy) return;
        float kt[NB];
        f4 wv;
        const uint32_t As = lds_addr(Ab) + (uint32_t)arow * 16;
        // granule (4 st + lk) of row crow sits at ((4 st + lk) ^ m) with m = crow & SWZ < 16, i.e. at
        // 16 (st >> 2) + 4 ((st & 3) ^ (m >> 2)) + (lk ^ (m & 3)): one base per st & 3
        const uint32_t Cr = lds_addr(Cb) + (uint32_t)crow * S::ROWB;
        const int m = crow & SWZ, mh = m >> 2, ml = lk ^ (m & 3);
        uint32_t Cq[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) Cq[k] = Cr + 16 * (4 * (k ^ mh) + ml);
        constexpr int NQ = NB / 4;  // 16-byte groups of weights per cosmology, 1..5
        const uint32_t kb = lds_addr(Cb + S::C_BUF) + (uint32_t)(16 * tk + lr) * (NB * 4);
        if constexpr (PREC == BLAST_FP32) {
            static_assert(NS >= 2, "pipelined FP32 steps");
            // weight groups of this b's cosmology (granules rotated when KROT); groups past NQ repeat
            // the last one
            uint32_t kq[4];
            const int rr = ((16 * tk + lr) >> 2) & 3;
#pragma unroll
            for (int j = 0; j < 4; ++j) kq[j] = KROT ? kb + 16 * ((j + rr) & 3) : kb + 16 * (j < NQ ? j : NQ - 1);
            U4 q[4], ua, ub;
            lds_read2<0, 0>(As, Cq[0], ua, ub);  // operands of step 0
            f4 c0, c1;
            // step st: basis at As + 1024 st, c at Cq[st & 3] + 256 (st >> 2)
            auto pipe = [&](auto stc) {
                constexpr int st = decltype(stc)::value;
                const f4v av = __builtin_bit_cast(f4v, ua), bv = __builtin_bit_cast(f4v, ub);
                if constexpr (st + 1 < NS) {
                    U4 na, nb;
                    if constexpr (st == 0)
                        mfma_first<1024, 0>(As, Cq[1], kq, av, bv, na, nb, q, c0, c1);
                    else
                        mfma_mid<(st + 1) * 1024, 256 * ((st + 1) >> 2)>(As, Cq[(st + 1) & 3], av, bv, na, nb, c0,
                                                                         c1);
                    ua = na;
                    ub = nb;
                } else {
                    mfma_last(av, bv, c0, c1);
                }
            };
            static_for<0, NS>(pipe);
#pragma unroll
            for (int j = 0; j < (NQ < 4 ? NQ : 4); ++j) {
                const f4v v = __builtin_bit_cast(f4v, q[j]);
                kt[4 * j] = v[0], kt[4 * j + 1] = v[1], kt[4 * j + 2] = v[2], kt[4 * j + 3] = v[3];
            }
            if constexpr (NQ > 4) {
                U4 q4, qd;
                lds_read2<64, 64>(kb, kb, q4, qd);
                const f4v v = __builtin_bit_cast(f4v, q4);
                kt[16] = v[0], kt[17] = v[1], kt[18] = v[2], kt[19] = v[3];
            }
            wv = c0 + c1;
            // a call that keeps w (FP32, for the adjoint) also stores the tile: 4 rows of one cosmology
            if (w_out && beta < batch && ti < ntile)
                *(float4 *)(w_out + ((size_t)beta * NP + (size_t)a * n_R + b) * rows_pad + 16 * (rt0 + ti) + 4 * lk) =
                    make_float4(wv[0], wv[1], wv[2], wv[3]);
        } else if constexpr (X3 && NS >= 2 && NB <= 16) {  // (20 bins: registers run out, steps below)
            constexpr int ALO = TR * NS * 1024;          // lo parts of the basis tiles
            constexpr int CLO = (int)(S::C_BUF / NPART);  // lo parts of the c rows
            uint32_t kq[4];
            const int rr = ((16 * tk + lr) >> 2) & 3;
#pragma unroll
            for (int j = 0; j < 4; ++j) kq[j] = KROT ? kb + 16 * ((j + rr) & 3) : kb + 16 * (j < NQ ? j : NQ - 1);
            const uint32_t sa =
                lds_addr(Cb + S::C_BUF + (size_t)KCH * 1024) + (uint32_t)(16 * min(ti, TR - 1) + 4 * lk) * 4;
            U4 q[4], qs, ua, ub, ual, ubl;
            lds_read4<0, 0, ALO, CLO>(As, Cq[0], As, Cq[0], ua, ub, ual, ubl);  // operands of step 0
            f4 c0, c1, c2;
            // step st: basis at As + 1024 st (+ ALO), c at Cq[st & 3] + 256 (st >> 2) (+ CLO)
            auto pipe = [&](auto stc) {
                constexpr int st = decltype(stc)::value;
                if constexpr (st + 1 < NS) {
                    constexpr int AO = (st + 1) * 1024, CO = 256 * ((st + 1) >> 2);
                    U4 na, nb, nal, nbl;
                    if constexpr (st == 0)
                        x3_first<PREC, AO, AO + ALO, CO, CO + CLO>(As, Cq[1], kq, sa, ua, ual, ub, ubl, na, nb, nal,
                                                                   nbl, q, qs, c0, c1, c2);
                    else
                        x3_mid<PREC, AO, AO + ALO, CO, CO + CLO>(As, Cq[(st + 1) & 3], ua, ual, ub, ubl, na, nb, nal,
                                                                 nbl, c0, c1, c2);
                    ua = na, ub = nb, ual = nal, ubl = nbl;
                } else {
                    x3_last<PREC>(ua, ual, ub, ubl, c0, c1, c2);
                }
            };
            static_for<0, NS>(pipe);
#pragma unroll
            for (int j = 0; j < (NQ < 4 ? NQ : 4); ++j) {
                const f4v v = __builtin_bit_cast(f4v, q[j]);
                kt[4 * j] = v[0], kt[4 * j + 1] = v[1], kt[4 * j + 2] = v[2], kt[4 * j + 3] = v[3];
            }
            if constexpr (NQ > 4) {
                U4 q4, qd;
                lds_read2<64, 64>(kb, kb, q4, qd);
                const f4v v = __builtin_bit_cast(f4v, q4);
                kt[16] = v[0], kt[17] = v[1], kt[18] = v[2], kt[19] = v[3];
            }
            const f4v sv = __builtin_bit_cast(f4v, qs);
            wv = c0 + (c1 + c2);
            wv[0] *= sv[0], wv[1] *= sv[1], wv[2] *= sv[2], wv[3] *= sv[3];
        } else {
            // weights of this b's cosmology and the row scales, from LDS
            float4 sc;
            {
                const uint32_t sa =
                    lds_addr(Cb + S::C_BUF + (size_t)KCH * 1024) + (uint32_t)(16 * min(ti, TR - 1) + 4 * lk) * 4;
                U4 q[6];
                if constexpr (KROT) {
                    const int rr = ((16 * tk + lr) >> 2) & 3;
                    lds_read4<0, 0, 0, 0>(kb + 16 * (rr & 3), kb + 16 * ((1 + rr) & 3), kb + 16 * ((2 + rr) & 3),
                                          kb + 16 * ((3 + rr) & 3), q[0], q[1], q[2], q[3]);
                } else {
                    lds_read4<0, (NQ > 1 ? 16 : 0), (NQ > 2 ? 32 : 0), (NQ > 3 ? 48 : 0)>(kb, kb, kb, kb, q[0], q[1],
                                                                                          q[2], q[3]);
                }
                lds_read2<(NQ > 4 ? 64 : 0), 0>(kb, sa, q[4], q[5]);
#pragma unroll
                for (int j = 0; j < NQ; ++j) {
                    const f4v v = __builtin_bit_cast(f4v, q[j]);
                    kt[4 * j] = v[0], kt[4 * j + 1] = v[1], kt[4 * j + 2] = v[2], kt[4 * j + 3] = v[3];
                }
                const f4v v = __builtin_bit_cast(f4v, q[5]);
                sc = make_float4(v[0], v[1], v[2], v[3]);
            }
            const uint32_t Asl = As + TR * NS * 64 * 16;
            uint32_t Cql[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) Cql[k] = Cq[k] + S::C_BUF / NPART;
            // four accumulators, so that consecutive MFMAs never wait for each other
            f4 acc[4] = {f4{0, 0, 0, 0}, f4{0, 0, 0, 0}, f4{0, 0, 0, 0}, f4{0, 0, 0, 0}};
            auto step_k = [&](auto stc) {
                constexpr int st = decltype(stc)::value;
                constexpr int coff = 256 * (st >> 2);
                const uint32_t cb = Cq[st & 3], cbl = Cql[st & 3];
                U4 ua, ub, ual, ubl;
                if constexpr (X3)
                    lds_read4<st * 1024, coff, st * 1024, coff>(As, cb, Asl, cbl, ua, ub, ual, ubl);
                else
                    lds_read2<st * 1024, coff>(As, cb, ua, ub);
                f4 &a0 = acc[st & 1];
                a0 = mfma16<PREC>(ua, ub, a0);
                if constexpr (X3) {
                    f4 &a1 = acc[2 + (st & 1)];
                    a1 = mfma16<PREC>(ua, ubl, a1);
                    a1 = mfma16<PREC>(ual, ub, a1);
                }
            };
            static_for<0, NS>(step_k);
            wv = (acc[0] + acc[1]) + (acc[2] + acc[3]);
            wv[0] *= sc.x, wv[1] *= sc.y, wv[2] *= sc.z, wv[3] *= sc.w;
        }
        // w tile of this b: lane holds rows 16 (rt0 + ti) + 4 lk + r for cosmology beta
#pragma unroll
        for (int g = 0; g < NB / 4; ++g)
            if ((gmask >> g) & 1)  // uniform over the wave
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int j = 4 * g; j < 4 * g + 4; ++j) y[r][j] += wv[r] * kt[j];
    };

    // issue order: A(0), c(0) + weights(0), A(1); then per b, after its barrier: c(b+1) +
    // weights(b+1), A(b+2).  Only DMAs are in flight, so the manual counts are exact.
    dma_A(0, A0);
    dma_C(0, C0);
    dma_X(0, C0);
    dma_A(1, A1);
    for (int b = 0; b < n_R; b += 6) {
        step(b, A0, C0, C1, A2);
        if (b + 1 < n_R) step(b + 1, A1, C1, C0, A0);
        if (b + 2 < n_R) step(b + 2, A2, C0, C1, A1);
        if (b + 3 < n_R) step(b + 3, A0, C1, C0, A2);
        if (b + 4 < n_R) step(b + 4, A1, C0, C1, A0);
        if (b + 5 < n_R) step(b + 5, A2, C1, C0, A1);
    }
    wait_vmcnt<0>();  // no DMA may outlive the work-group's LDS
    if (ti >= ntile || beta >= batch) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float *yp = Y + (((size_t)beta * rows_pad + 16 * (rt0 + ti) + 4 * lk + r) * n_chi + a) * NBP;
#pragma unroll
        for (int q = 0; q < NBP / 4; ++q) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (4 * q < NB) v = make_float4(y[r][4 * q], y[r][4 * q + 1], y[r][4 * q + 2], y[r][4 * q + 3]);
            ((float4 *)yp)[q] = v;
        }
    }
}

// FP16X3 fused kernel with wider wave tiles (NB <= 16).  The 12-wave kernel above is bound by the
// bytes it moves from L2 into LDS per (row, cosmology) pair; here a work-group is (chi_a, 64
// cosmologies, 4 row tiles) with 8 waves, and wave (i, k) makes two 16 x 16 tiles per b (row tile i,
// cosmologies 32k..32k+15 and 32k+16..32k+31), keeping Y for 4 rows x NB bins of both (two waves per
// SIMD).  Per b it moves 32 KB of basis and 32 KB of c rows for 4096 pairs, against 24 + 32 KB for
// 3072.  Basis and c one b ahead (two LDS buffers each, 138 KB); one barrier per b.  The time is
// that of the data movement (a copy without the MFMAs and R-sum takes as long), so the coefficients
// are point-major: the 64 rows of one point are one 16 KB block per part, where cosmology-major rows
// were 64 separate 256-byte pieces, 6 MB apart, and took 3.95 ms against 3.45 at full 3x2pt.
// Steps are not software-pipelined (the registers hold both tiles' accumulators and Y).
//
// Nodal variant (NOD): the basis operand is the nodal basis B = Ttilde D (the projection of
// Eq. dft applied to the basis when the plan is made), contracted with the FP32 nodal values P
// themselves, so no coefficients are made or stored per call.  Each wave loads 8 of the 64 P rows
// of a node (ncp floats each; past a row's n_cheb values, n_cheb % 4 == 0, its last 16-byte
// granule again, where the basis columns are zero) into registers one node ahead and splits them
// into the node's c buffer: per row a power-of-two scale puts the largest |P| in [2^14, 2^15),
// hi = fp16(v) and lo = fp16(v - hi), laid out as the coefficient rows (hi then lo part of each
// row, granules permuted by row), the row's inverse scale beside the weights.  After the barrier
// of node b a wave issues the DMAs of node b + 1, splits its rows of node b + 1 (loaded during node
// b - 1, so nothing waits), loads its rows of node b + 2 into the freed registers, then runs node
// b's MFMAs and R-sum: the split runs under the DMAs and one barrier per b still orders
// everything.  The inverse scale multiplies w with the basis row scale (both powers of two).
constexpr int kWideTR = 4;

template <int PREC, int NS, bool NOD = false>
struct WideShape {
    using E = uint16_t;
    static constexpr int VEC = 8, KSTEP = 32, ncp = NS * KSTEP, NPART = 2;
    static constexpr int ROWB = ncp * 2;                 // bytes of one row's part (hi or lo)
    static constexpr int CROW = NOD ? 2 * ROWB : ROWB;   // LDS stride of the c rows
    static constexpr int A_CH = kWideTR * NS * NPART, C_CH = 64 * ROWB * NPART / 1024;
    static constexpr int NW = 8;
    static constexpr int A_PW = (A_CH + NW - 1) / NW, C_PW = (C_CH + NW - 1) / NW;
    static constexpr size_t A_BUF = (size_t)A_CH * 1024, C_BUF = (size_t)C_CH * 1024;
    // weights (NB <= 16: <= 4 KB) and the basis row scales; nodal: the 64 P row scales after them
    static constexpr size_t X_BUF = (NOD ? 6 : 5) * 1024;
    static constexpr size_t LDS = 2 * A_BUF + 2 * (C_BUF + X_BUF);
};

// two 4-byte LDS reads at base + offsets, waited for
template <int O0, int O1>
__device__ inline void lds_read_f2(uint32_t b0, float &r0, float &r1) {
    asm volatile("ds_read_b32 %0, %2 offset:%3\n\tds_read_b32 %1, %2 offset:%4\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(r0), "=&v"(r1)
                 : "v"(b0), "i"(O0), "i"(O1)
                 : "memory");
}
__device__ inline void lds_write8(uint32_t a, uint64_t v) {
    asm volatile("ds_write_b64 %0, %1" : : "v"(a), "v"(v) : "memory");
}
__device__ inline void lds_write4(uint32_t a, float v) {
    asm volatile("ds_write_b32 %0, %1" : : "v"(a), "v"(v) : "memory");
}
// maximum over the 8 lanes of an aligned group (DPP: swap neighbours, swap pairs, mirror halves)
__device__ inline float max8(float m) {
    m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, m), 0xB1, 0xF, 0xF, false)));
    m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, m), 0x4E, 0xF, 0xF, false)));
    m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, m), 0x141, 0xF, 0xF, false)));
    return m;
}
typedef _Float16 h4v __attribute__((ext_vector_type(4)));

template <int PREC, int NB, int NBP, int NS, bool NOD>
__global__ __launch_bounds__(512) void contract_quad_wide_kernel(
    const uint16_t *__restrict__ basis, const uint16_t *__restrict__ basis_lo, const float *__restrict__ scale,
    const void *__restrict__ cv, const uint16_t *__restrict__ c_lo, const float *__restrict__ Kt, int batch,
    int n_chi, int n_R, int rows_pad, int nBT, int units, int n_ell, int nslots, int granges, int n_cheb,
    float *__restrict__ Y) {
    using S = WideShape<PREC, NS, NOD>;
    using E = typename S::E;
    constexpr int TR = kWideTR, VEC = S::VEC, ncp = S::ncp, NPART = S::NPART;
    constexpr int GPR = S::ROWB / 16;
    constexpr int SWZ = GPR % 16 == 0 ? 15 : (GPR % 8 == 0 ? 7 : (GPR % 4 == 0 ? 3 : (GPR % 2 == 0 ? 1 : 0)));
    constexpr bool KROT = NB == 16;
    static_assert(PREC == BLAST_FP16X3 && NB <= 16 && S::LDS <= 160 * 1024, "LDS of the wide fused kernel");
    static_assert(!NOD || S::C_PW * 1024 == 8 * S::CROW, "nodal: the 8 P rows of each wave fill the c buffer");
    __shared__ __align__(1024) unsigned char A0[S::A_BUF], A1[S::A_BUF];
    __shared__ __align__(1024) unsigned char C0[S::C_BUF + S::X_BUF], C1[S::C_BUF + S::X_BUF];

    const int groups = (rows_pad / 16 + TR - 1) / TR;
    const int per = (units + 7) / 8;
    const int unit = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (unit >= units) return;  // uniform over the work-group
    const int RT = rows_pad / 16;
    // the cosmology tiles of a row group next to each other (they read the same basis tiles): the
    // same time as row groups next to each other, 17.0 GB of HBM reads per launch against 20.6
    const int bt = unit % nBT, g = (unit / nBT) % groups, a = unit / (groups * nBT);
    const int rt0 = g * TR;
    const int ntile = min(TR, RT - rt0);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int ti = w >> 1, tk = w & 1;  // row tile, 32-cosmology half
    const int nb = min(64, batch - bt * 64);
    const size_t pt_u4 = (size_t)RT * NS * 64;
    const bool busy = ti < ntile && bt * 64 + 32 * tk < batch;
    int gq0 = NB / 4, gq1 = 0;
    {
        const int r0 = 16 * (rt0 + min(ti, TR - 1));
        const int s0 = min(r0 / n_ell, nslots - 1), s1 = min((r0 + 15) / n_ell, nslots - 1);
        for (int sl = s0; sl <= s1; ++sl) {
            gq0 = min(gq0, (granges >> (6 * sl)) & 7);
            gq1 = max(gq1, (granges >> (6 * sl + 3)) & 7);
        }
    }
    const int gmask = __builtin_amdgcn_readfirstlane(gq1 > gq0 ? ((1 << gq1) - 1) & ~((1 << gq0) - 1) : 0);

    // a wave issues up to A_PW basis and C_PW c DMAs per b (chunk indices past the end clamped: the
    // last chunk is written more than once with identical data); basis chunks of row tiles past the
    // end of the last group are skipped (each b waits for all DMAs, so the counts may differ)
    const U4 *srcA[S::A_PW];
    bool useA[S::A_PW];
    int nA = 0;  // basis DMAs this wave issues per b
#pragma unroll
    for (int k = 0; k < S::A_PW; ++k) {
        const int ch = min(w + k * S::NW, S::A_CH - 1);
        const int part = ch / (TR * NS), tl = (ch / NS) % TR, st = ch % NS;
        const int rt = min(rt0 + tl, RT - 1);
        srcA[k] = (const U4 *)(part ? basis_lo : basis) + ((size_t)rt * NS + st) * 64 + lane;
        useA[k] = tl < ntile;  // uniform over the wave
        nA += useA[k] ? 1 : 0;
    }
    auto dma_A = [&](int b, unsigned char *__restrict__ buf) {
        const size_t ab = (size_t)a * n_R + (b < n_R ? b : n_R - 1);
#pragma unroll
        for (int k = 0; k < S::A_PW; ++k)
            if (useA[k]) lds_dma16(srcA[k] + ab * pt_u4, buf + (size_t)min(w + k * S::NW, S::A_CH - 1) * 1024);
    };
    // weights Kt[ab][64 cosmologies][NB] and the row scales of the group: waves 0..KCH-1 move weight
    // chunks, wave KCH the scales, the others nothing
    constexpr int KCH = 64 * NB * 4 / 1024;
    static_assert(KCH + 1 <= S::NW && TR * 16 * 4 <= 1024 && KCH * 1024 + 1024 + (NOD ? 256 : 0) <= (int)S::X_BUF,
                  "extra region");
    constexpr int PSC = (int)S::C_BUF + (KCH + 1) * 1024;  // nodal: inverse P row scales [64]
    const int chX = min(w, KCH);
    const float *srcX;
    {
        int f = chX * 256 + lane * 4;
        if (KROT) {
            const int r = f / 16, sp = (f / 4) & 3;
            f = r * 16 + ((sp - (r >> 2)) & 3) * 4;
        }
        const int bl = f / NB;
        srcX = chX < KCH ? Kt + (size_t)(bt * 64 + (bl < nb ? bl : 0)) * NB + (bl < nb ? f % NB : 0)
                         : scale + min(16 * rt0 + 4 * lane, rows_pad - 4);
    }
    const size_t strideX = chX < KCH ? (size_t)batch * NB : (size_t)rows_pad;
    auto dma_X = [&](int b, unsigned char *__restrict__ buf) {
        if (w > KCH) return;
        const size_t ab = (size_t)a * n_R + (b < n_R ? b : n_R - 1);
        lds_dma16(srcX + ab * strideX, buf + S::C_BUF + (size_t)chX * 1024);
    };
    // coefficient path: the c rows of the tile by DMA (the nodal path loads P rows into registers)
    const char *srcC[S::C_PW] = {};
    size_t cstride = 0;
    if constexpr (!NOD) {
        const uint16_t *c = (const uint16_t *)cv;
#pragma unroll
        for (int k = 0; k < S::C_PW; ++k) {
            const int ch = min(w + k * S::NW, S::C_CH - 1);
            const int part = ch / (S::C_CH / NPART), chp = ch % (S::C_CH / NPART);
            const int pos = chp * 1024 + lane * 16;
            const int row = pos / S::ROWB, gp = (pos % S::ROWB) / 16;
            const int v = gp ^ (row & SWZ);
            const int bb = bt * 64 + (row < nb ? row : 0);
            srcC[k] = (const char *)((part ? c_lo : c) + (size_t)bb * ncp + v * VEC);
        }
        // point-major coefficients: the 64 rows of one point are one block of 64 ncp elements per part
        cstride = (size_t)batch * ncp * sizeof(E);
    }
    auto dma_C = [&](int b, unsigned char *__restrict__ buf) {
        const size_t ab = (size_t)a * n_R + (b < n_R ? b : n_R - 1);
#pragma unroll
        for (int k = 0; k < S::C_PW; ++k)
            lds_dma16(srcC[k] + ab * cstride, buf + (size_t)min(w + k * S::NW, S::C_CH - 1) * 1024);
    };
    // nodal: lane (row r = 8w + lane / 8 of the tile, sub = lane % 8) holds the 16-byte granules
    // sub + 8 (q ^ o) of its P row, o = r mod NS for NS = 2 and 4 (so that the four rows of a 32-lane
    // write phase write four different 64-byte quarters of a part); granules past n_cheb / 4 repeat
    // the last one
    const float *prow = (const float *)cv;
    int goff[NS];
    if constexpr (NOD) {
        const int r = 8 * w + (lane >> 3), sub = lane & 7;
        const int o = NS == 4 ? (r & 3) : (NS == 2 ? (r & 1) : 0);
        prow += (size_t)(bt * 64 + (r < nb ? r : 0)) * n_chi * n_R * n_cheb;
#pragma unroll
        for (int q = 0; q < NS; ++q) goff[q] = 4 * min(sub + 8 * (q ^ o), n_cheb / 4 - 1);
    }
    auto load_P = [&](int b, U4 (&raw)[NS]) {
        const float *pr = prow + ((size_t)a * n_R + (b < n_R ? b : n_R - 1)) * n_cheb;
#pragma unroll
        for (int q = 0; q < NS; ++q) raw[q] = *(const U4 *)(pr + goff[q]);
    };
    // split a node's P rows held in registers into buf: the row max over the 8 lanes of a row, the
    // power-of-two scale, FP16 hi and lo; then after() (which reloads raw), then the LDS writes
    auto split_rows = [&](const U4 (&raw)[NS], unsigned char *__restrict__ buf, auto &&after) {
        if constexpr (NOD) {
            const int r = 8 * w + (lane >> 3), sub = lane & 7;
            const int o = NS == 4 ? (r & 3) : (NS == 2 ? (r & 1) : 0);
            const uint32_t rb = lds_addr(buf) + (uint32_t)(r * S::CROW);
            float m = 0.f;
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const f4v v = __builtin_bit_cast(f4v, raw[q]);
#pragma unroll
                for (int e = 0; e < 4; ++e) m = fmaxf(m, fabsf(v[e]));
            }
            m = max8(m);
            const int ex = __builtin_amdgcn_frexp_expf(m) - 1;  // floor(log2 m); -1 for m = 0
            const float sc = __builtin_amdgcn_ldexpf(1.f, 14 - ex);
            h4v hh[NS], ll[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const f4v x = __builtin_bit_cast(f4v, raw[q]) * sc;
                hh[q] = __builtin_convertvector(x, h4v);
                ll[q] = __builtin_convertvector(x - __builtin_convertvector(hh[q], f4v), h4v);
            }
            __builtin_amdgcn_sched_barrier(0);
            after();  // raw is free from here on
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int gr = sub + 8 * (q ^ o), G = gr >> 1;
                const uint32_t oo = rb + (uint32_t)(((G ^ (r & SWZ)) << 4) | ((gr & 1) << 3));
                lds_write8(oo, __builtin_bit_cast(uint64_t, hh[q]));
                lds_write8(oo + S::ROWB, __builtin_bit_cast(uint64_t, ll[q]));
            }
            if (sub == 0) lds_write4(lds_addr(buf) + PSC + 4 * r, __builtin_amdgcn_ldexpf(1.f, ex - 14));
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        }
    };

    float y[2][4][NB];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < NB; ++q) y[j][r][q] = 0.f;
    const int arow = min(ti, TR - 1) * NS * 64 + lane;

    U4 R[NS];
    auto step = [&](int b, const unsigned char *__restrict__ Ab, const unsigned char *__restrict__ Cb,
                    unsigned char *__restrict__ Cnext, unsigned char *__restrict__ Anext) {
        // everything issued one b ago has landed (this wave's DMAs and P loads), then all waves'
        // (barrier)
        wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (!NOD) dma_C(b + 1, Cnext);
        dma_X(b + 1, Cnext);
        dma_A(b + 1, Anext);
        __builtin_amdgcn_sched_barrier(0);
        // nodal: the P rows of b + 1 (loaded during b - 1) split into their buffer under the DMAs
        // just issued, and the rows of b + 2 loaded into the same registers once converted
        if constexpr (NOD) split_rows(R, Cnext, [&] { load_P(b + 2, R); });
        if (busy) {
            constexpr int NQ = NB / 4;
            constexpr int ALO = TR * NS * 1024, CLO = NOD ? S::ROWB : (int)(S::C_BUF / NPART);
            // the second half's rows are 16 rows further on with the same granule permutation and
            // the same weight rotation (16 is a multiple of SWZ + 1 and of 16): fixed offsets
            constexpr int C16 = 16 * S::CROW, K16 = 16 * NB * 4;
            const uint32_t As = lds_addr(Ab) + (uint32_t)arow * 16;
            const int crow = 32 * tk + lr;
            uint32_t Cq[4], kq[4];
            {
                const uint32_t Cr = lds_addr(Cb) + (uint32_t)crow * S::CROW;
                const int m = crow & SWZ, mh = m >> 2, ml = lk ^ (m & 3);
#pragma unroll
                for (int k = 0; k < 4; ++k) Cq[k] = Cr + 16 * (4 * (k ^ mh) + ml);
                const uint32_t kb = lds_addr(Cb + S::C_BUF) + (uint32_t)crow * (NB * 4);
                const int rr = (crow >> 2) & 3;
#pragma unroll
                for (int q = 0; q < 4; ++q) kq[q] = KROT ? kb + 16 * ((q + rr) & 3) : kb + 16 * (q < NQ ? q : NQ - 1);
            }
            const uint32_t sa =
                lds_addr(Cb + S::C_BUF + (size_t)KCH * 1024) + (uint32_t)(16 * min(ti, TR - 1) + 4 * lk) * 4;
            f4 acc[2][3];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int u = 0; u < 3; ++u) acc[j][u] = f4{0, 0, 0, 0};
            auto step_k = [&](auto stc) {
                constexpr int st = decltype(stc)::value;
                constexpr int coff = 256 * (st >> 2);
                U4 ua, ual, ub0, ub0l, ub1, ub1l;
                const uint32_t cq = Cq[st & 3];
                lds_read6<st * 1024, st * 1024 + ALO, coff, coff + CLO, coff + C16, coff + C16 + CLO>(
                    As, cq, ua, ual, ub0, ub0l, ub1, ub1l);
                acc[0][0] = mfma16<PREC>(ua, ub0, acc[0][0]);
                acc[1][0] = mfma16<PREC>(ua, ub1, acc[1][0]);
                acc[0][1] = mfma16<PREC>(ua, ub0l, acc[0][1]);
                acc[1][1] = mfma16<PREC>(ua, ub1l, acc[1][1]);
                acc[0][2] = mfma16<PREC>(ual, ub0, acc[0][2]);
                acc[1][2] = mfma16<PREC>(ual, ub1, acc[1][2]);
            };
            static_for<0, NS>(step_k);
            float4 sc;
            {
                U4 qs, qd;
                lds_read2<0, 0>(sa, sa, qs, qd);
                const f4v v = __builtin_bit_cast(f4v, qs);
                sc = make_float4(v[0], v[1], v[2], v[3]);
            }
            float ps[2] = {1.f, 1.f};  // nodal: inverse P row scales of the lane's two cosmologies
            if constexpr (NOD) lds_read_f2<0, 64>(lds_addr(Cb) + PSC + 4 * crow, ps[0], ps[1]);
            // R-sum, one half at a time (its weights read just before)
            auto rsum = [&](auto jc) {
                constexpr int j = decltype(jc)::value;
                U4 q[4];
                lds_read4<j * K16, j * K16, j * K16, j * K16>(kq[0], kq[1], kq[2], kq[3], q[0], q[1], q[2], q[3]);
                float kt[NB];
#pragma unroll
                for (int g4 = 0; g4 < NQ; ++g4) {
                    const f4v v = __builtin_bit_cast(f4v, q[g4]);
#pragma unroll
                    for (int e = 0; e < 4; ++e) kt[4 * g4 + e] = v[e];
                }
                f4 wv = acc[j][0] + (acc[j][1] + acc[j][2]);
                if constexpr (NOD) {
                    wv[0] *= sc.x * ps[j], wv[1] *= sc.y * ps[j], wv[2] *= sc.z * ps[j], wv[3] *= sc.w * ps[j];
                } else {
                    wv[0] *= sc.x, wv[1] *= sc.y, wv[2] *= sc.z, wv[3] *= sc.w;
                }
#pragma unroll
                for (int gq = 0; gq < NB / 4; ++gq)
                    if ((gmask >> gq) & 1)  // uniform over the wave
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int qq = 4 * gq; qq < 4 * gq + 4; ++qq) y[j][r][qq] += wv[r] * kt[qq];
            };
            static_for<0, 2>(rsum);
        }
    };

    // issue order: c(0) + weights(0), A(0); then per b, after its barrier: c(b+1) + weights(b+1), A(b+1)
    if constexpr (NOD) {
        load_P(0, R);
    } else {
        dma_C(0, C0);
    }
    dma_X(0, C0);
    dma_A(0, A0);
    if constexpr (NOD) {
        wait_vmcnt<0>();
        split_rows(R, C0, [&] { load_P(1, R); });
    }
    for (int b = 0; b < n_R; b += 2) {
        step(b, A0, C0, C1, A1);
        if (b + 1 < n_R) step(b + 1, A1, C1, C0, A0);
    }
    wait_vmcnt<0>();  // no DMA may outlive the work-group's LDS
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int beta = bt * 64 + 32 * tk + 16 * j + lr;
        if (ti >= ntile || beta >= batch) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float *yp = Y + (((size_t)beta * rows_pad + 16 * (rt0 + ti) + 4 * lk + r) * n_chi + a) * NBP;
#pragma unroll
            for (int q = 0; q < NBP / 4; ++q) {
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (4 * q < NB) v = make_float4(y[j][r][4 * q], y[j][r][4 * q + 1], y[j][r][4 * q + 2], y[j][r][4 * q + 3]);
                ((float4 *)yp)[q] = v;
            }
        }
    }
}

// FP64 fused contraction and R-quadrature (no w_save, at most 16 bins): the FP64 path's w, like
// the mixed paths', never leaves the registers of the wave that makes it.
//   w[row][beta]          = sum_n Ttilde[a, b][row][n] c[beta][a, b][n]     (v_mfma_f64_16x16x4_f64)
//   Y[beta][row][a][bin] += w[row][beta] * Kt[a, b][beta][bin]            (FP64 FMA, per b)
// Work-group = (chi_a, 64 cosmologies, 2 row tiles), 8 waves: wave (i, j) makes the 16 x 16 tile
// (row tile i, cosmologies 16j..16j+15) and keeps Y for its 4 rows x NB bins in FP64.  Each b is
// taken in NSTG stages of KS Chebyshev columns; a stage's 32 basis row slices and 64 c row slices
// go from global memory straight to LDS (two buffers, one stage ahead, one barrier per stage), the
// weights of b (16 bins, zero padded) with b's first stage.  Rows sit in LDS with their 16-byte
// granules permuted (granule g of row r at g ^ (r & 15)) so that the 16 rows one instruction reads
// fall in distinct banks.  A lane reads two consecutive columns at once and feeds them to two
// MFMAs (two accumulator chains): lane group lk takes columns 8p + 2lk and 8p + 2lk + 1 of each
// group p of 8, so the two MFMAs of p together cover its 8 columns once.
constexpr int kF64TR = 2;

template <int KS>
struct F64Shape {
    static constexpr int ROWB = KS * 8;   // bytes of one row's slice in a stage
    static constexpr int GR = ROWB / 16;  // 16-byte granules per slice
    static constexpr int RPC = 1024 / ROWB;  // slices per 1 KB chunk
    static constexpr int NW = 8;
    static constexpr int A_CH = kF64TR * 16 / RPC, C_CH = 64 / RPC;
    static constexpr int A_PW = A_CH / NW, C_PW = C_CH / NW;
    static constexpr size_t A_BUF = (size_t)A_CH * 1024, C_BUF = (size_t)C_CH * 1024, K_BUF = 8 * 1024;
    static_assert(A_PW * NW == A_CH && C_PW * NW == C_CH, "whole chunks per wave");
};

// eight 16-byte reads (four at bases a[k], four at c[k], one compile-time offset), then a wait
template <int O>
__device__ inline void lds_read8(const uint32_t (&a)[4], const uint32_t (&c)[4], U4 (&ra)[4], U4 (&rc)[4]) {
    asm volatile(
        "ds_read_b128 %0, %8 offset:%16\n\tds_read_b128 %1, %9 offset:%16\n\t"
        "ds_read_b128 %2, %10 offset:%16\n\tds_read_b128 %3, %11 offset:%16\n\t"
        "ds_read_b128 %4, %12 offset:%16\n\tds_read_b128 %5, %13 offset:%16\n\t"
        "ds_read_b128 %6, %14 offset:%16\n\tds_read_b128 %7, %15 offset:%16\n\ts_waitcnt lgkmcnt(0)"
        : "=&v"(ra[0]), "=&v"(ra[1]), "=&v"(ra[2]), "=&v"(ra[3]), "=&v"(rc[0]), "=&v"(rc[1]), "=&v"(rc[2]),
          "=&v"(rc[3])
        : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "i"(O)
        : "memory");
}

template <int NB, int KS, int NSTG>
__global__ __launch_bounds__(512) void contract_quad_f64_kernel(const double *__restrict__ basis,
                                                                const double *__restrict__ c,
                                                                const double *__restrict__ Kt, int batch, int n_chi,
                                                                int n_R, int rows_pad, int nBT, int units,
                                                                double *__restrict__ Y) {
    using S = F64Shape<KS>;
    constexpr int ncp = KS * NSTG, NBK = 16, TR = kF64TR;
    static_assert(NB % 4 == 0 && NB <= NBK && KS % 32 == 0, "shape of the FP64 fused kernel");
    // two stage buffers of basis and c slices, two of weights; after the last stage the first
    // 64 KB hold the Y tiles on their way out (8 KB per wave)
    __shared__ __align__(1024) unsigned char lds[2 * (S::A_BUF + S::C_BUF + S::K_BUF)];
    static_assert(2 * (S::A_BUF + S::C_BUF + S::K_BUF) >= 64 * 1024, "room for the Y tiles");
    unsigned char *const A0 = lds, *const A1 = lds + S::A_BUF;
    unsigned char *const C0 = lds + 2 * S::A_BUF, *const C1 = C0 + S::C_BUF;
    unsigned char *const K0 = C1 + S::C_BUF, *const K1 = K0 + S::K_BUF;

    const int RT = rows_pad / 16;
    const int groups = (RT + TR - 1) / TR;
    const int per = (units + 7) / 8;
    const int unit = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (unit >= units) return;  // uniform over the work-group
    // the cosmology tiles of a row group next to each other (they read the same basis tiles): the
    // same time as row groups next to each other, with fewer HBM reads
    const int bt = unit % nBT, g = (unit / nBT) % groups, a = unit / (groups * nBT);
    const int rt0 = g * TR;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int ti = w >> 2, tj = w & 3;  // row tile, 16-cosmology tile
    const int nb = min(64, batch - bt * 64);
    const size_t NP = (size_t)n_chi * n_R;
    const bool busy = rt0 + ti < RT && 16 * tj < nb;

    // DMA sources at b = 0, stage 0 (element offsets); rows past the end read the last valid row
    size_t srcA[S::A_PW], srcC[S::C_PW];
#pragma unroll
    for (int k = 0; k < S::A_PW; ++k) {
        const int row = (w + k * S::NW) * S::RPC + lane / S::GR, gr = (lane % S::GR) ^ (row & 15);
        const int rt = min(rt0 + row / 16, RT - 1);
        srcA[k] = ((size_t)a * n_R * rows_pad + 16 * rt + row % 16) * ncp + 2 * gr;
    }
#pragma unroll
    for (int k = 0; k < S::C_PW; ++k) {
        const int row = (w + k * S::NW) * S::RPC + lane / S::GR, gr = (lane % S::GR) ^ (row & 15);
        const size_t beta = (size_t)bt * 64 + min(row, nb - 1);
        srcC[k] = (beta * NP + (size_t)a * n_R) * ncp + 2 * gr;
    }
    // weights: chunk w holds cosmologies 8w..8w+7 (128 bytes each), granule gk of cosmology cr in
    // slot (gk + cr / 2) % 8, so that the 16 cosmologies of a read fall in distinct banks
    size_t srcK;
    {
        const int cr = w * 8 + lane / 8, gk = (lane % 8 - (cr >> 1)) & 7;
        srcK = ((size_t)a * n_R * batch + (size_t)bt * 64 + min(cr, nb - 1)) * NBK + 2 * gk;
    }
    auto dma = [&](int idx) {
        const int b = idx / NSTG, s = idx % NSTG;
        unsigned char *Ab = (idx & 1) ? A1 : A0, *Cb = (idx & 1) ? C1 : C0;
        const size_t offA = (size_t)b * rows_pad * ncp + (size_t)s * KS, offC = (size_t)b * ncp + (size_t)s * KS;
#pragma unroll
        for (int k = 0; k < S::A_PW; ++k) lds_dma16(basis + srcA[k] + offA, Ab + (size_t)(w + k * S::NW) * 1024);
#pragma unroll
        for (int k = 0; k < S::C_PW; ++k) lds_dma16(c + srcC[k] + offC, Cb + (size_t)(w + k * S::NW) * 1024);
        if (s == 0) lds_dma16(Kt + srcK + (size_t)b * batch * NBK, ((b & 1) ? K1 : K0) + (size_t)w * 1024);
    };

    // LDS read offsets of the lane: pair p of a group of 4 (32 columns) at granule 4p + lk
    uint32_t offA[4], offC[4], offK[NB / 2];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t gp = 16u * (4u * (uint32_t)(p ^ (lr >> 2)) + (uint32_t)((lk ^ lr) & 3));
        offA[p] = (uint32_t)(16 * ti + lr) * S::ROWB + gp;
        offC[p] = (uint32_t)(16 * tj + lr) * S::ROWB + gp;
    }
    {
        const int cr = 16 * tj + lr;
#pragma unroll
        for (int q = 0; q < NB / 2; ++q) offK[q] = (uint32_t)cr * (NBK * 8) + 16u * (uint32_t)((q + (cr >> 1)) & 7);
    }

    double y[4][NB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < NB; ++q) y[r][q] = 0.0;
    d4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};

    const int total = n_R * NSTG;
    dma(0);
    for (int idx = 0; idx < total; ++idx) {
        // this wave's DMAs of stage idx have landed, then every wave's (barrier)
        wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (idx + 1 < total) dma(idx + 1);
        __builtin_amdgcn_sched_barrier(0);
        if (!busy) continue;
        const uint32_t ab = lds_addr((idx & 1) ? A1 : A0), cb = lds_addr((idx & 1) ? C1 : C0);
        uint32_t ra[4], rc[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) ra[p] = ab + offA[p], rc[p] = cb + offC[p];
        auto group = [&](auto gc) {
            constexpr int G = decltype(gc)::value;
            U4 xa[4], xc[4];
            lds_read8<256 * G>(ra, rc, xa, xc);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const d2v av = __builtin_bit_cast(d2v, xa[p]), cv = __builtin_bit_cast(d2v, xc[p]);
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], cv[0], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], cv[1], acc1, 0, 0, 0);
            }
        };
        static_for<0, KS / 32>(group);
        if (idx % NSTG == NSTG - 1) {
            // R-sum of b: lane holds w of rows lk + 4r of its row tile for cosmology 16 tj + lr
            const uint32_t kb = lds_addr(((idx / NSTG) & 1) ? K1 : K0);
            double kt[NB];
#pragma unroll
            for (int q0 = 0; q0 < NB / 2; q0 += 2) {
                U4 k0, k1;
                lds_read2<0, 0>(kb + offK[q0], kb + offK[q0 + 1], k0, k1);
                const d2v v0 = __builtin_bit_cast(d2v, k0), v1 = __builtin_bit_cast(d2v, k1);
                kt[2 * q0] = v0[0], kt[2 * q0 + 1] = v0[1], kt[2 * q0 + 2] = v1[0], kt[2 * q0 + 3] = v1[1];
            }
            const d4 wv = acc0 + acc1;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q < NB; ++q) y[r][q] = fma(wv[r], kt[q], y[r][q]);
            acc0 = d4{0, 0, 0, 0};
            acc1 = d4{0, 0, 0, 0};
        }
    }
    wait_vmcnt<0>();  // no DMA may outlive the work-group's LDS
    // Y rows are 128 bytes ([beta][row][a][16 bins]) and a lane holds 4 of them: they go out
    // through LDS so that each store instruction writes 8 whole rows (16 bytes per lane) rather
    // than 16 bytes of 64 rows.  Every wave has finished its last stage's reads past this barrier.
    __syncthreads();
    if (!busy) return;
    double *tile = (double *)(lds + (size_t)w * 8192);  // [cosmology lr][row lk][16 bins]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int q = 0; q < NBK; q += 2) {
            double2 v = make_double2(0.0, 0.0);
            if (q < NB) v = make_double2(y[r][q], y[r][q + 1]);
            *(double2 *)(tile + (lr * 4 + lk) * NBK + q) = v;
        }
        // LDS accesses of a wave complete in order; the asm keeps the compiler from moving the
        // reads of other lanes' rows above these writes (and the next pass's writes above them)
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int line = 8 * i + lane / 8, ch = lane % 8;  // line = 4 * cosmology + row
            const int beta = bt * 64 + 16 * tj + line / 4, row = 16 * (rt0 + ti) + line % 4 + 4 * r;
            const double2 v = *(const double2 *)(tile + line * NBK + 2 * ch);
            if (beta < batch) *(double2 *)(Y + (((size_t)beta * rows_pad + row) * n_chi + a) * NBK + 2 * ch) = v;
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
}

// Kt[a, b][beta][bin] = wR_b K_bin(R_b chi_a) (T = float or double, NB bins with zero padding) for
// the fused kernels.  A work-group transposes 64 points x KB cosmologies through LDS: coalesced
// 512-byte reads along the points, contiguous writes per point.
// With cs (FP16 coefficients, T = float) the weights also carry the coefficient row scale
// cs[beta][a, b], which the contraction of the scaled coefficients leaves out.
constexpr int kKtP = 64;  // points per work-group of kt_kernel
template <typename T>
constexpr int kt_cosmologies() { return sizeof(T) == 8 ? 4 : 8; }  // cosmologies per work-group

template <typename T>
__global__ __launch_bounds__(256) void kt_kernel(const double *__restrict__ Kchi2, const double *__restrict__ wR,
                                                 const float *__restrict__ cs, int batch, int nbins, int NB, int NP,
                                                 int n_R, T *__restrict__ Kt) {
    constexpr int KP = kKtP, KB = kt_cosmologies<T>();
    __shared__ T tile[KP][KB * 20 + 1];  // [point][beta_local * NB + bin], NB <= 20
    __shared__ float csl[KB][KP];        // coefficient row scales [beta_local][point]
    const int ab0 = blockIdx.x * KP, b0 = blockIdx.y * KB;
    const int nbeta = min(KB, batch - b0);
    if (cs) {
        for (int i = threadIdx.x; i < KB * KP; i += blockDim.x) {
            const int bl = i / KP, p = i % KP;
            csl[bl][p] = (bl < nbeta && ab0 + p < NP) ? cs[(size_t)(b0 + bl) * NP + ab0 + p] : 0.f;
        }
        __syncthreads();
    }
    // a thread always handles point ab0 + threadIdx.x % KP (blockDim is a multiple of KP), so its R
    // weight is loaded once; sixteen K_chi2 loads in flight per thread (clamped addresses, values masked)
    static_assert(256 % KP == 0, "point of a thread");
    const int pt = threadIdx.x % KP, ab = min(ab0 + pt, NP - 1);
    const double wv = wR[ab % n_R];
    constexpr int U = 16;
    const int total = KB * NB * KP;
    for (int i0 = threadIdx.x; i0 < total; i0 += U * blockDim.x) {
        double kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(i0 + u * (int)blockDim.x, total - 1);
            const int q = i / KP;  // q = beta_local * NB + bin
            const int bl = min(q / NB, nbeta - 1), bin = min(q % NB, nbins - 1);
            kv[u] = Kchi2[((size_t)(b0 + bl) * nbins + bin) * NP + min(ab0 + i % KP, NP - 1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            const int q = i / KP;
            if (i < total)
                tile[pt][q] = (q / NB < nbeta && q % NB < nbins && ab0 + pt < NP) ? (T)(wv * kv[u]) : (T)0;
        }
    }
    __syncthreads();
    // each point's nbeta * NB weights are contiguous in Kt: four values per thread (NB % 4 == 0, so
    // the four share one cosmology and its power-of-two coefficient scale: exact in FP32)
    const int rq = nbeta * NB / 4;
    for (int i = threadIdx.x; i < KP * rq; i += blockDim.x) {
        const int p = i / rq, q = 4 * (i % rq);
        if (ab0 + p >= NP) continue;
        T *o = Kt + ((size_t)(ab0 + p) * batch + b0) * NB + q;
        if constexpr (sizeof(T) == 8) {
            *(double2 *)o = make_double2(tile[p][q], tile[p][q + 1]);
            *(double2 *)(o + 2) = make_double2(tile[p][q + 2], tile[p][q + 3]);
        } else {
            const float sc = cs ? csl[q / NB][p] : 1.f;
            *(float4 *)o =
                make_float4(tile[p][q] * sc, tile[p][q + 1] * sc, tile[p][q + 2] * sc, tile[p][q + 3] * sc);
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

// chi-quadrature and pair assembly.  For one cosmology and one basis row (type t, multipole l):
//   Z[i][j] = sum_a Ktil_i(chi_a) Y[row][a][j],  Ktil_i(chi_a) = wchi_a chi_a K_i(chi_a)
//   C[p = (i, j)][l] = N_t(l) (Z[i][j] + Z[j][i])                                  (Eq. final_cls)
// Z is a [bins x n_chi] x [n_chi x bins] product on FP64 MFMA (Ktil from LDS, Y straight from
// global, 16 consecutive bins per lane group).  Work-group = (type slot x 16 output multipoles,
// cosmology); wave w handles rows w, w+4, ...
constexpr int kChiRows = 16;

template <typename YT, int NBT>
__global__ __launch_bounds__(256) void quad_c_mfma_kernel(const YT *__restrict__ Y, const double *__restrict__ Kchi,
                                                          const double *__restrict__ wchi,
                                                          const double *__restrict__ chi,
                                                          const double *__restrict__ pref, int n_chi, int rows_pad,
                                                          int n_ell, Slots slot_type, int ng, int ns, uint32_t types,
                                                          int npairs, EllSel sel, double *__restrict__ C) {
    constexpr int NBP = 16 * NBT;
    extern __shared__ __align__(16) double smem_c[];
    const int nbins = ng + ns;
    const int nc4 = (n_chi + 3) & ~3;
    // [nc4][NBP]: the 16 lanes of a K-step read 16 consecutive bins of one chi node (a bin-major
    // table would put all 16 in one bank)
    double *Kt = smem_c;
    double *Zs = smem_c + (size_t)NBP * nc4;       // [4 waves][NBP][NBP]
    const int nblk = (sel.n_out + kChiRows - 1) / kChiRows;
    const int slot = blockIdx.x / nblk, io0 = (blockIdx.x % nblk) * kChiRows;
    const int beta = blockIdx.y;
    const int t = slot_type.s[slot];
    if (!(t & types)) return;
    {
        // four loads in flight per thread (clamped addresses, masked values)
        const int tot = NBP * nc4;
        for (int i0 = threadIdx.x; i0 < tot; i0 += 4 * blockDim.x) {
            double kv[4], wc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = min(i0 + u * (int)blockDim.x, tot - 1);
                const int bin = min(i % NBP, nbins - 1), a = min(i / NBP, n_chi - 1);
                kv[u] = Kchi[((size_t)beta * nbins + bin) * n_chi + a];
                wc[u] = wchi[a] * chi[a];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                if (i < tot) Kt[i] = (i % NBP < nbins && i / NBP < n_chi) ? wc[u] * kv[u] : 0.0;
            }
        }
    }
    __syncthreads();
    int off, ntp;
    if (t == BLAST_GG) {
        off = 0;
        ntp = ng * (ng + 1) / 2;
    } else if (t == BLAST_GS) {
        off = (types & BLAST_GG) ? ng * (ng + 1) / 2 : 0;
        ntp = ng * ns;
    } else {
        off = ((types & BLAST_GG) ? ng * (ng + 1) / 2 : 0) + ((types & BLAST_GS) ? ng * ns : 0);
        ntp = ns * (ns + 1) / 2;
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    double *Z = Zs + (size_t)wv * NBP * NBP;
    for (int io = io0 + wv; io < min(io0 + kChiRows, sel.n_out); io += 4) {
        const int row = slot * n_ell + sel.idx[io];
        const YT *yr = Y + ((size_t)beta * rows_pad + row) * n_chi * NBP;
        d4 acc[NBT][NBT];
#pragma unroll
        for (int i = 0; i < NBT; ++i)
#pragma unroll
            for (int j = 0; j < NBT; ++j) acc[i][j] = d4{0, 0, 0, 0};
        // full blocks of KB K-steps: the raw loads of the block go out first (clamped addresses; the
        // scheduling barrier keeps the compiler from pairing each load with its use), then the
        // conversions, masks and MFMAs
        constexpr int KB = 16;
        const int nsteps = nc4 / 4;
        auto kstep = [&](int st, const YT(&raw)[NBT]) {
            const int a = 4 * st + lk;
            double av[NBT], b[NBT];
#pragma unroll
            for (int i = 0; i < NBT; ++i) {
                av[i] = Kt[(size_t)a * NBP + 16 * i + lr];
                b[i] = a < n_chi ? (double)raw[i] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < NBT; ++i)
#pragma unroll
                for (int j = 0; j < NBT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], b[j], acc[i][j], 0, 0, 0);
        };
        auto loadB = [&](int st, YT(&raw)[NBT]) {
            const int ac = min(4 * st + lk, n_chi - 1);
#pragma unroll
            for (int i = 0; i < NBT; ++i) raw[i] = yr[(size_t)ac * NBP + 16 * i + lr];
        };
        int s0 = 0;
        for (; s0 + KB <= nsteps; s0 += KB) {
            YT bv[KB][NBT];
#pragma unroll
            for (int u = 0; u < KB; ++u) loadB(s0 + u, bv[u]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < KB; ++u) kstep(s0 + u, bv[u]);
        }
        for (; s0 < nsteps; ++s0) {
            YT bv[NBT];
            loadB(s0, bv);
            kstep(s0, bv);
        }
        // D layout of f64 16x16: Z[i = 16*ti + lk + 4r][j = 16*tj + lr]
#pragma unroll
        for (int i = 0; i < NBT; ++i)
#pragma unroll
            for (int j = 0; j < NBT; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) Z[(16 * i + lk + 4 * r) * NBP + 16 * j + lr] = acc[i][j][r];
        // Z is private to this wave: a fence orders its LDS writes before the reads of other lanes
        __threadfence_block();
        const double pf = pref[row];
        for (int q = lane; q < ntp; q += 64) {
            int i, j;
            if (t == BLAST_GS) {
                i = q / ns;
                j = ng + q % ns;
            } else {
                const int n = t == BLAST_GG ? ng : ns, base = t == BLAST_GG ? 0 : ng;
                int r = 0, pp = q;
                while (pp >= n - r) {
                    pp -= n - r;
                    ++r;
                }
                i = base + r;
                j = base + r + pp;
            }
            C[((size_t)beta * npairs + off + q) * sel.n_out + io] = pf * (Z[i * NBP + j] + Z[j * NBP + i]);
        }
        __threadfence_block();
    }
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// ---------------------------------------------------------------------------------------------
// coefficient input (P given as the c_n of Eq. cheb_pk instead of nodal values)
// ---------------------------------------------------------------------------------------------
template <typename PT, int OUT>
__global__ __launch_bounds__(256) void coef_in_kernel(const PT *__restrict__ cin, int N, int ncp, long nrows,
                                                      void *__restrict__ c_out, uint16_t *__restrict__ c_lo) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows * ncp) return;
    const long row = i / ncp;
    const int n = (int)(i % ncp);
    const double v = n < N ? (double)cin[row * N + n] : 0.0;
    if (OUT == 0) {
        ((double *)c_out)[i] = v;
    } else if (OUT == 1) {
        ((float *)c_out)[i] = (float)v;
    } else {
        const float f = (float)v;
        const uint16_t h = bf16_rne(f);
        ((uint16_t *)c_out)[i] = h;
        if (c_lo) c_lo[i] = bf16_rne(f - bf16_val(h));
    }
}

// FP16 hi and lo parts of coefficients given as input, one wave per row: the same power-of-two
// row scale as the projection's FP16 output (largest |c_n| in [2^14, 2^15), cs[row] = scale), and
// written point-major like it (row = beta * NP + point goes to point * batch + beta)
template <typename PT>
__global__ __launch_bounds__(256) void coef_in16_kernel(const PT *__restrict__ cin, int N, int ncp, long nrows,
                                                        uint16_t *__restrict__ c_hi, uint16_t *__restrict__ c_lo,
                                                        float *__restrict__ cs, long NP, int batch) {
    const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;  // uniform over the wave
    float v[kMaxCheb / 64];
    float mx = 0.f;
#pragma unroll
    for (int i = 0; i < kMaxCheb / 64; ++i) {
        const int n = lane + 64 * i;
        v[i] = n < N ? (float)cin[row * N + n] : 0.f;
        mx = fmaxf(mx, fabsf(v[i]));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    const int e = mx > 0.f ? min(max(ilogbf(mx), -100), 127) : 14;
    const float mul = ldexpf(1.f, 14 - e);
    if (lane == 0) cs[row] = ldexpf(1.f, e - 14);
    const size_t orow = (size_t)(row % NP) * batch + row / NP;
#pragma unroll
    for (int i = 0; i < kMaxCheb / 64; ++i) {
        const int n = lane + 64 * i;
        if (n >= ncp) break;
        const float x = v[i] * mul;
        const _Float16 h = (_Float16)x;
        c_hi[orow * ncp + n] = __builtin_bit_cast(uint16_t, h);
        c_lo[orow * ncp + n] = __builtin_bit_cast(uint16_t, (_Float16)(x - (float)h));
    }
}

// ---------------------------------------------------------------------------------------------
// adjoint kernels (FP64 or FP32 arithmetic T; small reductions in FP64)
// ---------------------------------------------------------------------------------------------
struct EllInv {
    int16_t io[kMaxEll];  // output position of each plan multipole, -1 if not requested
};

// dY[beta][row][a][m] = sum_l S[m][l] Ktil_l(chi_a), with S the symmetric matrix of pair
// cotangents of this row: S[i][j] = S[j][i] = N_t(l) dC[p=(i,j)] (2 N_t dC on the diagonal).
// S is also stored for the kernel gradient.  Rows that are not part of the output get zeros.
template <typename T, int NB>
__global__ __launch_bounds__(256) void adj_dy_kernel(const double *__restrict__ dC, const double *__restrict__ Kchi,
                                                     const double *__restrict__ wchi, const double *__restrict__ chi,
                                                     const double *__restrict__ pref, int n_chi, int rows_pad,
                                                     int n_ell, Slots slot_type, int ng, int ns, uint32_t types,
                                                     int npairs, int n_out, EllInv inv, T *__restrict__ dY,
                                                     double *__restrict__ Sg) {
    __shared__ double S[NB][NB];
    const int row = blockIdx.x, beta = blockIdx.y;
    const int slot = row / n_ell, il = row % n_ell;
    const int t = slot_type.s[slot];
    const int io = inv.io[il];
    const bool active = (t & types) && io >= 0;
    const int nbins = ng + ns;
    for (int i = threadIdx.x; i < NB * NB; i += blockDim.x) S[i / NB][i % NB] = 0.0;
    __syncthreads();
    if (active) {
        int off, ntp;
        if (t == BLAST_GG) {
            off = 0;
            ntp = ng * (ng + 1) / 2;
        } else if (t == BLAST_GS) {
            off = (types & BLAST_GG) ? ng * (ng + 1) / 2 : 0;
            ntp = ng * ns;
        } else {
            off = ((types & BLAST_GG) ? ng * (ng + 1) / 2 : 0) + ((types & BLAST_GS) ? ng * ns : 0);
            ntp = ns * (ns + 1) / 2;
        }
        const double pf = pref[row];
        for (int q = threadIdx.x; q < ntp; q += blockDim.x) {
            int i, j;
            if (t == BLAST_GS) {
                i = q / ns;
                j = ng + q % ns;
            } else {
                const int n = t == BLAST_GG ? ng : ns, base = t == BLAST_GG ? 0 : ng;
                int r = 0, pp = q;
                while (pp >= n - r) {
                    pp -= n - r;
                    ++r;
                }
                i = base + r;
                j = base + r + pp;
            }
            const double g = pf * dC[((size_t)beta * npairs + off + q) * n_out + io];
            if (i == j) {
                S[i][i] = 2.0 * g;
            } else {
                S[i][j] = g;
                S[j][i] = g;
            }
        }
    }
    __syncthreads();
    double *sg = Sg + ((size_t)beta * rows_pad + row) * NB * NB;
    for (int i = threadIdx.x; i < NB * NB; i += blockDim.x) sg[i] = S[i / NB][i % NB];
    T *dy = dY + ((size_t)beta * rows_pad + row) * n_chi * NB;
    const double *Kb = Kchi + (size_t)beta * nbins * n_chi;
    for (int i = threadIdx.x; i < n_chi * NB; i += blockDim.x) {
        const int a = i / NB, m = i % NB;
        double v = 0.0;
        if (active && m < nbins) {
            const double wa = wchi[a] * chi[a];
            for (int l = 0; l < nbins; ++l) v += S[m][l] * wa * Kb[(size_t)l * n_chi + a];
        }
        dy[i] = (T)v;
    }
}

// FP32 path of adj_dy_kernel: kAdjRG rows of one cosmology per work-group.  Each row's symmetric
// S (pair cotangents times N_t(l), as adj_dy_kernel builds it) goes to LDS in FP64 and to Sg; the
// weighted kernels Ktil[l][a] = wchi_a chi_a K_l(chi_a) of the cosmology sit in LDS transposed
// ([a][l], rows padded to 16 a and NB + 4 floats); then per row
//   dY[a][m] = sum_l S[m][l] Ktil[l][a]      (v_mfma_f32_16x16x4_f32: M = bins m, N = chi nodes a)
// with the K order permuted so that a lane reads 4 consecutive l of S and of Ktil; a lane's result
// is 4 consecutive m of one a, stored as 16 bytes (a wave writes 1 KB of dY contiguously).
constexpr int kAdjRG = 8;
template <int NB>
__global__ __launch_bounds__(256) void adj_dy_mfma_kernel(const double *__restrict__ dC, const double *__restrict__ Kchi,
                                                          const double *__restrict__ wchi, const double *__restrict__ chi,
                                                          const double *__restrict__ pref, int n_chi, int rows,
                                                          int rows_pad, int n_ell, Slots slot_type, int ng, int ns,
                                                          uint32_t types, int npairs, int n_out, EllInv inv,
                                                          float *__restrict__ dY, double *__restrict__ Sg) {
    constexpr int KS = NB + 4;
    extern __shared__ __align__(16) unsigned char smem_dy[];
    double *Sd = (double *)smem_dy;                          // [kAdjRG][NB][NB]
    float *KtT = (float *)(Sd + (size_t)kAdjRG * NB * NB);  // [n_chi rounded to 16][KS]
    const int beta = blockIdx.y, row0 = blockIdx.x * kAdjRG;
    const int nbins = ng + ns;
    const int nca = (n_chi + 15) / 16 * 16;
    for (int i = threadIdx.x; i < kAdjRG * NB * NB; i += blockDim.x) Sd[i] = 0.0;
    const double *Kb = Kchi + (size_t)beta * nbins * n_chi;
    for (int i = threadIdx.x; i < nca * NB; i += blockDim.x) {
        const int a = i / NB, l = i % NB;
        KtT[(size_t)a * KS + l] = (a < n_chi && l < nbins) ? (float)(wchi[a] * chi[a] * Kb[(size_t)l * n_chi + a]) : 0.f;
    }
    __syncthreads();
    for (int r = 0; r < kAdjRG; ++r) {
        const int row = row0 + r;
        if (row >= rows) break;
        const int slot = row / n_ell, il = row % n_ell;
        const int t = slot_type.s[slot];
        const int io = inv.io[il];
        if (!((t & types) && io >= 0)) continue;
        int off, ntp;
        if (t == BLAST_GG) {
            off = 0;
            ntp = ng * (ng + 1) / 2;
        } else if (t == BLAST_GS) {
            off = (types & BLAST_GG) ? ng * (ng + 1) / 2 : 0;
            ntp = ng * ns;
        } else {
            off = ((types & BLAST_GG) ? ng * (ng + 1) / 2 : 0) + ((types & BLAST_GS) ? ng * ns : 0);
            ntp = ns * (ns + 1) / 2;
        }
        const double pf = pref[row];
        double *S = Sd + (size_t)r * NB * NB;
        for (int q = threadIdx.x; q < ntp; q += blockDim.x) {
            int i, j;
            if (t == BLAST_GS) {
                i = q / ns;
                j = ng + q % ns;
            } else {
                const int n = t == BLAST_GG ? ng : ns, base = t == BLAST_GG ? 0 : ng;
                int rr = 0, pp = q;
                while (pp >= n - rr) {
                    pp -= n - rr;
                    ++rr;
                }
                i = base + rr;
                j = base + rr + pp;
            }
            const double g = pf * dC[((size_t)beta * npairs + off + q) * n_out + io];
            if (i == j) {
                S[i * NB + i] = 2.0 * g;
            } else {
                S[i * NB + j] = g;
                S[j * NB + i] = g;
            }
        }
    }
    __syncthreads();
    for (int r = 0; r < kAdjRG; ++r) {
        const int row = row0 + r;
        if (row >= rows) break;
        double *sg = Sg + ((size_t)beta * rows_pad + row) * NB * NB;
        for (int i = threadIdx.x; i < NB * NB; i += blockDim.x) sg[i] = Sd[(size_t)r * NB * NB + i];
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    constexpr int MT = NB / 16;
    const int AT = nca / 16;
    for (int tile = wv; tile < kAdjRG * MT * AT; tile += 4) {
        const int r = tile / (MT * AT), mt = (tile / AT) % MT, at = tile % AT;
        const int row = row0 + r;
        if (row >= rows) break;  // tiles are ordered by row
        const double *S = Sd + (size_t)r * NB * NB + (size_t)(16 * mt + lr) * NB;
        const float *kt = KtT + (size_t)(16 * at + lr) * KS;
        f4 acc = f4{0, 0, 0, 0};
#pragma unroll
        for (int h = 0; h < NB / 16; ++h) {
            const int l0 = 16 * h + 4 * lk;
            const double2 s0 = *(const double2 *)(S + l0), s1 = *(const double2 *)(S + l0 + 2);
            const float4 k = *(const float4 *)(kt + l0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)s0.x, k.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)s0.y, k.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)s1.x, k.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)s1.y, k.w, acc, 0, 0, 0);
        }
        const int a = 16 * at + lr;
        if (a < n_chi)
            *(float4 *)(dY + (((size_t)beta * rows_pad + row) * n_chi + a) * NB + 16 * mt + 4 * lk) =
                make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
}

// dK_chi[beta][l][a] = wchi_a chi_a sum_{row, m} S[row][m][l] Y[row][a][m]
// Work-group = (64 chi nodes, cosmology), 4 waves: lane = chi node, wave w takes rows w, w + 4, ...
// and keeps NB sums (one per l).  A wave copies its row's S (NB x NB) into its own LDS slot with
// coalesced loads and reads it back as broadcasts (every lane the same address); the row's Y
// entries are 16-byte loads per lane.  The waves' sums are added in LDS in a fixed order.
template <typename T, int NB>
__global__ __launch_bounds__(256) void adj_kchi_kernel(const T *__restrict__ Y, const double *__restrict__ Sg,
                                                       const double *__restrict__ wchi,
                                                       const double *__restrict__ chi, int n_chi, int rows,
                                                       int rows_pad, int nbins, double *__restrict__ dK) {
    constexpr int KV = 16 / sizeof(T), SV = NB * NB / 2;  // 16-byte pieces of one S
    __shared__ __align__(16) double Ss[4][NB * NB];
    __shared__ double part[3][64][NB + 1];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int beta = blockIdx.y;
    const int a = blockIdx.x * 64 + lane, ac = min(a, n_chi - 1);
    double *sw = Ss[w];
    double acc[NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) acc[l] = 0.0;
    for (int row = w; row < rows; row += 4) {
        const double *sg = Sg + ((size_t)beta * rows_pad + row) * NB * NB;
        const T *y = Y + (((size_t)beta * rows_pad + row) * n_chi + ac) * NB;
        T yv[NB];
#pragma unroll
        for (int q = 0; q < NB; q += KV) *(U4 *)(yv + q) = *(const U4 *)(y + q);
#pragma unroll
        for (int q = lane; q < SV; q += 64) *(U4 *)(sw + 2 * q) = *(const U4 *)(sg + 2 * q);
        // the slot's writes are done before any lane reads them (LDS accesses of a wave complete
        // in order; the asm also keeps the compiler from moving accesses across it)
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const double ym = (double)yv[m];
#pragma unroll
            for (int l = 0; l < NB; l += 2) {
                const double2 sv = *(const double2 *)(sw + m * NB + l);
                acc[l] = fma(sv.x, ym, acc[l]);
                acc[l + 1] = fma(sv.y, ym, acc[l + 1]);
            }
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // reads done before the next row's writes
    }
    if (w > 0)
#pragma unroll
        for (int l = 0; l < NB; ++l) part[w - 1][lane][l] = acc[l];
    __syncthreads();
    if (w == 0 && a < n_chi) {
        const double f = wchi[a] * chi[a];
#pragma unroll
        for (int l = 0; l < NB; ++l)
            if (l < nbins)
                dK[((size_t)beta * nbins + l) * n_chi + a] =
                    f * (((acc[l] + part[0][lane][l]) + part[1][lane][l]) + part[2][lane][l]);
    }
}

// per (chi_a, cosmology):  dw[b][row] = wR_b sum_m K2_m(a, b) dY[row][a][m]
//                          dK2[m][a][b] = wR_b sum_row dY[row][a][m] w[b][row]
// dY of the work-group's chi_a sits in LDS with rows NB + 1 doubles apart, so that lanes reading
// consecutive rows hit distinct banks.  (dK2 with one wave per R node, lanes over rows and
// a shuffle reduction of the NB sums measured slower than this loop.)
template <int NB>
constexpr int adj_w_stride() { return NB + 1; }

template <typename T, int NB>
__global__ __launch_bounds__(256) void adj_w_kernel(const T *__restrict__ dY, const T *__restrict__ w,
                                                    const double *__restrict__ Kchi2, const double *__restrict__ wR,
                                                    int NP, int nR, int n_chi, int rows, int rows_pad, int nbins,
                                                    T *__restrict__ dw, double *__restrict__ dK2) {
    constexpr int DS = adj_w_stride<NB>();
    extern __shared__ __align__(16) unsigned char smem_a[];
    double *Kh = (double *)smem_a;                   // [nR][NB]
    double *dYa = Kh + (size_t)nR * NB;              // [rows_pad][DS]
    const int a = blockIdx.x, beta = blockIdx.y;
    for (int i = threadIdx.x; i < nR * NB; i += blockDim.x) {
        const int b = i / NB, m = i % NB;
        Kh[i] = m < nbins ? wR[b] * Kchi2[(((size_t)beta * nbins + m) * n_chi + a) * nR + b] : 0.0;
    }
    for (int i = threadIdx.x; i < rows_pad * NB; i += blockDim.x) {
        const int row = i / NB, m = i % NB;
        dYa[row * DS + m] = row < rows ? (double)dY[(((size_t)beta * rows_pad + row) * n_chi + a) * NB + m] : 0.0;
    }
    __syncthreads();
    const size_t base = ((size_t)beta * NP + (size_t)a * nR) * rows_pad;
    // dw: item = (row, quarter of the R nodes); the row's dY stays in registers and the weights of
    // a node are the same address for the whole wave (broadcast reads)
    for (int i = threadIdx.x; i < 4 * rows_pad; i += blockDim.x) {
        const int row = i % rows_pad, q = i / rows_pad;
        double yr[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) yr[m] = dYa[row * DS + m];
        for (int b = q * nR / 4; b < (q + 1) * nR / 4; ++b) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < NB; ++m) v += Kh[b * NB + m] * yr[m];
            dw[base + (size_t)b * rows_pad + row] = (T)v;
        }
    }
    if (dK2) {
        for (int i = threadIdx.x; i < nR * NB; i += blockDim.x) {
            const int b = i / NB, m = i % NB;
            if (m >= nbins) continue;
            const T *wr = w + base + (size_t)b * rows_pad;
            double v = 0.0;
            for (int row = 0; row < rows; ++row) v += dYa[row * DS + m] * (double)wr[row];
            dK2[(((size_t)beta * nbins + m) * n_chi + a) * nR + b] = wR[b] * v;
        }
    }
}

// FP32 path of adj_w_kernel on MFMA (v_mfma_f32_16x16x4_f32), per (chi_a, cosmology):
//   dw^T [rows x n_R] = dY [rows x NB] x Kh^T [NB x n_R],     Kh[b][m] = wR_b K2_m(a, b)
//   dK2  [n_R x NB]   = w  [n_R x rows] x dY [rows x NB]      (then times wR_b)
// The K order of an MFMA is a free permutation shared by its operands: for dw, MFMA s of a tile
// takes bins 4 lk + s % 4 + 16 (s / 4) from lane group lk, so a lane reads its row's bins as
// 16-byte pieces; for dK2, MFMA e of a 16-row chunk takes row 16 c + 4 lk + e, so a lane reads w
// of its node and dY^T of its bin as 16-byte pieces.  Kh and dY^T (rows past `rows` zero) sit in
// LDS; w is read from global memory, a chunk of 16-row steps at a time.  Wave v makes the dw tiles
// v, v + 4, ... and the dK2 node tiles v, v + 4.
template <int NB>
__global__ __launch_bounds__(256) void adj_w_mfma_kernel(const float *__restrict__ dY, const float *__restrict__ w,
                                                         const double *__restrict__ Kchi2,
                                                         const double *__restrict__ wR, int NP, int nR, int n_chi,
                                                         int rows, int rows_pad, int nbins, float *__restrict__ dw,
                                                         double *__restrict__ dK2) {
    extern __shared__ __align__(16) unsigned char smem_aw[];
    const int nRt = (nR + 15) / 16, nRp = 16 * nRt;
    float *Kh = (float *)smem_aw;                 // [nRp][NB]
    float *dYt = Kh + (size_t)nRp * NB;            // [NB][rows_pad + 4]
    const int ds = rows_pad + 4;
    const int a = blockIdx.x, beta = blockIdx.y;
    for (int i = threadIdx.x; i < nRp * NB; i += blockDim.x) {
        const int b = i / NB, m = i % NB;
        Kh[i] = (b < nR && m < nbins) ? (float)(wR[b] * Kchi2[(((size_t)beta * nbins + m) * n_chi + a) * nR + b])
                                      : 0.f;
    }
    const float *dya = dY + ((size_t)beta * rows_pad * n_chi + a) * NB;  // + row * n_chi * NB + m (rows < rows)
    for (int i = threadIdx.x; i < rows_pad * NB; i += blockDim.x) {
        const int row = i / NB, m = i % NB;
        dYt[(size_t)m * ds + row] = row < rows ? dya[(size_t)row * n_chi * NB + m] : 0.f;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const size_t base = ((size_t)beta * NP + (size_t)a * nR) * rows_pad;  // w, dw of node b: + b * rows_pad
    const int RTn = rows_pad / 16;
    constexpr int NQ = NB / 16;  // 16-bin groups
    // dw (the A operand from dY^T in LDS: lanes of consecutive rows read consecutive words); staging
    // a node tile's rows in LDS for contiguous stores measured slower (two barriers per tile)
    for (int tile = wv; tile < RTn * nRt; tile += 4) {
        const int rt = tile % RTn, bt = tile / RTn;
        const int row = 16 * rt + lr, b = 16 * bt + lr;
        f4 acc = f4{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float *yt = dYt + (size_t)(16 * q + 4 * lk) * ds + row;
            const float4 y = make_float4(yt[0], yt[ds], yt[2 * ds], yt[3 * ds]);
            const float4 k = *(const float4 *)(Kh + (size_t)b * NB + 16 * q + 4 * lk);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(y.x, k.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(y.y, k.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(y.z, k.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(y.w, k.w, acc, 0, 0, 0);
        }
        // lane holds rows 16 rt + 4 lk .. + 3 of node b = 16 bt + lr
        if (b < nR) *(float4 *)(dw + base + (size_t)b * rows_pad + 16 * rt + 4 * lk) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
    // dK2: node tiles wv, wv + 4, ...; lane (node 16 bt + lr) reads w of that node
    if (dK2) {
        for (int bt = wv; bt < nRt; bt += 4) {
            const int b = min(16 * bt + lr, nR - 1);
            const float *wr = w + base + (size_t)b * rows_pad;
            f4 acc[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] = f4{0, 0, 0, 0};
            // the node's w in chunks of kWChunk 16-row steps, every load of a chunk issued before its MFMAs
            constexpr int kWChunk = 6;
            for (int c0 = 0; c0 < RTn; c0 += kWChunk) {
                float4 x[kWChunk];
#pragma unroll
                for (int u = 0; u < kWChunk; ++u)
                    x[u] = *(const float4 *)(wr + 16 * min(c0 + u, RTn - 1) + 4 * lk);
#pragma unroll
                for (int u = 0; u < kWChunk; ++u) {
                    if (c0 + u >= RTn) break;
                    const int c = c0 + u;
                    const float xv[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const float4 y = *(const float4 *)(dYt + (size_t)(16 * q + lr) * ds + 16 * c + 4 * lk);
                        const float yv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[e], yv[e], acc[q], 0, 0, 0);
                    }
                }
            }
            // lane holds nodes 16 bt + 4 lk + r of bin 16 q + lr
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int m = 16 * q + lr;
                if (m >= nbins) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int bb = 16 * bt + 4 * lk + r;
                    if (bb < nR) dK2[(((size_t)beta * nbins + m) * n_chi + a) * nR + bb] = wR[bb] * (double)acc[q][r];
                }
            }
        }
    }
}

// transpose contraction: dc[beta][ab][n] = sum_row Ttilde[ab][row][n] dw[beta][ab][row]
// M = n (wave w owns n tiles w, w+4), N = cosmologies (BT), K = rows, on MFMA.
template <bool F64>
__global__ __launch_bounds__(256) void contract_t_kernel(const typename std::conditional<F64, double, float>::type
                                                             *__restrict__ basis,
                                                         const typename std::conditional<F64, double, float>::type
                                                             *__restrict__ dw,
                                                         int batch, int NP, int rows_pad, int ncp,
                                                         typename std::conditional<F64, double, float>::type
                                                             *__restrict__ dc) {
    using T = typename std::conditional<F64, double, float>::type;
    using Acc = typename std::conditional<F64, d4, f4>::type;
    constexpr int BT = F64 ? 32 : 64, BTN = BT / 16;
    extern __shared__ __align__(16) unsigned char smem_t[];
    const int dst = rows_pad + 1;
    T *ws = (T *)smem_t;  // [BT][rows_pad + 1]
    int ab, tile;
    if (!point_tile(NP, (batch + BT - 1) / BT, ab, tile)) return;  // uniform over the work-group
    const int beta0 = tile * BT;
    const int nb = min(BT, batch - beta0);
    for (int i = threadIdx.x; i < BT * rows_pad; i += blockDim.x) {
        const int bb = i / rows_pad, row = i % rows_pad;
        ws[bb * dst + row] = bb < nb ? dw[((size_t)(beta0 + bb) * NP + ab) * rows_pad + row] : (T)0;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int NT = ncp >> 4;
    const T *bp = basis + (size_t)ab * rows_pad * ncp;  // FP64: row-major; FP32: tiled layout
    Acc acc[2][BTN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < BTN; ++j) acc[i][j] = Acc{0, 0, 0, 0};
    // K steps of 4 rows in groups of 4 (rows_pad / 4 is a multiple of 4); the basis values of the
    // next group are loaded while the current one runs on the MFMA units
    const int S4 = rows_pad / 4;
    auto loadA = [&](int st0, T(&av)[4][2]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int row = 4 * (st0 + u) + lk;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int nt = wv + 4 * i;
                const size_t o = F64 ? (size_t)row * ncp + 16 * nt + lr : tiled_off(row, 16 * nt + lr, ncp / 16, 4);
                av[u][i] = nt < NT ? bp[o] : (T)0;
            }
        }
    };
    auto compute = [&](int st0, const T(&av)[4][2]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int row = 4 * (st0 + u) + lk;
            T bv[BTN];
#pragma unroll
            for (int j = 0; j < BTN; ++j) bv[j] = ws[(16 * j + lr) * dst + row];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < BTN; ++j) {
                    if constexpr (F64)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][i], bv[j], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u][i], bv[j], acc[i][j], 0, 0, 0);
                }
        }
    };
    T a0[4][2], a1[4][2];
    loadA(0, a0);
    for (int st0 = 0; st0 < S4; st0 += 8) {
        if (st0 + 4 < S4) loadA(st0 + 4, a1);
        compute(st0, a0);
        if (st0 + 4 < S4) {
            if (st0 + 8 < S4) loadA(st0 + 8, a0);
            compute(st0 + 4, a1);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int nt = wv + 4 * i;
        if (nt >= NT) continue;
#pragma unroll
        for (int j = 0; j < BTN; ++j) {
            const int bb = 16 * j + lr;
            if (bb >= nb) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * nt + (F64 ? lk + 4 * r : 4 * lk + r);
                dc[((size_t)(beta0 + bb) * NP + ab) * ncp + n] = acc[i][j][r];
            }
        }
    }
}

// dP[row][j] = sum_{n < N} D[n][j] dc[row][n] (nodal input) or dP[row][n] = dc[row][n]
// (coefficient input), written in P's dtype; N <= 128.  Work-group = kAdjRows rows, whose dc rows
// sit in LDS in FP64; thread (j, h) makes column j of the rows of parity h, so each D[n][j] it
// reads serves 32 independent FP64 accumulators (LDS reads of dc are broadcasts: every lane of a
// wave reads the same row).
constexpr int kAdjRows = 64;
template <typename T, typename PT>
__global__ __launch_bounds__(256) void adj_project_kernel(const T *__restrict__ dc, const double *__restrict__ Dn,
                                                          int N, int ncp, long nrows, int coef, PT *__restrict__ dP) {
    constexpr int RH = kAdjRows / 2;
    static_assert(kMaxCheb <= 128, "one thread column per Chebyshev node");
    __shared__ double cs[kAdjRows][128 + 1];
    const long row0 = (long)blockIdx.x * kAdjRows;
    for (int i = threadIdx.x; i < kAdjRows * N; i += blockDim.x) {
        const int r = i / N, n = i % N;
        cs[r][n] = row0 + r < nrows ? (double)dc[(row0 + r) * ncp + n] : 0.0;
    }
    __syncthreads();
    const int j = threadIdx.x % 128, h = threadIdx.x / 128;
    if (j >= N) return;
    double acc[RH];
    if (coef) {
#pragma unroll
        for (int k = 0; k < RH; ++k) acc[k] = cs[2 * k + h][j];
    } else {
#pragma unroll
        for (int k = 0; k < RH; ++k) acc[k] = 0.0;
        for (int n = 0; n < N; ++n) {
            const double d = Dn[(size_t)n * N + j];
#pragma unroll
            for (int k = 0; k < RH; ++k) acc[k] = fma(d, cs[2 * k + h][n], acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < RH; ++k) {
        const long row = row0 + 2 * k + h;
        if (row < nrows) dP[row * N + j] = (PT)acc[k];
    }
}

// The transposed projection on MFMA for N % 8 == 0 (nodal P), with the even/odd split of the
// forward one: with D[n][N-1-j] = (-1)^n D[n][j], for j < N/2
//     e_j = sum_m D[2m][j] dc_{2m},   o_j = sum_m D[2m+1][j] dc_{2m+1},
//     dP_j = e_j + o_j,               dP_{N-1-j} = e_j - o_j,
// two [rows x N/2] x [N/2 x N/2] products.  The tables Et[j][m] = D[2m][j] and Ot[j][m] = D[2m+1][j]
// (zero past N/2) sit in LDS; a lane loads 8 consecutive dc values of its row per step (the even
// ones feed e, the odd ones o).  FP32 path: v_mfma_f32_16x16x4_f32, two row tiles per wave, 128
// rows per work-group; FP64 path: v_mfma_f64_16x16x4_f64, one row tile per wave, 64 rows.
template <typename PT, int NT>
__global__ __launch_bounds__(256) void adj_project_split_kernel(const float *__restrict__ dc,
                                                                const float *__restrict__ Dn, int N, int ncp,
                                                                long nrows, PT *__restrict__ dP) {
    constexpr int RT = 2, KSTEP = 16;
    extern __shared__ __align__(16) unsigned char smem_ap[];
    const int H = N / 2;
    constexpr int Hp = 16 * NT, hs = Hp + 4;
    float *Et = (float *)smem_ap, *Ot = Et + (size_t)Hp * hs;
    for (int i = threadIdx.x; i < Hp * Hp; i += blockDim.x) {
        const int j = i / Hp, m = i % Hp;
        const bool in = j < H && m < H;
        Et[(size_t)j * hs + m] = in ? Dn[(size_t)(2 * m) * N + j] : 0.f;
        Ot[(size_t)j * hs + m] = in ? Dn[(size_t)(2 * m + 1) * N + j] : 0.f;
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const long row0 = (long)blockIdx.x * (64 * RT) + 16 * RT * w;
    const float *prow[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) prow[r] = dc + min(row0 + 16 * r + lr, nrows - 1) * (long)ncp;
    f4 ae[RT][NT], ao[RT][NT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) ae[r][t] = ao[r][t] = f4{0, 0, 0, 0};
    // dc[2 m0 .. 2 m0 + 7] of each row; clamped below N/2, where the tables are zero anyway
    auto load = [&](int st, float4 (&lo)[RT], float4 (&hi)[RT]) {
        const int m0 = min(st * KSTEP + lk * 4, H - 4);
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            lo[r] = *(const float4 *)(prow[r] + 2 * m0);
            hi[r] = *(const float4 *)(prow[r] + 2 * m0 + 4);
        }
    };
    auto compute = [&](int st, const float4 (&lo)[RT], const float4 (&hi)[RT]) {
        const int m0 = st * KSTEP + lk * 4;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float4 de = *(const float4 *)(Et + (size_t)(16 * t + lr) * hs + m0);
            const float4 dd = *(const float4 *)(Ot + (size_t)(16 * t + lr) * hs + m0);
            const float dev[4] = {de.x, de.y, de.z, de.w}, dov[4] = {dd.x, dd.y, dd.z, dd.w};
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const float ev[4] = {lo[r].x, lo[r].z, hi[r].x, hi[r].z}, ov[4] = {lo[r].y, lo[r].w, hi[r].y, hi[r].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ae[r][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ev[e], dev[e], ae[r][t], 0, 0, 0);
                    ao[r][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ov[e], dov[e], ao[r][t], 0, 0, 0);
                }
            }
        }
    };
    float4 lo[2][RT], hi[2][RT];
    load(0, lo[0], hi[0]);
#pragma unroll
    for (int st = 0; st < NT; ++st) {
        if (st + 1 < NT) load(st + 1, lo[(st + 1) & 1], hi[(st + 1) & 1]);
        compute(st, lo[st & 1], hi[st & 1]);
    }
    // lane holds rows 16 r + 4 lk + q of column j = 16 t + lr
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = 16 * t + lr;
            if (j >= H) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long row = row0 + 16 * r + 4 * lk + q;
                if (row >= nrows) continue;
                const float e = ae[r][t][q], o = ao[r][t][q];
                dP[row * N + j] = (PT)(e + o);
                dP[row * N + N - 1 - j] = (PT)(e - o);
            }
        }
}

template <typename PT, int NT>
__global__ __launch_bounds__(256) void adj_project_split64_kernel(const double *__restrict__ dc,
                                                                  const double *__restrict__ Dn, int N, int ncp,
                                                                  long nrows, PT *__restrict__ dP) {
    constexpr int KSTEP = 16;
    extern __shared__ __align__(16) unsigned char smem_ap64[];
    const int H = N / 2;
    constexpr int Hp = 16 * NT, hs = Hp + 2;
    double *Et = (double *)smem_ap64, *Ot = Et + (size_t)Hp * hs;
    for (int i = threadIdx.x; i < Hp * Hp; i += blockDim.x) {
        const int j = i / Hp, m = i % Hp;
        const bool in = j < H && m < H;
        Et[(size_t)j * hs + m] = in ? Dn[(size_t)(2 * m) * N + j] : 0.0;
        Ot[(size_t)j * hs + m] = in ? Dn[(size_t)(2 * m + 1) * N + j] : 0.0;
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const long row0 = (long)blockIdx.x * 64 + 16 * w;
    const double *pr = dc + min(row0 + lr, nrows - 1) * (long)ncp;
    d4 ae[NT], ao[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) ae[t] = ao[t] = d4{0, 0, 0, 0};
    auto load = [&](int st, double (&v)[8]) {
        const int m0 = min(st * KSTEP + lk * 4, H - 4);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double2 x = *(const double2 *)(pr + 2 * m0 + 2 * u);
            v[2 * u] = x.x, v[2 * u + 1] = x.y;
        }
    };
    auto compute = [&](int st, const double (&v)[8]) {
        const int m0 = st * KSTEP + lk * 4;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double *de = Et + (size_t)(16 * t + lr) * hs + m0, *dd = Ot + (size_t)(16 * t + lr) * hs + m0;
            const double2 e0 = *(const double2 *)de, e1 = *(const double2 *)(de + 2);
            const double2 o0 = *(const double2 *)dd, o1 = *(const double2 *)(dd + 2);
            const double dev[4] = {e0.x, e0.y, e1.x, e1.y}, dov[4] = {o0.x, o0.y, o1.x, o1.y};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ae[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[2 * e], dev[e], ae[t], 0, 0, 0);
                ao[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[2 * e + 1], dov[e], ao[t], 0, 0, 0);
            }
        }
    };
    double v[2][8];
    load(0, v[0]);
#pragma unroll
    for (int st = 0; st < NT; ++st) {
        if (st + 1 < NT) {
            load(st + 1, v[(st + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);  // keep the next step's loads ahead of these MFMAs
        }
        compute(st, v[st & 1]);
    }
    // f64 result layout: row 4 r + lk of the tile in register r of lane j % 16 + 16 lk
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int j = 16 * t + lr;
        if (j >= H) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long row = row0 + 4 * r + lk;
            if (row >= nrows) continue;
            const double e = ae[t][r], o = ao[t][r];
            dP[row * N + j] = (PT)(e + o);
            dP[row * N + N - 1 - j] = (PT)(e - o);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
struct Ctx {
    int prec, ng, ns, nbins, npairs, nbp;
    // the call contracts the nodal basis (B = Ttilde D) with its nodal P: P read in place of c, or
    // converted into c's layout as coefficient input is (no projection either way)
    bool nodal = false;
    bool direct = false;  // nodal, with P itself as the contraction's operand
    EllSel sel;
    EllInv inv;
};

struct Layout {
    size_t c, clo, cs, w, kt, y, dy, sg, dw, dc, total;
};

// cosmologies per work-group of the adjoint's transposed contraction (their dw rows sit in LDS)
constexpr int kAdjBT = 32;

// Below this batch the fused kernel, which keeps one work-group per CU busy with a barrier per
// b, streams the basis more slowly than the unfused contraction (many independent work-groups);
// there the w round trip through HBM is the cheaper part.
constexpr int kFusedMinBatch = 32;

// bins computed by the fused kernel (multiple of 4), 0 when it does not apply
int fused_nb(int prec, int nbins, int batch) {
    if (prec == BLAST_FP64 || nbins > 20 || (batch < kFusedMinBatch && prec != BLAST_FP16X3)) return 0;
    return (nbins + 3) / 4 * 4;
}

// FP32 calls that keep w take the fused path too (its kernel stores the w tiles as it goes)
bool fused_keeps_w(int prec, int nbins, int batch) { return prec == BLAST_FP32 && fused_nb(prec, nbins, batch); }

Layout layout_of(const blast_plan *p, int batch, int prec, int nbins, bool need_w, bool adjoint,
                 bool nodal = false) {
    Layout L{};
    const size_t nc = nodal ? 0 : (size_t)batch * p->NP * p->nc_pad;
    const size_t ce = prec == BLAST_FP64 ? 8 : (prec == BLAST_FP32 ? 4 : 2);
    const size_t te = prec == BLAST_FP64 ? 8 : 4;
    const int nbp = nbins <= 16 ? 16 : 32;
    const size_t ny = (size_t)batch * p->n_chi * p->rows_pad * nbp;
    size_t off = 0;
    L.c = off;
    off += align256(nc * ce);
    L.clo = off;
    if (prec == BLAST_BF16X3 || prec == BLAST_FP16X3) off += align256(nc * 2);
    L.cs = off;
    if (prec == BLAST_FP16X3 && !nodal) off += align256((size_t)batch * p->NP * 4);
    L.w = off;
    L.kt = off;
    if (need_w) {
        const int fnb = adjoint ? 0 : fused_nb(prec, nbins, batch);
        // the fused path keeps Kt where the unfused one keeps w
        off += align256(std::max((size_t)batch * p->NP * p->rows_pad * te, (size_t)batch * p->NP * fnb * 4));
    } else if (!adjoint && fused_keeps_w(prec, nbins, batch)) {
        off += align256((size_t)batch * p->NP * fused_nb(prec, nbins, batch) * 4);
    }
    L.y = off;
    off += align256(ny * te);
    if (adjoint) {
        L.dy = off;
        off += align256(ny * te);
        L.sg = off;
        off += align256((size_t)batch * p->rows_pad * nbp * nbp * 8);
        L.dw = off;
        off += align256((size_t)batch * p->NP * p->rows_pad * te);
        L.dc = off;
        off += align256(nc * te);
    }
    L.total = off;
    return L;
}

size_t workspace_bytes_impl(const blast_plan *p, int batch, int prec, int n_bins) {
    const size_t f = layout_of(p, batch, prec, n_bins, true, false).total;
    const size_t b = prec <= BLAST_FP32 ? layout_of(p, batch, prec, n_bins, true, true).total : 0;
    return f > b ? f : b;
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
            (const void *)quad_y_kernel<double, 16>, (const void *)quad_y_kernel<double, 32>,
            (const void *)quad_y_kernel<float, 16>, (const void *)quad_y_kernel<float, 32>,
            (const void *)quad_c_mfma_kernel<double, 1>, (const void *)quad_c_mfma_kernel<double, 2>,
            (const void *)quad_c_mfma_kernel<float, 1>, (const void *)quad_c_mfma_kernel<float, 2>,
            (const void *)adj_w_kernel<double, 16>, (const void *)adj_w_kernel<double, 32>,
            (const void *)adj_w_kernel<float, 16>, (const void *)adj_w_kernel<float, 32>,
            (const void *)contract_t_kernel<true>, (const void *)contract_t_kernel<false>,
            (const void *)adj_project_split64_kernel<double, 4>, (const void *)adj_project_split64_kernel<float, 4>,
            (const void *)adj_project_split64_kernel<double, 3>, (const void *)adj_project_split64_kernel<float, 3>,
            (const void *)adj_w_mfma_kernel<16>, (const void *)adj_w_mfma_kernel<32>,
            (const void *)contract_tiled_kernel<BLAST_FP32, 4, kAdjBT>,
            (const void *)contract_tiled_kernel<BLAST_FP32, 4, 2 * kAdjBT, 1>,
            (const void *)adj_dy_mfma_kernel<16>, (const void *)adj_dy_mfma_kernel<32>,
        };
        for (const void *f : fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
            if (e != hipSuccess) err = e;
        }
    });
    return err;
}

// Threads per work-group of quad_y_kernel: a work-group of T threads spans at most
// (T - 1) / RQ + 2 chi nodes, whose R weights [node][n_R][NB] it keeps in LDS; the largest of
// 256, 192, 128, 64 whose table fits in 160 KB (0: none fits).
int quad_y_threads(const blast_plan *p, bool f64, int nbp) {
    const int rq = p->rows_pad / (f64 ? 2 : 4);
    const size_t el = f64 ? 8 : 4;
    for (int t = 256; t >= 64; t -= 64)
        if ((size_t)((t - 1) / rq + 2) * p->n_R * nbp * el <= 160 * 1024) return t;
    return 0;
}


blast_status check_args(const blast_plan *p, const blast_cl_args *a, Ctx &x) {
    if (a->batch < 1) return set_error("batch must be >= 1"), BLAST_E_INVALID;
    if (a->precision < 0 || a->precision > 4) return set_error("unknown precision %d", a->precision), BLAST_E_INVALID;
    x.prec = a->precision;
    const int prec = x.prec;
    const bool resident = (prec == BLAST_FP64 && p->basis.f64) || (prec == BLAST_FP32 && p->basis.f32) ||
                          (prec == BLAST_BF16 && p->basis.hi) || (prec == BLAST_BF16X3 && p->basis.lo) ||
                          (prec == BLAST_FP16X3 && p->basis.l16);
    if (!resident) return set_error("precision %d is not resident in this plan", prec), BLAST_E_INVALID;
    if (a->p_dtype != 0 && a->p_dtype != 1) return set_error("p_dtype must be 0 (FP64) or 1 (FP32)"), BLAST_E_INVALID;
    if (a->p_kind != 0 && a->p_kind != 1) return set_error("p_kind must be 0 (nodal) or 1 (coefficients)"), BLAST_E_INVALID;
    if (!a->P || !a->K_chi || !a->K_chi2) return set_error("P, K_chi and K_chi2 are required"), BLAST_E_INVALID;
    // every route reads P in 16-byte pieces (the projections' vector loads, the nodal DMAs)
    if ((uintptr_t)a->P & 15) return set_error("P must be 16-byte aligned"), BLAST_E_INVALID;
    x.ng = a->n_g;
    x.ns = a->n_s;
    x.nbins = x.ng + x.ns;
    if (x.ng < 0 || x.ns < 0 || x.nbins < 1 || x.nbins > kMaxBins)
        return set_error("need n_g, n_s >= 0 and 1 <= n_g + n_s <= %d", kMaxBins), BLAST_E_INVALID;
    x.nbp = x.nbins <= 16 ? 16 : 32;
    if (a->types == 0 || (a->types & ~p->types))
        return set_error("types 0x%x not a non-empty subset of the plan's 0x%x", a->types, p->types), BLAST_E_INVALID;
    x.npairs = npairs_of(x.ng, x.ns, a->types);
    if (x.npairs < 1) return set_error("no bin pairs for these types and bins"), BLAST_E_INVALID;
    x.sel = EllSel{};
    for (int i = 0; i < kMaxEll; ++i) x.inv.io[i] = -1;
    if (a->n_ell_out == 0) {
        x.sel.n_out = p->n_ell;
        for (int i = 0; i < p->n_ell; ++i) x.sel.idx[i] = (int16_t)i;
    } else {
        if (a->n_ell_out < 0 || a->n_ell_out > p->n_ell || !a->ell_idx)
            return set_error("bad n_ell_out / ell_idx"), BLAST_E_INVALID;
        x.sel.n_out = a->n_ell_out;
        for (int i = 0; i < a->n_ell_out; ++i) {
            const int v = a->ell_idx[i];
            if (v < 0 || v >= p->n_ell || (i && v <= a->ell_idx[i - 1]))
                return set_error("ell_idx must be increasing indices into the plan's ell"), BLAST_E_INVALID;
            x.sel.idx[i] = (int16_t)v;
        }
    }
    for (int i = 0; i < x.sel.n_out; ++i) x.inv.io[x.sel.idx[i]] = (int16_t)i;
    if (((size_t)x.nbp * (p->n_chi + 4) + 4 * 32 * 32) * sizeof(double) > 160 * 1024)
        return set_error("n_chi too large for the chi-quadrature tile"), BLAST_E_UNSUPPORTED;
    if (!quad_y_threads(p, x.prec == BLAST_FP64, x.nbp))
        return set_error("n_R too large for the R-quadrature tile"), BLAST_E_UNSUPPORTED;
    return BLAST_OK;
}

unsigned char *get_workspace(blast_plan *p, const blast_cl_args *a, size_t need, blast_status &st) {
    st = BLAST_OK;
    if (a->workspace) {
        if (a->workspace_bytes < need) {
            set_error("workspace of %zu bytes is smaller than the %zu needed", a->workspace_bytes, need);
            st = BLAST_E_INVALID;
            return nullptr;
        }
        return (unsigned char *)a->workspace;
    }
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->scratch_bytes < need) {
        (void)hipDeviceSynchronize();
        if (p->scratch) (void)hipFree(p->scratch);
        p->scratch = nullptr;
        p->scratch_bytes = 0;
        hipError_t e = hipMalloc(&p->scratch, need);
        if (e != hipSuccess) {
            p->scratch = nullptr;
            set_error("plan scratch of %zu bytes: %s", need, hipGetErrorString(e));
            st = BLAST_E_OOM;
            return nullptr;
        }
        p->scratch_bytes = need;
    }
    return (unsigned char *)p->scratch;
}

// stage 1: P (nodal values or coefficients) -> c in the contraction's layout
void stage_project(blast_plan *p, const blast_cl_args *a, const Ctx &x, void *c, uint16_t *clo, float *cs,
                   hipStream_t s) {
    const int prec = x.prec;
    const long nrows = (long)a->batch * p->NP;
    const int N = p->n_cheb, ncp = p->nc_pad;
    const bool f64 = prec == BLAST_FP64;
    const bool p64 = a->p_dtype == 0;
    const int out = f64 ? 0 : (prec == BLAST_FP32 ? 1 : (prec == BLAST_FP16X3 ? 3 : 2));
    if (a->p_kind == 1 && out == 3) {
        dim3 grid((unsigned)((nrows + 3) / 4));
        if (p64)
            hipLaunchKernelGGL((coef_in16_kernel<double>), grid, dim3(256), 0, s, (const double *)a->P, N, ncp, nrows,
                               (uint16_t *)c, clo, cs, (long)p->NP, a->batch);
        else
            hipLaunchKernelGGL((coef_in16_kernel<float>), grid, dim3(256), 0, s, (const float *)a->P, N, ncp, nrows,
                               (uint16_t *)c, clo, cs, (long)p->NP, a->batch);
        return;
    }
    if (a->p_kind == 1) {
        dim3 grid((unsigned)((nrows * ncp + 255) / 256));
#define BLAST_CI(PT, O) \
    hipLaunchKernelGGL((coef_in_kernel<PT, O>), grid, dim3(256), 0, s, (const PT *)a->P, N, ncp, nrows, c, clo)
        if (p64 && out == 0) BLAST_CI(double, 0);
        if (p64 && out == 1) BLAST_CI(double, 1);
        if (p64 && out == 2) BLAST_CI(double, 2);
        if (!p64 && out == 0) BLAST_CI(float, 0);
        if (!p64 && out == 1) BLAST_CI(float, 1);
        if (!p64 && out == 2) BLAST_CI(float, 2);
#undef BLAST_CI
        return;
    }
    if (f64 && N % 8 == 0) {
        dim3 grid((unsigned)((nrows + 63) / 64));
        const size_t shp = (size_t)2 * (ncp / 2) * (ncp / 2 + 2) * sizeof(double);
        auto launch = [&](auto ptag, auto nttag) {
            using PT = typename decltype(ptag)::type;
            constexpr int NT = decltype(nttag)::value;
            hipLaunchKernelGGL((project_split64_kernel<PT, NT>), grid, dim3(256), shp, s, (const PT *)a->P,
                               p->d_dctn64, N, ncp, nrows, (double *)c);
        };
        auto by_nt = [&](auto ptag) {
            switch (ncp / 32) {  // Hp / 16 = ncp / 32
                case 1: launch(ptag, std::integral_constant<int, 1>()); break;
                case 2: launch(ptag, std::integral_constant<int, 2>()); break;
                case 3: launch(ptag, std::integral_constant<int, 3>()); break;
                default: launch(ptag, std::integral_constant<int, 4>()); break;
            }
        };
        if (p64) by_nt(TypeTag<double>());
        else by_nt(TypeTag<float>());
    } else if (!f64 && N % 8 == 0) {
        const size_t shp = (size_t)2 * (ncp / 2) * (ncp / 2 + 4) * sizeof(float);
        auto launch = [&](auto ptag, auto otag, auto nttag) {
            using PT = typename decltype(ptag)::type;
            constexpr int O = decltype(otag)::value, NT = decltype(nttag)::value;
            constexpr int rows_wg = 64 * split_rt();
            dim3 grid((unsigned)((nrows + rows_wg - 1) / rows_wg));
            hipLaunchKernelGGL((project_split_kernel<PT, O, NT>), grid, dim3(256), shp, s, (const PT *)a->P,
                               p->d_dctn32, N, ncp, nrows, c, clo);
        };
        auto by_nt = [&](auto ptag, auto otag) {
            switch (ncp / 32) {  // Hp / 16 = ncp / 32, ncp a multiple of 32 up to 128
                case 1: launch(ptag, otag, std::integral_constant<int, 1>()); break;
                case 2: launch(ptag, otag, std::integral_constant<int, 2>()); break;
                case 3: launch(ptag, otag, std::integral_constant<int, 3>()); break;
                default: launch(ptag, otag, std::integral_constant<int, 4>()); break;
            }
        };
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        if (p64 && out == 1) by_nt(TypeTag<double>(), I1());
        if (p64 && out == 2) by_nt(TypeTag<double>(), I2());
        if (!p64 && out == 1) by_nt(TypeTag<float>(), I1());
        if (!p64 && out == 2) by_nt(TypeTag<float>(), I2());
        if (out == 3) {
            // FP16 MFMA form: 16 points x 4 npass cosmologies per work-group, the work-groups of
            // kProjPG consecutive point blocks next to each other
            const int npass = std::min(kProjPasses, (a->batch + 3) / 4);
            const long NPB = (p->NP + 15) / 16, NBB = (a->batch + 4 * npass - 1) / (4 * npass);
            const dim3 grid((unsigned)((NPB + kProjPG - 1) / kProjPG * kProjPG * NBB));
            const int g = dct16_exp(N);
            auto launch16 = [&](auto ptag, auto nttag) {
                using PT = typename decltype(ptag)::type;
                constexpr int NT = decltype(nttag)::value;
                hipLaunchKernelGGL((project_h16_kernel<PT, NT>), grid, dim3(256), 0, s, (const PT *)a->P,
                                   p->d_dct16, N, ncp, g, (long)p->NP, a->batch, (uint16_t *)c, clo, cs, npass);
            };
            auto by_nt16 = [&](auto ptag) {
                switch (ncp / 32) {
                    case 1: launch16(ptag, std::integral_constant<int, 1>()); break;
                    case 2: launch16(ptag, std::integral_constant<int, 2>()); break;
                    case 3: launch16(ptag, std::integral_constant<int, 3>()); break;
                    default: launch16(ptag, std::integral_constant<int, 4>()); break;
                }
            };
            if (p64) by_nt16(TypeTag<double>());
            else by_nt16(TypeTag<float>());
        }
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

// stage 2: w = Ttilde c
void stage_contract(blast_plan *p, const blast_cl_args *a, const Ctx &x, const void *c, const uint16_t *clo, void *w,
                    hipStream_t s) {
    const int ncp = p->nc_pad;
    auto launch = [&](auto tag) {
        constexpr int PR = decltype(tag)::value;
        using E = typename Cfg<PR>::E;
        const int BT = Cfg<PR>::BT;
        const size_t cst = ncp + 16 / sizeof(E);
        const size_t sh = (size_t)BT * cst * sizeof(E) + (PR == BLAST_BF16X3 ? (size_t)BT * cst * 2 : 0);
        const dim3 grid = point_tile_grid(p->NP, (a->batch + BT - 1) / BT);
        const E *bas = PR == BLAST_FP64
                           ? (const E *)(x.nodal ? p->basis.nf64 : p->basis.f64)
                           : (PR == BLAST_FP32 ? (const E *)(x.nodal ? p->basis.nf32 : p->basis.f32)
                                               : (const E *)p->basis.hi);
        if constexpr (PR == BLAST_FP64) {
            hipLaunchKernelGGL((contract_kernel<PR>), grid, dim3(256), sh, s, bas, p->basis.lo, p->basis.scale,
                               (const E *)c, clo, a->batch, p->NP, p->rows_pad, ncp, w);
        } else {
            const int RT = p->rows_pad / 16;
            const int W = std::min((RT + kTilesPerWave - 1) / kTilesPerWave, 8);
            hipLaunchKernelGGL((contract_tiled_kernel<PR>), grid, dim3(64 * W), sh, s, bas, p->basis.lo,
                               p->basis.scale, (const E *)c, clo, a->batch, p->NP, p->rows_pad, ncp, (float *)w,
                               x.direct ? p->n_cheb : ncp);
        }
    };
    if (x.prec == BLAST_FP64) launch(std::integral_constant<int, BLAST_FP64>());
    if (x.prec == BLAST_FP32) launch(std::integral_constant<int, BLAST_FP32>());
    if (x.prec == BLAST_BF16) launch(std::integral_constant<int, BLAST_BF16>());
    if (x.prec == BLAST_BF16X3) launch(std::integral_constant<int, BLAST_BF16X3>());
}

// stage 3: Y = R-quadrature of w
void stage_quad_y(blast_plan *p, const blast_cl_args *a, const Ctx &x, const void *w, void *Y, hipStream_t s) {
    const bool f64 = x.prec == BLAST_FP64;
    const int rq = p->rows_pad / (f64 ? 2 : 4);
    const long total = (long)p->n_chi * rq;
    const int T = quad_y_threads(p, f64, x.nbp);  // > 0: checked when the call was prepared
    dim3 gq((unsigned)((total + T - 1) / T), a->batch);
    const int na_max = (T - 1) / rq + 2;
#define BLAST_QY(TY, NB)                                                                                        \
    hipLaunchKernelGGL((quad_y_kernel<TY, NB>), gq, dim3(T), (size_t)na_max * p->n_R * NB * sizeof(TY), s,   \
                       (const TY *)w, a->K_chi2, p->d_wR, p->NP, p->n_R, p->n_chi, p->rows_pad, x.nbins, (TY *)Y)
    if (f64 && x.nbp == 16) BLAST_QY(double, 16);
    if (f64 && x.nbp == 32) BLAST_QY(double, 32);
    if (!f64 && x.nbp == 16) BLAST_QY(float, 16);
    if (!f64 && x.nbp == 32) BLAST_QY(float, 32);
#undef BLAST_QY
}

// stages 2 + 3 fused (mixed precisions without w_save)
void stage_r_weights(blast_plan *p, const blast_cl_args *a, const Ctx &x, int nb, const float *cs, float *Kt,
                     hipStream_t s) {
    constexpr int KB = kt_cosmologies<float>();
    dim3 gk((unsigned)((p->NP + kKtP - 1) / kKtP), (unsigned)((a->batch + KB - 1) / KB));
    hipLaunchKernelGGL(kt_kernel<float>, gk, dim3(256), 0, s, a->K_chi2, p->d_wR, cs, a->batch, x.nbins, nb, p->NP,
                       p->n_R, Kt);
}

// x.nodal: c is the caller's FP32 P and the basis operand the nodal basis
void stage_contract_quad(blast_plan *p, const blast_cl_args *a, const Ctx &x, int nb, const void *c,
                         const uint16_t *clo, const float *Kt, float *Y, float *w_out, hipStream_t s) {
    const bool nodal = x.nodal;
    const int RT = p->rows_pad / 16, nBT = (a->batch + 63) / 64;
    const int groups = (RT + kFusedTR - 1) / kFusedTR;
    const int units = p->n_chi * nBT * groups;
    const unsigned grid = (unsigned)((units + 7) / 8 * 8);
    // 4-bin groups the R-sum needs per type slot (clustering bins first): gg [0, ng), gs all,
    // ss [ng, nbins); 3 bits per bound
    int granges = 0;
    for (int sl = 0; sl < p->nt; ++sl) {
        const int t = p->tslot_type[sl];
        const int b0 = t == BLAST_SS ? x.ng : 0, b1 = t == BLAST_GG ? x.ng : x.nbins;
        const int q0 = b1 > b0 ? b0 / 4 : 0, q1 = b1 > b0 ? (b1 + 3) / 4 : 0;
        granges |= (q0 | (q1 << 3)) << (6 * sl);
    }
    auto launch = [&](auto ptag, auto nbtag, auto nbptag, auto nstag) {
        constexpr int PR = decltype(ptag)::value, NB = decltype(nbtag)::value, NBP = decltype(nbptag)::value;
        constexpr int NS = decltype(nstag)::value;
        using E = typename Cfg<PR>::E;
        constexpr bool H = PR == BLAST_FP16X3;
        if constexpr (H && NB <= 16) {
            // wide wave tiles (8 waves, 4 row tiles, 64 cosmologies per work-group)
            const int wgroups = (RT + kWideTR - 1) / kWideTR;
            const int wunits = p->n_chi * nBT * wgroups;
            const dim3 wg((unsigned)((wunits + 7) / 8 * 8));
            if (x.direct)
                hipLaunchKernelGGL((contract_quad_wide_kernel<PR, NB, NBP, NS, true>), wg, dim3(512), 0, s,
                                   (const uint16_t *)p->basis.n16, p->basis.nl16, p->basis.nscale16, c, nullptr, Kt,
                                   a->batch, p->n_chi, p->n_R, p->rows_pad, nBT, wunits, p->n_ell, p->nt, granges,
                                   p->n_cheb, Y);
            else
                hipLaunchKernelGGL((contract_quad_wide_kernel<PR, NB, NBP, NS, false>), wg, dim3(512), 0, s,
                                   (const uint16_t *)p->basis.h16, p->basis.l16, p->basis.scale16, c, clo, Kt,
                                   a->batch, p->n_chi, p->n_R, p->rows_pad, nBT, wunits, p->n_ell, p->nt, granges,
                                   p->n_cheb, Y);
            return;
        }
        const E *bas = PR == BLAST_FP32 ? (const E *)(nodal ? p->basis.nf32 : p->basis.f32)
                                        : (const E *)(H ? (nodal ? p->basis.n16 : p->basis.h16) : p->basis.hi);
        const uint16_t *blo = H ? (nodal ? p->basis.nl16 : p->basis.l16) : p->basis.lo;
        const float *bsc = H ? (nodal ? p->basis.nscale16 : p->basis.scale16) : p->basis.scale;
        // all LDS of the fused kernel is static (FusedShape::LDS bytes)
        hipLaunchKernelGGL((contract_quad_kernel<PR, NB, NBP, NS>), dim3(grid), dim3(256 * kFusedTR), 0, s, bas,
                           blo, bsc, (const E *)c, clo,
                           Kt, a->batch, p->n_chi, p->n_R, p->rows_pad, nBT, units, p->n_ell, p->nt, granges, Y,
                           w_out, x.direct ? p->n_cheb : p->nc_pad);
    };
    // nc_pad is a multiple of 32 up to 128: 1..4 blocks of 32 columns
    auto by_ns = [&](auto ptag, auto nbtag, auto nbptag) {
        constexpr int PR = decltype(ptag)::value;
        constexpr int S32 = PR == BLAST_FP32 ? 2 : 1;  // steps per 32 columns
        switch (p->nc_pad / 32) {
            case 1: launch(ptag, nbtag, nbptag, std::integral_constant<int, S32>()); break;
            case 2: launch(ptag, nbtag, nbptag, std::integral_constant<int, 2 * S32>()); break;
            case 3: launch(ptag, nbtag, nbptag, std::integral_constant<int, 3 * S32>()); break;
            default: launch(ptag, nbtag, nbptag, std::integral_constant<int, 4 * S32>()); break;
        }
    };
    auto by_nb = [&](auto ptag) {
        switch (nb) {
            case 4: by_ns(ptag, std::integral_constant<int, 4>(), std::integral_constant<int, 16>()); break;
            case 8: by_ns(ptag, std::integral_constant<int, 8>(), std::integral_constant<int, 16>()); break;
            case 12: by_ns(ptag, std::integral_constant<int, 12>(), std::integral_constant<int, 16>()); break;
            case 16: by_ns(ptag, std::integral_constant<int, 16>(), std::integral_constant<int, 16>()); break;
            default: by_ns(ptag, std::integral_constant<int, 20>(), std::integral_constant<int, 32>()); break;
        }
    };
    if (x.prec == BLAST_FP32) by_nb(std::integral_constant<int, BLAST_FP32>());
    if (x.prec == BLAST_BF16) by_nb(std::integral_constant<int, BLAST_BF16>());
    if (x.prec == BLAST_BF16X3) by_nb(std::integral_constant<int, BLAST_BF16X3>());
    if (x.prec == BLAST_FP16X3) by_nb(std::integral_constant<int, BLAST_FP16X3>());
}

// FP64 stages 2 + 3 fused: without w_save, at most 16 bins, batches of kFusedMinBatch or more
bool fused_f64(int nbins, int batch) { return nbins <= 16 && batch >= kFusedMinBatch; }

// the FP64 weights table Kt[a, b][beta][16] (bins past nbins zero)
void stage_r_weights64(blast_plan *p, const blast_cl_args *a, const Ctx &x, double *Kt, hipStream_t s) {
    constexpr int KB = kt_cosmologies<double>();
    dim3 gk((unsigned)((p->NP + kKtP - 1) / kKtP), (unsigned)((a->batch + KB - 1) / KB));
    hipLaunchKernelGGL(kt_kernel<double>, gk, dim3(256), 0, s, a->K_chi2, p->d_wR, (const float *)nullptr,
                       a->batch, x.nbins, 16, p->NP, p->n_R, Kt);
}

void stage_contract_quad_f64(blast_plan *p, const blast_cl_args *a, const Ctx &x, const void *c, const double *Kt,
                             double *Y, hipStream_t s) {
    const int RT = p->rows_pad / 16, nBT = (a->batch + 63) / 64;
    const int units = p->n_chi * nBT * ((RT + kF64TR - 1) / kF64TR);
    const unsigned grid = (unsigned)((units + 7) / 8 * 8);
    auto launch = [&](auto nbtag, auto kstag, auto nstag) {
        constexpr int NB = decltype(nbtag)::value, KS = decltype(kstag)::value, NSTG = decltype(nstag)::value;
        hipLaunchKernelGGL((contract_quad_f64_kernel<NB, KS, NSTG>), dim3(grid), dim3(512), 0, s,
                           x.nodal ? p->basis.nf64 : p->basis.f64,
                           (const double *)c, Kt, a->batch, p->n_chi, p->n_R, p->rows_pad, nBT, units, Y);
    };
    using I32 = std::integral_constant<int, 32>;
    using I64 = std::integral_constant<int, 64>;
    using S1 = std::integral_constant<int, 1>;
    // nc_pad is a multiple of 32 up to 128: stages of 64 columns where they divide it, else 32
    auto by_ncp = [&](auto nbtag) {
        switch (p->nc_pad / 32) {
            case 1: launch(nbtag, I32(), S1()); break;
            case 2: launch(nbtag, I64(), S1()); break;
            case 3: launch(nbtag, I32(), std::integral_constant<int, 3>()); break;
            default: launch(nbtag, I64(), std::integral_constant<int, 2>()); break;
        }
    };
    switch ((x.nbins + 3) / 4) {
        case 1: by_ncp(std::integral_constant<int, 4>()); break;
        case 2: by_ncp(std::integral_constant<int, 8>()); break;
        case 3: by_ncp(std::integral_constant<int, 12>()); break;
        default: by_ncp(std::integral_constant<int, 16>()); break;
    }
}

// stage 4: C = chi-quadrature and pair assembly
void stage_quad_c(blast_plan *p, const blast_cl_args *a, const Ctx &x, const void *Y, hipStream_t s) {
    Slots st{{p->tslot_type[0], p->tslot_type[1], p->tslot_type[2]}};
    const int nblk = (x.sel.n_out + kChiRows - 1) / kChiRows;
    dim3 g2((unsigned)(p->nt * nblk), a->batch);
    const int nc4 = (p->n_chi + 3) & ~3;
    const size_t sh2 = ((size_t)x.nbp * nc4 + 4 * (size_t)x.nbp * x.nbp) * sizeof(double);
#define BLAST_QC(YT, NB)                                                                                          \
    hipLaunchKernelGGL((quad_c_mfma_kernel<YT, NB>), g2, dim3(256), sh2, s, (const YT *)Y, a->K_chi, p->d_wchi, \
                       p->d_chi, p->d_pref, p->n_chi, p->rows_pad, p->n_ell, st, x.ng, x.ns, a->types, x.npairs,  \
                       x.sel, a->C)
    const bool f64 = x.prec == BLAST_FP64;
    if (f64 && x.nbp == 16) BLAST_QC(double, 1);
    if (f64 && x.nbp == 32) BLAST_QC(double, 2);
    if (!f64 && x.nbp == 16) BLAST_QC(float, 1);
    if (!f64 && x.nbp == 32) BLAST_QC(float, 2);
#undef BLAST_QC
}

// Device memory a call uses in place of plan-owned or caller scratch (the no-alloc entry point)
struct FixedScratch {
    unsigned char *ptr;
    size_t bytes;
};

template <typename Mark>
blast_status forward_impl(blast_plan *p, const blast_cl_args *a, hipStream_t s, Mark &mark,
                          const FixedScratch *fixed = nullptr) {
    Ctx x;
    blast_status st = check_args(p, a, x);
    if (st != BLAST_OK) return st;
    if (!a->C) return set_error("C is required"), BLAST_E_INVALID;
    if (x.prec == BLAST_FP16X3) {
        if (a->w_save) return set_error("FP16X3 runs the fused path only and cannot keep w"), BLAST_E_UNSUPPORTED;
        if (x.nbins > 20) return set_error("FP16X3 takes at most 20 bins"), BLAST_E_UNSUPPORTED;
        // nodal P: the projection's even/odd split needs n_cheb % 8 == 0; FP32 P with the FP16 nodal
        // basis (n_cheb % 4 == 0) needs no projection
        if (a->p_kind == 0 && p->n_cheb % 8 && !(a->p_dtype == 1 && p->basis.n16))
            return set_error("FP16X3 on nodal P needs n_cheb % 8 == 0, or FP32 P with n_cheb % 4 == 0"),
                   BLAST_E_UNSUPPORTED;
    }
    BLAST_HIP_TRY(allow_large_lds());
    const bool need_w = a->w_save == nullptr;
    // nodal values: the nodal basis contracted with P itself (direct): FP16X3 on FP32 P (at most
    // 16 bins; P split in the kernel), FP32 on FP32 P (P rows of n_cheb % 4 == 0 elements read in
    // place of c rows) and FP64 on FP64 P (P rows in the coefficient rows' layout: n_cheb ==
    // nc_pad).  FP32 P on FP16X3 with more bins: the nodal basis, with P
    // split as coefficient input is (conv).  The BF16 paths keep the projection: with 8 or 16 bits
    // per operand and no row scale on P, the rounding of every P_j can cost more than the
    // cancellation the nodal sum saves (BF16X3 measured both better and worse than through c)
    // P read in place of c is read in 16-byte pieces, as the library's own c buffers are (P is
    // 16-byte aligned, checked with the arguments)
    const bool fp32p = a->p_kind == 0 && a->p_dtype == 1, fp64p = a->p_kind == 0 && a->p_dtype == 0;
    const bool h16 = x.prec == BLAST_FP16X3 && p->basis.n16 && fused_nb(x.prec, x.nbins, a->batch) <= 16;
    const bool nodal = (fp32p && (h16 || (x.prec == BLAST_FP32 && p->basis.nf32 && p->n_cheb % 4 == 0))) ||
                       (fp64p && x.prec == BLAST_FP64 && p->basis.nf64);
    const bool conv = !nodal && fp32p && x.prec == BLAST_FP16X3 && p->basis.n16;
    x.nodal = nodal || conv;
    x.direct = nodal;
    const Layout L = layout_of(p, a->batch, x.prec, x.nbins, need_w, false, nodal);
    unsigned char *ws = nullptr;
    if (fixed) {
        if (L.total > fixed->bytes)
            return set_error("this call needs %zu bytes of scratch; the fixed scratch holds %zu", L.total,
                             fixed->bytes),
                   BLAST_E_UNSUPPORTED;
        ws = fixed->ptr;
    } else {
        ws = get_workspace(p, a, L.total, st);
        if (!ws) return st;
    }
    const void *c = nodal ? a->P : (const void *)(ws + L.c);
    uint16_t *clo = !nodal && (x.prec == BLAST_BF16X3 || x.prec == BLAST_FP16X3) ? (uint16_t *)(ws + L.clo) : nullptr;
    float *cs = !nodal && x.prec == BLAST_FP16X3 ? (float *)(ws + L.cs) : nullptr;
    void *w = need_w ? (void *)(ws + L.w) : a->w_save;
    void *Y = a->y_save ? a->y_save : (void *)(ws + L.y);
    const bool keep_fused = !need_w && fused_keeps_w(x.prec, x.nbins, a->batch);
    const int fnb = need_w || keep_fused ? fused_nb(x.prec, x.nbins, a->batch) : 0;
    const bool f64f = need_w && x.prec == BLAST_FP64 && fused_f64(x.nbins, a->batch);
    mark(0);
    if (conv) {
        blast_cl_args ac = *a;
        ac.p_kind = 1;  // P's nodal values are the nodal basis' coefficients
        stage_project(p, &ac, x, (void *)c, clo, cs, s);
    } else if (!nodal) {
        stage_project(p, a, x, (void *)c, clo, cs, s);
    }
    mark(1);
    if (fnb) {
        // fused path: interval 1 = the R-weights table, interval 2 = contraction + R-quadrature
        stage_r_weights(p, a, x, fnb, cs, (float *)(ws + L.kt), s);
        mark(2);
        stage_contract_quad(p, a, x, fnb, c, clo, (float *)(ws + L.kt), (float *)Y,
                            keep_fused ? (float *)a->w_save : nullptr, s);
    } else if (f64f) {
        stage_r_weights64(p, a, x, (double *)(ws + L.kt), s);
        mark(2);
        stage_contract_quad_f64(p, a, x, c, (const double *)(ws + L.kt), (double *)Y, s);
    } else {
        stage_contract(p, a, x, c, clo, w, s);
        mark(2);
        stage_quad_y(p, a, x, w, Y, s);
    }
    mark(3);
    stage_quad_c(p, a, x, Y, s);
    mark(4);
    BLAST_HIP_TRY(hipGetLastError());
    return BLAST_OK;
}

// ---------------------------------------------------------------------------------------------
// Scratch of the forward that allocates nothing: a file-scope device array.  Each GPU the library
// runs on holds its own copy, at its own address, from the time the library's code is loaded there
// until the process ends.  In host code `scratch` names a host-side stand-in, not device memory:
// kernels get the address hipGetSymbolAddress returns for the current device, taken once per
// device when a plan is made there and kept in noalloc_ptr.
// ---------------------------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
unsigned char *noalloc_ptr[kMaxDevices];
hipError_t noalloc_err[kMaxDevices];

struct NoMark {
    void operator()(int) const {}
};

}  // namespace

void noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (noalloc_ptr[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    noalloc_err[device] = e;
    if (e == hipSuccess) noalloc_ptr[device] = (unsigned char *)ptr;
}

blast_status forward_noalloc(blast_plan *p, const blast_cl_args *a, hipStream_t s) {
    if (a->workspace) return set_error("the no-alloc forward takes no workspace (its scratch is fixed)"), BLAST_E_INVALID;
    FixedScratch fx{nullptr, kNoAllocScratchBytes};
    {
        std::lock_guard<std::mutex> lk(noalloc_mu);
        if (p->device >= 0 && p->device < kMaxDevices) fx.ptr = noalloc_ptr[p->device];
        if (!fx.ptr)
            return set_error("no fixed scratch on device %d: %s", p->device,
                             p->device >= 0 && p->device < kMaxDevices ? hipGetErrorString(noalloc_err[p->device])
                                                                       : "device index out of range"),
                   BLAST_E_HIP;
    }
    NoMark mark;
    return forward_impl(p, a, s, mark, &fx);
}

size_t workspace_bytes(const blast_plan *p, int batch, int prec, int n_bins) {
    return workspace_bytes_impl(p, batch, prec, n_bins);
}

size_t forward_workspace_bytes(const blast_plan *p, int batch, int prec, int n_bins) {
    return layout_of(p, batch, prec, n_bins, true, false).total;
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

blast_status backward(blast_plan *p, const blast_cl_args *a, const double *dC, void *dP, double *dK_chi,
                      double *dK_chi2, hipStream_t s) {
    Ctx x;
    blast_status st = check_args(p, a, x);
    if (st != BLAST_OK) return st;
    if (x.prec != BLAST_FP64 && x.prec != BLAST_FP32)
        return set_error("the adjoint runs in FP64 or FP32"), BLAST_E_UNSUPPORTED;
    // adj_w_kernel keeps the R weights and dY of one chi node in LDS
    if (((size_t)p->n_R * x.nbp + (size_t)p->rows_pad * (x.nbp + 1)) * sizeof(double) > 160 * 1024)
        return set_error("n_R and the multipoles too large for the adjoint's R tile"), BLAST_E_UNSUPPORTED;
    if (!dC) return set_error("dC is required"), BLAST_E_INVALID;
    if ((uintptr_t)dP & 15) return set_error("dP must be 16-byte aligned"), BLAST_E_INVALID;
    const bool f64 = x.prec == BLAST_FP64;
    // the transposed contraction keeps the dw rows of a tile of 32 cosmologies in LDS
    if (dP && (size_t)kAdjBT * (f64 ? (size_t)(p->rows_pad + 1) * 8 : (size_t)(p->rows_pad + 4) * 4) > 160 * 1024)
        return set_error("the multipoles are too many for the transposed contraction's tile (dP)"),
               BLAST_E_UNSUPPORTED;
    BLAST_HIP_TRY(allow_large_lds());
    // Y of a forward call with the same inputs, when the caller kept it
    const bool have_y = a->y_save != nullptr;
    // w is read only for dK_chi2, and for dK_chi when Y has to be summed again: a backward that
    // asks for neither (dP alone, or dK_chi with Y kept) never recomputes it
    const bool use_w = dK_chi2 != nullptr || (dK_chi != nullptr && !have_y);
    const bool make_w = a->w_save == nullptr && use_w;
    const Layout L = layout_of(p, a->batch, x.prec, x.nbins, make_w, true);
    unsigned char *ws = get_workspace(p, a, L.total, st);
    if (!ws) return st;
    void *c = ws + L.c;
    void *w = a->w_save ? a->w_save : (make_w ? (void *)(ws + L.w) : nullptr);
    void *Y = have_y ? a->y_save : (void *)(ws + L.y), *dY = ws + L.dy, *dw = ws + L.dw, *dc = ws + L.dc;
    double *Sg = (double *)(ws + L.sg);
    if (make_w) {
        stage_project(p, a, x, c, nullptr, nullptr, s);
        stage_contract(p, a, x, c, nullptr, w, s);
    }
    if (dK_chi && !have_y) stage_quad_y(p, a, x, w, Y, s);
    Slots sl{{p->tslot_type[0], p->tslot_type[1], p->tslot_type[2]}};
    dim3 g1((unsigned)(p->nt * p->n_ell), a->batch);
#define BLAST_ADJ(T, NB)                                                                                          \
    do {                                                                                                          \
        const size_t shd = (size_t)kAdjRG * NB * NB * 8 + (size_t)((p->n_chi + 15) / 16 * 16) * (NB + 4) * 4;     \
        if (std::is_same<T, float>::value && shd <= 160 * 1024)                                                  \
            hipLaunchKernelGGL((adj_dy_mfma_kernel<NB>), dim3((unsigned)((p->rows + kAdjRG - 1) / kAdjRG), a->batch), \
                               dim3(256), shd, s, dC, a->K_chi, p->d_wchi, p->d_chi, p->d_pref, p->n_chi, p->rows, \
                               p->rows_pad, p->n_ell, sl, x.ng, x.ns, a->types, x.npairs, x.sel.n_out, x.inv,    \
                               (float *)dY, Sg);                                                                \
        else                                                                                                      \
            hipLaunchKernelGGL((adj_dy_kernel<T, NB>), g1, dim3(256), 0, s, dC, a->K_chi, p->d_wchi, p->d_chi,    \
                               p->d_pref, p->n_chi, p->rows_pad, p->n_ell, sl, x.ng, x.ns, a->types, x.npairs,    \
                               x.sel.n_out, x.inv, (T *)dY, Sg);                                                  \
        if (dK_chi) {                                                                                             \
            dim3 gk((unsigned)((p->n_chi + 63) / 64), a->batch);                                                  \
            hipLaunchKernelGGL((adj_kchi_kernel<T, NB>), gk, dim3(256), 0, s, (const T *)Y, Sg, p->d_wchi,        \
                               p->d_chi, p->n_chi, p->rows, p->rows_pad, x.nbins, dK_chi);                        \
        }                                                                                                         \
        dim3 gw(p->n_chi, a->batch);                                                                              \
        if constexpr (std::is_same<T, float>::value) {                                                           \
            const size_t shw = ((size_t)((p->n_R + 15) / 16 * 16) * NB + (size_t)NB * (p->rows_pad + 4)) * 4;    \
            hipLaunchKernelGGL((adj_w_mfma_kernel<NB>), gw, dim3(256), shw, s, (const float *)dY,               \
                               (const float *)w, a->K_chi2, p->d_wR, p->NP, p->n_R, p->n_chi, p->rows,          \
                               p->rows_pad, x.nbins, (float *)dw, dK_chi2);                                     \
        } else {                                                                                                  \
            const size_t shw = ((size_t)p->n_R * NB + (size_t)p->rows_pad * adj_w_stride<NB>()) * sizeof(double); \
            hipLaunchKernelGGL((adj_w_kernel<T, NB>), gw, dim3(256), shw, s, (const T *)dY, (const T *)w,       \
                               a->K_chi2, p->d_wR, p->NP, p->n_R, p->n_chi, p->rows, p->rows_pad, x.nbins,      \
                               (T *)dw, dK_chi2);                                                               \
        }                                                                                                         \
    } while (0)
    if (f64 && x.nbp == 16) BLAST_ADJ(double, 16);
    if (f64 && x.nbp == 32) BLAST_ADJ(double, 32);
    if (!f64 && x.nbp == 16) BLAST_ADJ(float, 16);
    if (!f64 && x.nbp == 32) BLAST_ADJ(float, 32);
#undef BLAST_ADJ
    if (dP) {
        const dim3 gt = point_tile_grid(p->NP, (a->batch + kAdjBT - 1) / kAdjBT);
        // nodal P of the path's own type with n_cheb == nc_pad: dP = B^T dw with the nodal basis
        // B = Ttilde D (the adjoint of the projection folded in), written straight into dP
        const bool ndp = a->p_kind == 0 && p->n_cheb == p->nc_pad &&
                         (f64 ? a->p_dtype == 0 && p->basis.nf64 : a->p_dtype == 1 && p->basis.nf32);
        void *dcn = ndp ? dP : dc;
        if (f64) {
            const size_t sht = (size_t)kAdjBT * (p->rows_pad + 1) * 8;
            hipLaunchKernelGGL((contract_t_kernel<true>), gt, dim3(256), sht, s, ndp ? p->basis.nf64 : p->basis.f64,
                               (const double *)dw, a->batch, p->NP, p->rows_pad, p->nc_pad, (double *)dcn);
        } else {
            // dc = Ttilde^T dw is the forward contraction's product with the transposed basis (rows of
            // Ttilde^T: the nc_pad Chebyshev columns; its K: the rows_pad basis rows) and dw in place of c
            {
                std::lock_guard<std::mutex> lk(p->mu);
                st = ndp ? ensure_nf32t(p, s) : ensure_f32t(p, s);
            }
            if (st != BLAST_OK) return st;
            const float *bt = ndp ? p->basis.nf32t : p->basis.f32t;
            const int RT = p->nc_pad / 16;
            const size_t sh64 = (size_t)2 * kAdjBT * (p->rows_pad + 4) * sizeof(float);
            if (sh64 <= 160 * 1024) {
                // 64 cosmologies per work-group and one row tile per wave: each basis tile read from
                // L2 feeds twice the MFMAs of the 32-cosmology tile
                const dim3 g64 = point_tile_grid(p->NP, (a->batch + 2 * kAdjBT - 1) / (2 * kAdjBT));
                hipLaunchKernelGGL((contract_tiled_kernel<BLAST_FP32, 4, 2 * kAdjBT, 1>), g64, dim3(64 * RT), sh64,
                                   s, bt, nullptr, nullptr, (const float *)dw, nullptr, a->batch, p->NP, p->nc_pad,
                                   p->rows_pad, (float *)dcn, p->rows_pad);
            } else {
                const int W = std::min((RT + kTilesPerWave - 1) / kTilesPerWave, 8);
                const size_t sht = (size_t)kAdjBT * (p->rows_pad + 4) * sizeof(float);
                hipLaunchKernelGGL((contract_tiled_kernel<BLAST_FP32, 4, kAdjBT>), gt, dim3(64 * W), sht, s, bt,
                                   nullptr, nullptr, (const float *)dw, nullptr, a->batch, p->NP, p->nc_pad,
                                   p->rows_pad, (float *)dcn, p->rows_pad);
            }
        }
        if (ndp) {
            BLAST_HIP_TRY(hipGetLastError());
            return BLAST_OK;
        }
        const long nrows = (long)a->batch * p->NP;
        const int N = p->n_cheb;
        if (a->p_kind == 0 && N % 8 == 0) {
            const int nt = (N / 2 + 15) / 16;  // 1..4 tiles of 16 per parity
            auto launch = [&](auto ptag, auto nttag) {
                using PT = typename decltype(ptag)::type;
                constexpr int NT = decltype(nttag)::value;
                if (f64)
                    hipLaunchKernelGGL((adj_project_split64_kernel<PT, NT>), dim3((unsigned)((nrows + 63) / 64)),
                                       dim3(256), (size_t)2 * 16 * NT * (16 * NT + 2) * sizeof(double), s,
                                       (const double *)dc, p->d_dctn64, N, p->nc_pad, nrows, (PT *)dP);
                else
                    hipLaunchKernelGGL((adj_project_split_kernel<PT, NT>), dim3((unsigned)((nrows + 127) / 128)),
                                       dim3(256), (size_t)2 * 16 * NT * (16 * NT + 4) * sizeof(float), s,
                                       (const float *)dc, p->d_dctn32, N, p->nc_pad, nrows, (PT *)dP);
            };
            auto by_nt = [&](auto ptag) {
                switch (nt) {
                    case 1: launch(ptag, std::integral_constant<int, 1>()); break;
                    case 2: launch(ptag, std::integral_constant<int, 2>()); break;
                    case 3: launch(ptag, std::integral_constant<int, 3>()); break;
                    default: launch(ptag, std::integral_constant<int, 4>()); break;
                }
            };
            if (a->p_dtype == 0) by_nt(TypeTag<double>());
            else by_nt(TypeTag<float>());
        } else {
            dim3 gp((unsigned)((nrows + kAdjRows - 1) / kAdjRows));
#define BLAST_AP(T, PT)                                                                                        \
    hipLaunchKernelGGL((adj_project_kernel<T, PT>), gp, dim3(256), 0, s, (const T *)dc, p->d_dctn64, p->n_cheb, \
                       p->nc_pad, nrows, a->p_kind, (PT *)dP)
            if (f64 && a->p_dtype == 0) BLAST_AP(double, double);
            if (f64 && a->p_dtype == 1) BLAST_AP(double, float);
            if (!f64 && a->p_dtype == 0) BLAST_AP(float, double);
            if (!f64 && a->p_dtype == 1) BLAST_AP(float, float);
#undef BLAST_AP
        }
    }
    BLAST_HIP_TRY(hipGetLastError());
    return BLAST_OK;
}

}  // namespace blast
