// Internal declarations of the beyond-Limber C_ell library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "blast_hip.h"

namespace blast {

void set_error(const char *fmt, ...);
void clear_error();

constexpr int kMaxBins = 32;     // n_g + n_s per call
constexpr int kMaxEll = 512;     // multipoles per plan
constexpr int kMaxCheb = 128;    // Chebyshev nodes per plan
constexpr int kBatchTile = 64;   // cosmologies per contraction work-group pass

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Reduced-precision basis copies (FP32, BF16 hi/lo) are stored per (chi_a, R_b) point in the
// register image of the contraction's MFMA A operand: 16-row tiles, steps of KSTEP = 4*VEC
// columns, and inside one (tile, step) the 16-byte vectors of the 64 lanes in lane order
// (lane = row % 16 + 16 * ((n % KSTEP) / VEC)), so that each load of a tile is 1 KB contiguous.
// VEC = 16 bytes / element size; nsteps = nc_pad / KSTEP.  Returns the element offset of
// (row, n) inside the point's rows_pad * nc_pad block.
__host__ __device__ inline size_t tiled_off(int row, int n, int nsteps, int VEC) {
    const int KSTEP = 4 * VEC;
    const int lane = (row & 15) + 16 * ((n % KSTEP) / VEC);
    return (((size_t)(row >> 4) * nsteps + n / KSTEP) * 64 + lane) * VEC + n % VEC;
}

// FP16 hi + lo copy of the projection matrix used by the FP16X3 projection, in the register order
// of the B operand of v_mfma_f32_16x16x32_f16.  With NT = nc_pad / 32 output tiles of 16 per parity
// and NK = (NT + 1) / 2 steps of 32 columns, entry (parity p, tile t, step k, part hl, lane L) is
// 8 halves: element e is 2^g D[2 (16 t + L % 16) + p][32 k + 8 (L / 16) + e], zero for columns
// j >= n_cheb / 2 and rows n >= n_cheb (D[n][j] = the DCT-II matrix entry of c_n and P_j, whose
// rows have the parity symmetry D[n][N-1-j] = (-1)^n D[n][j]), hi = fp16(x) and lo = fp16(x - hi).
// g = dct16_exp(n_cheb) puts the largest |2^g D| in [2^14, 2^15).  Returns the offset in halves.
__host__ __device__ inline size_t dct16_off(int p, int t, int k, int hl, int lane, int NT, int NK) {
    return (((((size_t)p * NT + t) * NK + k) * 2 + hl) * 64 + lane) * 8;
}
inline int dct16_exp(int N) { return 14 - std::ilogb(2.0 / N); }

// Power-of-two scale and the BF16 bit pattern helpers shared by host conversions.
struct BasisBuffers {
    double *f64 = nullptr;     // [NP][rows_pad][nc_pad]
    float *f32 = nullptr;      // [NP][rows_pad][nc_pad]
    uint16_t *hi = nullptr;    // BF16 bits of (value / scale), same layout
    uint16_t *lo = nullptr;    // BF16 bits of the remainder
    float *scale = nullptr;    // [NP][rows_pad] power-of-two row scales
    uint16_t *h16 = nullptr;   // FP16 bits of (value / scale16), tiled layout
    uint16_t *l16 = nullptr;   // FP16 bits of the remainder
    float *scale16 = nullptr;  // [NP][rows_pad] power-of-two row scales of the FP16 parts
    // the nodal basis B = Ttilde D (D: the DCT-II matrix taking nodal P to Chebyshev coefficients),
    // split the same way: sum_j B[row][j] P_j = sum_n Ttilde[row][n] c_n, contracted with P itself
    uint16_t *n16 = nullptr;   // FP16 bits of (B / nscale16), tiled layout (column = k node)
    uint16_t *nl16 = nullptr;  // FP16 bits of the remainder
    float *nscale16 = nullptr; // [NP][rows_pad]
    float *nf32 = nullptr;     // FP32 nodal basis, layout of f32 (plans with n_cheb % 4 == 0)
    double *nf64 = nullptr;    // FP64 nodal basis, layout of f64 (plans with n_cheb == nc_pad)
    float *nf32t = nullptr;    // FP32 nodal basis transposed, layout of f32t (made by the first FP32
                               // adjoint on nodal FP32 P that asks for dP)
    float *f32t = nullptr;     // FP32 transpose per point, [nc_pad][rows_pad] in the tiled layout
                               // (made by the first FP32 adjoint call that asks for dP)
};

}  // namespace blast

struct blast_plan {
    int device = 0;
    // multipoles and types
    int n_ell = 0;
    std::vector<double> ell;   // multipoles (any real values >= 2)
    bool int_ell = true;       // every multipole is an integer
    uint32_t types = 0;
    int nt = 0;              // number of resident types
    int slot[3] = {-1, -1, -1};  // slot of gg, gs, ss rows (or -1)
    int tslot_type[3] = {0, 0, 0}; // type bit of each slot
    int rows = 0, rows_pad = 0;
    // grids
    int n_chi = 0, n_R = 0, NP = 0;
    std::vector<double> chi, w_chi, R, w_R;
    double kmin = 0, kmax = 0;
    int n_cheb = 0, nc_pad = 0;
    std::vector<double> knodes;
    // quadrature of the basis
    int kq_panels = 0;
    double kq_phase = 0;
    int64_t kq_nodes = 0;
    double build_ms = 0;
    uint32_t precisions = 0;
    // device data
    blast::BasisBuffers basis;
    double *d_dct64 = nullptr;  // projection matrix, transposed: [n_cheb j][nc_pad n]
    float *d_dct32 = nullptr;
    double *d_dctn64 = nullptr; // projection matrix [nc_pad n][n_cheb j] (MFMA path)
    float *d_dctn32 = nullptr;
    uint16_t *d_dct16 = nullptr;  // FP16 hi + lo operand table of the FP16X3 projection (dct16_off)
    double *d_chi = nullptr, *d_wchi = nullptr, *d_wR = nullptr;
    double *d_pref = nullptr;   // [rows] N_t(l)
    double *d_ell = nullptr;    // [n_ell] multipoles
    int *d_elli = nullptr;      // [n_ell] the same as integers (integer plans only)
    // stage timing: 5 events per recorded forward call
    bool profile = false;
    std::vector<hipEvent_t> prof_events;
    // plan-owned scratch for calls without a caller workspace
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    // Limber path: 5-node stencils for the second and third derivative at each chi node
    // (weights [n_chi][2][5], first node [n_chi]; absent when n_chi < 5) and its own scratch
    double *d_fd = nullptr;
    int *d_fds = nullptr;
    void *limb_ws = nullptr;
    size_t limb_ws_bytes = 0;
    std::mutex mu;
};

namespace blast {

// basis.hip
blast_status build_basis(blast_plan *p, hipStream_t s);
blast_status derive_precisions(blast_plan *p, hipStream_t s);
// the transposed FP32 copy of the basis, made on `s` if it does not exist yet (caller holds p->mu)
blast_status ensure_f32t(blast_plan *p, hipStream_t s);
// the transposed FP32 nodal basis, likewise (plans with n_cheb == nc_pad)
blast_status ensure_nf32t(blast_plan *p, hipStream_t s);

// eval.hip
blast_status forward(blast_plan *p, const blast_cl_args *a, hipStream_t s);
blast_status backward(blast_plan *p, const blast_cl_args *a, const double *dC, void *dP, double *dK_chi,
                      double *dK_chi2, hipStream_t s);
size_t workspace_bytes(const blast_plan *p, int batch, int prec, int n_bins);
// scratch of a forward call alone (no w_save), the part the server reserves per launch
size_t forward_workspace_bytes(const blast_plan *p, int batch, int prec, int n_bins);
// the forward that allocates nothing: its scratch is a fixed device array, whose address on a
// device noalloc_init (called with that device current, when a plan is made there) looks up once
void noalloc_init(int device);
blast_status forward_noalloc(blast_plan *p, const blast_cl_args *a, hipStream_t s);

// limber.hip
blast_status limber(blast_plan *p, const blast_limber_args *a, hipStream_t s);

}  // namespace blast

#define BLAST_HIP_TRY(expr)                                                                          \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            blast::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
            return BLAST_E_HIP;                                                                      \
        }                                                                                            \
    } while (0)
