// C ABI entry points: errors, grids, plan lifetime, forward dispatch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <algorithm>
#include <cstdio>

#include "internal.h"

namespace {
thread_local char g_err[1024] = "";

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

const double kPi = 3.141592653589793238462643383279502884;
}  // namespace

namespace blast {
void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = 0; }
}  // namespace blast

extern "C" const char *blast_last_error(void) { return g_err; }
extern "C" const char *blast_version(void) { return "blast-hip 0.1 (gfx950)"; }

// --------------------------------------------------------------------------------------------
// grids
// --------------------------------------------------------------------------------------------

extern "C" blast_status blast_grid_chi_simpson(int32_t n, double lo, double hi, double *chi, double *w) {
    if (n < 4 || !(hi > lo) || !chi || !w) {
        blast::set_error("blast_grid_chi_simpson: need n >= 4 and hi > lo");
        return BLAST_E_INVALID;
    }
    const double h = (hi - lo) / (n - 1);
    for (int i = 0; i < n; ++i) {
        chi[i] = lo + i * h;
        w[i] = 0.0;
    }
    // panels of two intervals (1/3 rule) while more than three intervals remain odd
    int intervals = n - 1;
    int start = 0;
    if (intervals % 2 == 1) {
        // three-interval 3/8 panel at the end
        const int s = n - 4;
        const double c = 3.0 * h / 8.0;
        w[s] += c;
        w[s + 1] += 3.0 * c;
        w[s + 2] += 3.0 * c;
        w[s + 3] += c;
        intervals -= 3;
    }
    for (int p = 0; p < intervals / 2; ++p) {
        const int s = start + 2 * p;
        w[s] += h / 3.0;
        w[s + 1] += 4.0 * h / 3.0;
        w[s + 2] += h / 3.0;
    }
    return BLAST_OK;
}

extern "C" blast_status blast_grid_R_fejer(int32_t n, double R_min, double *R, double *w) {
    if (n < 1 || !(R_min >= 0.0 && R_min < 1.0) || !R || !w) {
        blast::set_error("blast_grid_R_fejer: need n >= 1 and 0 <= R_min < 1");
        return BLAST_E_INVALID;
    }
    const double half = 0.5 * (1.0 - R_min);
    for (int i = 0; i < n; ++i) {
        // ascending order: node i is the first-kind point with angle pi - (2i+1)pi/2n
        const double th = kPi - (2.0 * i + 1.0) * kPi / (2.0 * n);
        double acc = 1.0;
        for (int m = 1; 2 * m <= n; ++m) acc -= 2.0 * std::cos(2.0 * m * th) / (4.0 * m * m - 1.0);
        R[i] = R_min + half * (1.0 + std::cos(th));
        w[i] = half * 2.0 / n * acc;
    }
    return BLAST_OK;
}

extern "C" blast_status blast_grid_k_cheb(int32_t n, double k_min, double k_max, double *k) {
    if (n < 1 || !(k_min > 0.0) || !(k_max > k_min) || !k) {
        blast::set_error("blast_grid_k_cheb: need n >= 1 and 0 < k_min < k_max");
        return BLAST_E_INVALID;
    }
    const double l0 = std::log(k_min), span = std::log(k_max) - std::log(k_min);
    for (int i = 0; i < n; ++i) {
        const double x = std::cos(kPi - (2.0 * i + 1.0) * kPi / (2.0 * n));
        k[i] = std::exp(l0 + 0.5 * (x + 1.0) * span);
    }
    return BLAST_OK;
}

// --------------------------------------------------------------------------------------------
// plan
// --------------------------------------------------------------------------------------------

// N_t(l) for real l (the factorial ratio continues as Gamma(l+3)/Gamma(l-1) = (l+2)(l+1)l(l-1))
static double prefactor(int type_bit, double l) {
    const double L = l;
    const double r = (L + 2.0) * (L + 1.0) * L * (L - 1.0);  // (l+2)!/(l-2)!
    if (type_bit == BLAST_GG) return 2.0 / kPi;
    if (type_bit == BLAST_GS) return 2.0 / kPi * std::sqrt(r);
    return 2.0 / kPi * r;
}

static void free_plan(blast_plan *p) {
    if (!p) return;
    auto f = [](void *q) {
        if (q) (void)hipFree(q);
    };
    f(p->basis.f64);
    f(p->basis.f32);
    f(p->basis.hi);
    f(p->basis.lo);
    f(p->basis.scale);
    f(p->basis.h16);
    f(p->basis.l16);
    f(p->basis.scale16);
    f(p->basis.n16);
    f(p->basis.nl16);
    f(p->basis.nscale16);
    f(p->basis.nf32);
    f(p->basis.nf64);
    f(p->basis.nf32t);
    f(p->basis.f32t);
    f(p->d_dct64);
    f(p->d_dct32);
    f(p->d_dctn64);
    f(p->d_dctn32);
    f(p->d_dct16);
    f(p->d_chi);
    f(p->d_wchi);
    f(p->d_wR);
    f(p->d_pref);
    f(p->d_ell);
    f(p->d_elli);
    f(p->scratch);
    f(p->d_fd);
    f(p->d_fds);
    f(p->limb_ws);
    for (hipEvent_t e : p->prof_events) (void)hipEventDestroy(e);
    delete p;
}

static blast_status validate_desc(const blast_plan_desc *d) {
    if (!d) return blast::set_error("blast_plan_create: desc is NULL"), BLAST_E_INVALID;
    if (d->n_ell < 1 || d->n_ell > blast::kMaxEll || !d->ell)
        return blast::set_error("n_ell must be in [1, %d]", blast::kMaxEll), BLAST_E_INVALID;
    for (int i = 0; i < d->n_ell; ++i) {
        if (!(d->ell[i] >= 2.0 && d->ell[i] <= 4096.0))
            return blast::set_error("ell[%d] = %g outside [2, 4096]", i, d->ell[i]), BLAST_E_INVALID;
        if (i && d->ell[i] <= d->ell[i - 1])
            return blast::set_error("ell must be strictly increasing (index %d)", i), BLAST_E_INVALID;
    }
    if (d->n_chi < 1 || !d->chi || !d->w_chi) return blast::set_error("bad chi grid"), BLAST_E_INVALID;
    for (int i = 0; i < d->n_chi; ++i)
        if (!(d->chi[i] > 0.0) || !std::isfinite(d->chi[i]) || !std::isfinite(d->w_chi[i]))
            return blast::set_error("chi[%d] must be positive and finite", i), BLAST_E_INVALID;
    if (d->n_R < 1 || !d->R || !d->w_R) return blast::set_error("bad R grid"), BLAST_E_INVALID;
    for (int i = 0; i < d->n_R; ++i)
        if (!(d->R[i] > 0.0 && d->R[i] <= 1.0) || !std::isfinite(d->w_R[i]))
            return blast::set_error("R[%d] must lie in (0, 1]", i), BLAST_E_INVALID;
    if (!(d->k_min > 0.0) || !(d->k_max > d->k_min) || !std::isfinite(d->k_max))
        return blast::set_error("need 0 < k_min < k_max"), BLAST_E_INVALID;
    if (d->n_cheb < 2 || d->n_cheb > blast::kMaxCheb)
        return blast::set_error("n_cheb must be in [2, %d]", blast::kMaxCheb), BLAST_E_INVALID;
    if (d->types == 0 || (d->types & ~7u)) return blast::set_error("types must be a non-empty subset of 7"), BLAST_E_INVALID;
    if (d->precisions & ~31u) return blast::set_error("unknown precision bits"), BLAST_E_INVALID;
    if (d->kq_panels < 0 || d->kq_panels > 4096) return blast::set_error("kq_panels out of range"), BLAST_E_INVALID;
    if (d->kq_phase < 0 || !std::isfinite(d->kq_phase)) return blast::set_error("kq_phase must be >= 0"), BLAST_E_INVALID;
    return BLAST_OK;
}

// Second and third derivative at every chi node from the 5 nearest nodes (the first / last
// five at the two ends): Fornberg's recursion (Math. Comp. 51 (1988) 699) for the weights of
// the derivatives at z of the polynomial through the stencil.  fd[a][m-2][q], m = 2, 3.
static void derivative_stencils(const std::vector<double> &x, std::vector<double> &fd, std::vector<int> &fds) {
    const int n = (int)x.size(), S = 5, M = 3;
    fd.assign((size_t)n * 2 * S, 0.0);
    fds.assign(n, 0);
    for (int a = 0; a < n; ++a) {
        const int s0 = std::min(std::max(a - 2, 0), n - S);
        fds[a] = s0;
        const double z = x[a];
        double c[S][M + 1] = {};
        double c1 = 1.0, c4 = x[s0] - z;
        c[0][0] = 1.0;
        for (int i = 1; i < S; ++i) {
            const int mn = std::min(i, M);
            double c2 = 1.0;
            const double c5 = c4;
            c4 = x[s0 + i] - z;
            for (int j = 0; j < i; ++j) {
                const double c3 = x[s0 + i] - x[s0 + j];
                c2 *= c3;
                if (j == i - 1) {
                    for (int k = mn; k >= 1; --k) c[i][k] = c1 * (k * c[i - 1][k - 1] - c5 * c[i - 1][k]) / c2;
                    c[i][0] = -c1 * c5 * c[i - 1][0] / c2;
                }
                for (int k = mn; k >= 1; --k) c[j][k] = (c4 * c[j][k] - k * c[j][k - 1]) / c3;
                c[j][0] = c4 * c[j][0] / c3;
            }
            c1 = c2;
        }
        for (int q = 0; q < S; ++q) {
            fd[((size_t)a * 2 + 0) * S + q] = c[q][2];
            fd[((size_t)a * 2 + 1) * S + q] = c[q][3];
        }
    }
}

// the basis comes either from the device precompute or from a saved file (reader != nullptr)
typedef blast_status (*BasisReader)(blast_plan *p, void *ctx);

static blast_status plan_create_impl(const blast_plan_desc *d, int32_t device, BasisReader reader, void *rctx,
                                     blast_plan **out) {
    if (!out) return blast::set_error("out is NULL"), BLAST_E_INVALID;
    *out = nullptr;
    blast_status st = validate_desc(d);
    if (st != BLAST_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return blast::set_error("device %d not available (%d devices)", device, ndev), BLAST_E_INVALID;

    blast_plan *p = new (std::nothrow) blast_plan();
    if (!p) return blast::set_error("host allocation failed"), BLAST_E_OOM;
    p->device = device;
    p->n_ell = d->n_ell;
    p->ell.assign(d->ell, d->ell + d->n_ell);
    for (double l : p->ell) p->int_ell = p->int_ell && l == std::floor(l);
    p->types = d->types;
    const int bits[3] = {BLAST_GG, BLAST_GS, BLAST_SS};
    for (int t = 0; t < 3; ++t)
        if (d->types & bits[t]) {
            p->slot[t] = p->nt;
            p->tslot_type[p->nt] = bits[t];
            p->nt++;
        }
    p->rows = p->nt * p->n_ell;
    p->rows_pad = blast::round_up(p->rows, 16);
    p->n_chi = d->n_chi;
    p->n_R = d->n_R;
    p->NP = d->n_chi * d->n_R;
    p->chi.assign(d->chi, d->chi + d->n_chi);
    p->w_chi.assign(d->w_chi, d->w_chi + d->n_chi);
    p->R.assign(d->R, d->R + d->n_R);
    p->w_R.assign(d->w_R, d->w_R + d->n_R);
    p->kmin = d->k_min;
    p->kmax = d->k_max;
    p->n_cheb = d->n_cheb;
    p->nc_pad = blast::round_up(d->n_cheb, 32);
    p->knodes.resize(d->n_cheb);
    blast_grid_k_cheb(d->n_cheb, d->k_min, d->k_max, p->knodes.data());
    p->kq_panels = d->kq_panels ? d->kq_panels : d->n_cheb;
    p->kq_phase = d->kq_phase > 0 ? d->kq_phase : 8.0;
    p->precisions = d->precisions | 1u;

    DeviceGuard guard(device);
    blast::noalloc_init(device);  // once per device: the fixed scratch of blast_cl_forward_noalloc
    hipStream_t s = nullptr;
    auto fail = [&](blast_status e) {
        if (s) (void)hipStreamDestroy(s);
        free_plan(p);
        return e;
    };
    if (hipStreamCreate(&s) != hipSuccess) return blast::set_error("hipStreamCreate failed"), fail(BLAST_E_HIP);

    // small device tables
    {
        const int N = p->n_cheb, ncp = p->nc_pad;
        std::vector<double> dct((size_t)N * ncp, 0.0), dctn((size_t)ncp * N, 0.0);
        std::vector<float> dct32((size_t)N * ncp, 0.0f), dctn32((size_t)ncp * N, 0.0f);
        // c_n = sum_j D[n][j] P_j with j the ascending-k node index (node angle pi - (2j+1)pi/2N):
        // D[n][j] = (2 - delta_n0)/N cos(n (pi - (2j+1)pi/2N))
        for (int j = 0; j < N; ++j)
            for (int n = 0; n < N; ++n) {
                double v = (n == 0 ? 1.0 : 2.0) / N * std::cos(n * (kPi - (2.0 * j + 1.0) * kPi / (2.0 * N)));
                dct[(size_t)j * ncp + n] = v;
                dct32[(size_t)j * ncp + n] = (float)v;
                dctn[(size_t)n * N + j] = v;
                dctn32[(size_t)n * N + j] = (float)v;
            }
        std::vector<double> pref(p->rows);
        for (int sl = 0; sl < p->nt; ++sl)
            for (int l = 0; l < p->n_ell; ++l) pref[sl * p->n_ell + l] = prefactor(p->tslot_type[sl], p->ell[l]);
        auto up = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
            hipError_t e = hipMalloc(dst, bytes);
            if (e != hipSuccess) return e;
            return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        };
        hipError_t e = hipSuccess;
        if (e == hipSuccess) e = up((void **)&p->d_dct64, dct.data(), dct.size() * sizeof(double));
        if (e == hipSuccess) e = up((void **)&p->d_dct32, dct32.data(), dct32.size() * sizeof(float));
        if (e == hipSuccess) e = up((void **)&p->d_dctn64, dctn.data(), dctn.size() * sizeof(double));
        if (e == hipSuccess) e = up((void **)&p->d_dctn32, dctn32.data(), dctn32.size() * sizeof(float));
        if (e == hipSuccess) e = up((void **)&p->d_chi, p->chi.data(), p->n_chi * sizeof(double));
        if (e == hipSuccess) e = up((void **)&p->d_wchi, p->w_chi.data(), p->n_chi * sizeof(double));
        if (e == hipSuccess) e = up((void **)&p->d_wR, p->w_R.data(), p->n_R * sizeof(double));
        if (e == hipSuccess) e = up((void **)&p->d_pref, pref.data(), pref.size() * sizeof(double));
        if (e == hipSuccess) e = up((void **)&p->d_ell, p->ell.data(), p->n_ell * sizeof(double));
        if (e == hipSuccess && p->int_ell) {
            std::vector<int> li(p->ell.begin(), p->ell.end());
            e = up((void **)&p->d_elli, li.data(), li.size() * sizeof(int));
        }
        if (e == hipSuccess && p->n_chi >= 5) {
            std::vector<double> fd;
            std::vector<int> fds;
            derivative_stencils(p->chi, fd, fds);
            e = up((void **)&p->d_fd, fd.data(), fd.size() * sizeof(double));
            if (e == hipSuccess) e = up((void **)&p->d_fds, fds.data(), fds.size() * sizeof(int));
        }
        if (e != hipSuccess) {
            blast::set_error("device tables: %s", hipGetErrorString(e));
            return fail(e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP);
        }
    }

    auto t0 = std::chrono::steady_clock::now();
    st = reader ? reader(p, rctx) : blast::build_basis(p, s);
    if (st == BLAST_OK) st = blast::derive_precisions(p, s);
    if (st == BLAST_OK && hipStreamSynchronize(s) != hipSuccess) {
        blast::set_error("basis build failed on the device");
        st = BLAST_E_HIP;
    }
    if (st != BLAST_OK) return fail(st);
    p->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    (void)hipStreamDestroy(s);
    *out = p;
    return BLAST_OK;
}

extern "C" blast_status blast_plan_create(const blast_plan_desc *d, int32_t device, blast_plan **out) {
    blast::clear_error();
    return plan_create_impl(d, device, nullptr, nullptr, out);
}

// --------------------------------------------------------------------------------------------
// persistence of the basis
// --------------------------------------------------------------------------------------------

namespace {
const char kMagic[8] = {'B', 'L', 'A', 'S', 'T', 'P', 'L', '1'};
const uint32_t kFileVersion = 2;  // 2: multipoles stored as FP64

// 64-bit word-wise FNV-1a style hash (tail bytes folded one by one)
struct Hash64 {
    uint64_t h = 1469598103934665603ull;
    void add(const void *data, size_t n) {
        const unsigned char *c = (const unsigned char *)data;
        size_t i = 0;
        for (; i + 8 <= n; i += 8) {
            uint64_t w;
            std::memcpy(&w, c + i, 8);
            h = (h ^ w) * 1099511628211ull;
        }
        for (; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    }
};

struct Writer {
    FILE *f;
    Hash64 hs;
    bool ok = true;
    void put(const void *d, size_t n) {
        if (ok && n && fwrite(d, 1, n, f) != n) ok = false;
        hs.add(d, n);
    }
};

struct Reader {
    FILE *f;
    Hash64 hs;
    bool ok = true;
    void get(void *d, size_t n) {
        if (ok && n && fread(d, 1, n, f) != n) ok = false;
        if (ok) hs.add(d, n);
    }
};

blast_status read_basis_from_file(blast_plan *p, void *ctx) {
    Reader &r = *(Reader *)ctx;
    const size_t n = (size_t)p->NP * p->rows_pad * p->nc_pad;
    hipError_t e = hipMalloc(&p->basis.f64, n * sizeof(double));
    if (e != hipSuccess) {
        p->basis.f64 = nullptr;
        blast::set_error("basis allocation: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP;
    }
    const size_t chunk = (size_t)8 << 20;  // doubles per read
    std::vector<double> buf(std::min(n, chunk));
    for (size_t off = 0; off < n; off += chunk) {
        const size_t m = std::min(chunk, n - off);
        r.get(buf.data(), m * sizeof(double));
        if (!r.ok) return blast::set_error("plan file truncated"), BLAST_E_INVALID;
        BLAST_HIP_TRY(hipMemcpy(p->basis.f64 + off, buf.data(), m * sizeof(double), hipMemcpyHostToDevice));
    }
    uint64_t stored = 0;
    const uint64_t computed = r.hs.h;
    if (fread(&stored, 1, 8, r.f) != 8 || stored != computed)
        return blast::set_error("plan file checksum mismatch"), BLAST_E_INVALID;
    return BLAST_OK;
}
}  // namespace

extern "C" blast_status blast_plan_save(const blast_plan *p, const char *path) {
    blast::clear_error();
    if (!p || !path) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    FILE *f = std::fopen(path, "wb");
    if (!f) return blast::set_error("cannot open %s for writing", path), BLAST_E_INVALID;
    DeviceGuard guard(p->device);
    Writer w{f};
    w.put(kMagic, 8);
    const int32_t hdr[8] = {(int32_t)kFileVersion, p->n_ell, p->n_chi, p->n_R, p->n_cheb, (int32_t)p->types,
                            (int32_t)p->precisions, p->kq_panels};
    w.put(hdr, sizeof(hdr));
    const double hd[3] = {p->kmin, p->kmax, p->kq_phase};
    w.put(hd, sizeof(hd));
    w.put(p->ell.data(), sizeof(double) * p->n_ell);
    w.put(p->chi.data(), sizeof(double) * p->n_chi);
    w.put(p->w_chi.data(), sizeof(double) * p->n_chi);
    w.put(p->R.data(), sizeof(double) * p->n_R);
    w.put(p->w_R.data(), sizeof(double) * p->n_R);
    const size_t n = (size_t)p->NP * p->rows_pad * p->nc_pad;
    const size_t chunk = (size_t)8 << 20;
    std::vector<double> buf(std::min(n, chunk));
    blast_status st = BLAST_OK;
    for (size_t off = 0; off < n && st == BLAST_OK; off += chunk) {
        const size_t m = std::min(chunk, n - off);
        if (hipMemcpy(buf.data(), p->basis.f64 + off, m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            blast::set_error("basis download failed");
            st = BLAST_E_HIP;
            break;
        }
        w.put(buf.data(), m * sizeof(double));
    }
    const uint64_t h = w.hs.h;
    if (st == BLAST_OK && fwrite(&h, 1, 8, f) != 8) w.ok = false;
    if (std::fclose(f) != 0) w.ok = false;
    if (st == BLAST_OK && !w.ok) {
        blast::set_error("write to %s failed", path);
        st = BLAST_E_INVALID;
    }
    return st;
}

extern "C" blast_status blast_plan_load(const char *path, int32_t device, uint32_t precisions, blast_plan **out) {
    blast::clear_error();
    if (!path || !out) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return blast::set_error("cannot open %s", path), BLAST_E_INVALID;
    Reader r{f};
    char magic[8];
    r.get(magic, 8);
    int32_t hdr[8] = {0};
    double hd[3] = {0};
    r.get(hdr, sizeof(hdr));
    r.get(hd, sizeof(hd));
    blast_status st = BLAST_OK;
    if (!r.ok || std::memcmp(magic, kMagic, 8) != 0) {
        st = BLAST_E_INVALID;
        blast::set_error("%s is not a plan file", path);
    } else if (hdr[0] != (int32_t)kFileVersion) {
        st = BLAST_E_INVALID;
        blast::set_error("plan file version %d, expected %u", hdr[0], kFileVersion);
    } else if (hdr[1] < 1 || hdr[1] > blast::kMaxEll || hdr[2] < 1 || hdr[2] > (1 << 20) || hdr[3] < 1 ||
               hdr[3] > (1 << 20)) {
        st = BLAST_E_INVALID;
        blast::set_error("corrupt plan header");
    }
    if (st != BLAST_OK) {
        std::fclose(f);
        return st;
    }
    std::vector<double> ell(hdr[1]);
    std::vector<double> chi(hdr[2]), wchi(hdr[2]), R(hdr[3]), wR(hdr[3]);
    r.get(ell.data(), sizeof(double) * ell.size());
    r.get(chi.data(), sizeof(double) * chi.size());
    r.get(wchi.data(), sizeof(double) * wchi.size());
    r.get(R.data(), sizeof(double) * R.size());
    r.get(wR.data(), sizeof(double) * wR.size());
    if (!r.ok) {
        std::fclose(f);
        return blast::set_error("plan file truncated"), BLAST_E_INVALID;
    }
    blast_plan_desc d{};
    d.n_ell = hdr[1];
    d.ell = ell.data();
    d.n_chi = hdr[2];
    d.chi = chi.data();
    d.w_chi = wchi.data();
    d.n_R = hdr[3];
    d.R = R.data();
    d.w_R = wR.data();
    d.k_min = hd[0];
    d.k_max = hd[1];
    d.n_cheb = hdr[4];
    d.types = (uint32_t)hdr[5];
    d.precisions = precisions ? precisions : (uint32_t)hdr[6];
    d.kq_panels = hdr[7];
    d.kq_phase = hd[2];
    st = plan_create_impl(&d, device, read_basis_from_file, &r, out);
    std::fclose(f);
    return st;
}

extern "C" blast_status blast_plan_grids(const blast_plan *p, int32_t *n_ell, int32_t *n_chi, int32_t *n_R,
                                         int32_t *n_cheb, uint32_t *types, double *k_min, double *k_max,
                                         double *ell, double *chi, double *w_chi, double *R, double *w_R) {
    if (!p) return blast::set_error("plan is NULL"), BLAST_E_INVALID;
    if (n_ell) *n_ell = p->n_ell;
    if (n_chi) *n_chi = p->n_chi;
    if (n_R) *n_R = p->n_R;
    if (n_cheb) *n_cheb = p->n_cheb;
    if (types) *types = p->types;
    if (k_min) *k_min = p->kmin;
    if (k_max) *k_max = p->kmax;
    if (ell) std::memcpy(ell, p->ell.data(), sizeof(double) * p->n_ell);
    if (chi) std::memcpy(chi, p->chi.data(), sizeof(double) * p->n_chi);
    if (w_chi) std::memcpy(w_chi, p->w_chi.data(), sizeof(double) * p->n_chi);
    if (R) std::memcpy(R, p->R.data(), sizeof(double) * p->n_R);
    if (w_R) std::memcpy(w_R, p->w_R.data(), sizeof(double) * p->n_R);
    return BLAST_OK;
}

extern "C" blast_status blast_plan_eval_points(const blast_plan *p, double *chi, double *chi2) {
    if (!p) return blast::set_error("plan is NULL"), BLAST_E_INVALID;
    if (chi) std::memcpy(chi, p->chi.data(), sizeof(double) * p->n_chi);
    if (chi2)
        for (int a = 0; a < p->n_chi; ++a)
            for (int b = 0; b < p->n_R; ++b) chi2[(size_t)a * p->n_R + b] = p->R[b] * p->chi[a];
    return BLAST_OK;
}

extern "C" blast_status blast_plan_limber_k(const blast_plan *p, double *k) {
    if (!p || !k) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    for (int l = 0; l < p->n_ell; ++l)
        for (int a = 0; a < p->n_chi; ++a) k[(size_t)l * p->n_chi + a] = (p->ell[l] + 0.5) / p->chi[a];
    return BLAST_OK;
}

extern "C" blast_status blast_cl_limber(blast_plan *plan, const blast_limber_args *args, void *stream) {
    blast::clear_error();
    if (!plan || !args) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    DeviceGuard guard(plan->device);
    return blast::limber(plan, args, (hipStream_t)stream);
}

extern "C" blast_status blast_plan_destroy(blast_plan *plan) {
    if (!plan) return BLAST_OK;
    DeviceGuard guard(plan->device);
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return BLAST_OK;
}

extern "C" blast_status blast_plan_info(const blast_plan *p, int32_t *rows, int32_t *n_cheb_pad, size_t *basis_bytes,
                                        int64_t *kq_nodes, double *build_ms) {
    if (!p) return blast::set_error("plan is NULL"), BLAST_E_INVALID;
    if (rows) *rows = p->rows;
    if (n_cheb_pad) *n_cheb_pad = p->nc_pad;
    if (basis_bytes) {
        const size_t n = (size_t)p->NP * p->rows_pad * p->nc_pad, sc = (size_t)p->NP * p->rows_pad * 4;
        basis_bytes[0] = (p->basis.f64 ? n * 8 : 0) + (p->basis.nf64 ? n * 8 : 0);
        basis_bytes[1] = (p->basis.f32 ? n * 4 : 0) + (p->basis.nf32 ? n * 4 : 0);
        basis_bytes[2] = p->basis.hi ? n * 2 + sc : 0;
        basis_bytes[3] = p->basis.lo ? n * 4 + sc : 0;
        basis_bytes[4] = (p->basis.l16 ? n * 4 + sc : 0) + (p->basis.nl16 ? n * 4 + sc : 0);
    }
    if (kq_nodes) *kq_nodes = p->kq_nodes;
    if (build_ms) *build_ms = p->build_ms;
    return BLAST_OK;
}

extern "C" blast_status blast_plan_k_nodes(const blast_plan *p, double *k) {
    if (!p || !k) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    std::memcpy(k, p->knodes.data(), sizeof(double) * p->n_cheb);
    return BLAST_OK;
}

extern "C" blast_status blast_plan_basis_point(const blast_plan *p, int32_t a, int32_t b, double *out) {
    if (!p || !out) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    if (a < 0 || a >= p->n_chi || b < 0 || b >= p->n_R) return blast::set_error("(a, b) out of range"), BLAST_E_INVALID;
    DeviceGuard guard(p->device);
    std::vector<double> tmp((size_t)p->rows_pad * p->nc_pad);
    const size_t off = ((size_t)a * p->n_R + b) * p->rows_pad * p->nc_pad;
    BLAST_HIP_TRY(hipMemcpy(tmp.data(), p->basis.f64 + off, tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int r = 0; r < p->rows; ++r)
        for (int n = 0; n < p->n_cheb; ++n) out[(size_t)r * p->n_cheb + n] = tmp[(size_t)r * p->nc_pad + n];
    return BLAST_OK;
}

// --------------------------------------------------------------------------------------------
// forward
// --------------------------------------------------------------------------------------------

extern "C" blast_status blast_cl_workspace_bytes(const blast_plan *p, int32_t batch, int32_t precision, int32_t n_bins,
                                                 size_t *bytes) {
    if (!p || !bytes || batch < 1 || precision < 0 || precision > 4 || n_bins < 1 || n_bins > blast::kMaxBins)
        return blast::set_error("blast_cl_workspace_bytes: bad argument"), BLAST_E_INVALID;
    *bytes = blast::workspace_bytes(p, batch, precision, n_bins);
    return BLAST_OK;
}

extern "C" blast_status blast_cl_forward(blast_plan *p, const blast_cl_args *a, void *stream) {
    blast::clear_error();
    if (!p || !a) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    DeviceGuard guard(p->device);
    return blast::forward(p, a, (hipStream_t)stream);
}

extern "C" blast_status blast_cl_forward_noalloc(blast_plan *p, const blast_cl_args *a, void *stream) {
    blast::clear_error();
    if (!p || !a) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    DeviceGuard guard(p->device);
    return blast::forward_noalloc(p, a, (hipStream_t)stream);
}

extern "C" blast_status blast_cl_backward(blast_plan *p, const blast_cl_args *a, const double *dC, void *dP,
                                          double *dK_chi, double *dK_chi2, void *stream) {
    blast::clear_error();
    if (!p || !a) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    DeviceGuard guard(p->device);
    return blast::backward(p, a, dC, dP, dK_chi, dK_chi2, (hipStream_t)stream);
}

// --------------------------------------------------------------------------------------------
// stage timing
// --------------------------------------------------------------------------------------------

extern "C" blast_status blast_plan_profile(blast_plan *p, int32_t enable) {
    if (!p) return blast::set_error("plan is NULL"), BLAST_E_INVALID;
    std::lock_guard<std::mutex> lk(p->mu);
    p->profile = enable != 0;
    return BLAST_OK;
}

extern "C" blast_status blast_plan_profile_read(blast_plan *p, double *stage_ms, int64_t *calls) {
    if (!p || !stage_ms) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    DeviceGuard guard(p->device);
    std::lock_guard<std::mutex> lk(p->mu);
    for (int i = 0; i < 4; ++i) stage_ms[i] = 0.0;
    const size_t n = p->prof_events.size() / 5;
    blast_status st = BLAST_OK;
    for (size_t c = 0; c < n && st == BLAST_OK; ++c) {
        hipEvent_t *e = &p->prof_events[5 * c];
        if (hipEventSynchronize(e[4]) != hipSuccess) {
            blast::set_error("hipEventSynchronize failed");
            st = BLAST_E_HIP;
            break;
        }
        for (int i = 0; i < 4; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e[i], e[i + 1]) != hipSuccess) {
                blast::set_error("hipEventElapsedTime failed");
                st = BLAST_E_HIP;
                break;
            }
            stage_ms[i] += ms;
        }
    }
    for (hipEvent_t e : p->prof_events) (void)hipEventDestroy(e);
    p->prof_events.clear();
    if (calls) *calls = (int64_t)n;
    return st;
}
