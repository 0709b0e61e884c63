// Continuous-batching server: independent single-cosmology requests -> batched forward calls.
//
// The server's device memory is split into slot-sets, each one arena with a stream of its own.
// A request's bins fall in a bucket: its clustering bins rounded up to a multiple of 4 (at most
// max_g, 0 when it has none), and max_s shear bins.  A launch has the bucket of its largest
// request and as many cosmologies as requests; for every bucket and every batch size 1, 2, 4, ...
// whose inputs, outputs and forward scratch fit the arena, a hipGraph is captured at creation
// with the arena laid out for that shape.  The scheduler thread admits queued requests in
// arrival order into the forming set while the launch they would make still fits its arena
// (admission by memory: requests with fewer bins take fewer bytes), launches the set when the
// next request does not fit, when its oldest request has waited max_wait_ms or when no other set
// runs: the requests' inputs go into the arena in the layout of the shape, the graph of the
// smallest captured batch that holds them is replayed, C comes back to pinned host memory and
// an event marks completion.  Sets launched while others run overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t id = 0;
    blast_request r{};
    std::vector<int32_t> ell_idx;
    Clock::time_point t_submit;
};

struct Done {
    blast_status st;
    double lat_ms;
};

struct Graph {
    int batch = 0, G = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
};

// where the inputs, outputs and scratch of one launch shape sit in a set's arena
struct Lay {
    size_t P = 0, K1 = 0, K2 = 0, C = 0, ws = 0, ws_bytes = 0, total = 0;
};

struct Set {
    hipStream_t stream = nullptr;
    unsigned char *arena = nullptr;
    double *C_host = nullptr;  // pinned
    std::vector<Graph> graphs;
    hipEvent_t done = nullptr;
    std::vector<Req> slots;
    int G = 0;              // clustering-bin bucket of the requests admitted so far
    int run_batch = 0, run_G = 0;
    bool in_flight = false;
};

int npairs(int ng, int ns, uint32_t t) {
    int n = 0;
    if (t & BLAST_GG) n += ng * (ng + 1) / 2;
    if (t & BLAST_GS) n += ng * ns;
    if (t & BLAST_SS) n += ns * (ns + 1) / 2;
    return n;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

struct blast_server {
    blast_plan *plan = nullptr;
    blast_server_desc d{};
    size_t p_elem = 0, P_slot = 0, set_bytes = 0;
    std::vector<int> buckets;       // clustering-bin buckets, ascending
    std::map<int, int> bmax;        // bucket -> most requests a launch of that bucket can hold
    std::vector<Set> sets;
    int forming = -1;
    std::deque<Req> queue;
    std::unordered_map<uint64_t, Done> done;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::thread th;
    bool stop = false;
    uint64_t next_id = 1;
    int64_t submitted = 0, completed = 0, rejected = 0, cancelled = 0, launches = 0, fill_sum = 0;
    int64_t max_sets_in_flight = 0;
    std::vector<double> lat;
    Clock::time_point t_first, t_last;
    bool have_first = false;
    blast_status fatal = BLAST_OK;
};

namespace {

int bucket_of(const blast_server *S, int n_g) {
    if (n_g == 0) return 0;
    return std::min(S->d.max_g, (n_g + 3) / 4 * 4);
}

Lay lay_of(const blast_server *S, int batch, int G) {
    const blast_plan *p = S->plan;
    const int nb = G + S->d.max_s;
    Lay L;
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off += align256(n);
        return o;
    };
    L.P = take((size_t)batch * S->P_slot);
    L.K1 = take((size_t)batch * nb * p->n_chi * sizeof(double));
    L.K2 = take((size_t)batch * nb * p->NP * sizeof(double));
    L.C = take((size_t)batch * npairs(G, S->d.max_s, p->types) * p->n_ell * sizeof(double));
    L.ws_bytes = blast::forward_workspace_bytes(p, batch, S->d.precision, nb);
    L.ws = take(L.ws_bytes);
    L.total = off;
    return L;
}

// position of a request's pair (t, i, j) (its own bin numbering) in the pair list of a launch
// with G clustering and Sn shear bins
int padded_pair(uint32_t types, int G, int Sn, int t, int i, int j) {
    int off = 0;
    if (t == BLAST_GG) return i * G - i * (i - 1) / 2 + (j - i);
    if (types & BLAST_GG) off += G * (G + 1) / 2;
    if (t == BLAST_GS) return off + i * Sn + j;
    if (types & BLAST_GS) off += G * Sn;
    return off + i * Sn - i * (i - 1) / 2 + (j - i);
}

blast_cl_args launch_args(blast_server *S, Set &st, int batch, int G) {
    const Lay L = lay_of(S, batch, G);
    blast_cl_args a{};
    a.batch = batch;
    a.precision = S->d.precision;
    a.p_dtype = S->d.p_dtype;
    a.p_kind = 0;
    a.P = st.arena + L.P;
    a.n_g = G;
    a.n_s = S->d.max_s;
    a.K_chi = (const double *)(st.arena + L.K1);
    a.K_chi2 = (const double *)(st.arena + L.K2);
    a.types = S->plan->types;
    a.n_ell_out = 0;
    a.ell_idx = nullptr;
    a.C = (double *)(st.arena + L.C);
    a.w_save = nullptr;
    a.workspace = st.arena + L.ws;
    a.workspace_bytes = L.ws_bytes;
    return a;
}

hipError_t launch_set(blast_server *S, Set &st) {
    const int n = (int)st.slots.size();
    const blast_plan *p = S->plan;
    int G = 0;
    for (const Req &q : st.slots) G = std::max(G, bucket_of(S, q.r.n_g));
    // the smallest captured batch of this bucket that holds the requests (plain calls: exactly n)
    const Graph *g = nullptr;
    if (S->d.use_graphs)
        for (const Graph &gr : st.graphs)
            if (gr.G == G && gr.batch >= n && (!g || gr.batch < g->batch)) g = &gr;
    const int b = g ? g->batch : n;
    const Lay L = lay_of(S, b, G);
    const int nb = G + S->d.max_s;
    hipError_t e = hipSuccess;
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        const blast_request &r = st.slots[k].r;
        e = hipMemcpyAsync(st.arena + L.P + (size_t)k * S->P_slot, r.P, S->P_slot, hipMemcpyHostToDevice, st.stream);
        double *K1 = (double *)(st.arena + L.K1) + (size_t)k * nb * p->n_chi;
        double *K2 = (double *)(st.arena + L.K2) + (size_t)k * nb * p->NP;
        if (e == hipSuccess) e = hipMemsetAsync(K1, 0, sizeof(double) * nb * p->n_chi, st.stream);
        if (e == hipSuccess) e = hipMemsetAsync(K2, 0, sizeof(double) * nb * p->NP, st.stream);
        // clustering bins at 0..n_g-1, shear bins at G..G+n_s-1
        if (e == hipSuccess && r.n_g)
            e = hipMemcpyAsync(K1, r.K_chi, sizeof(double) * r.n_g * p->n_chi, hipMemcpyHostToDevice, st.stream);
        if (e == hipSuccess && r.n_s)
            e = hipMemcpyAsync(K1 + (size_t)G * p->n_chi, r.K_chi + (size_t)r.n_g * p->n_chi,
                               sizeof(double) * r.n_s * p->n_chi, hipMemcpyHostToDevice, st.stream);
        if (e == hipSuccess && r.n_g)
            e = hipMemcpyAsync(K2, r.K_chi2, sizeof(double) * r.n_g * p->NP, hipMemcpyHostToDevice, st.stream);
        if (e == hipSuccess && r.n_s)
            e = hipMemcpyAsync(K2 + (size_t)G * p->NP, r.K_chi2 + (size_t)r.n_g * p->NP,
                               sizeof(double) * r.n_s * p->NP, hipMemcpyHostToDevice, st.stream);
    }
    if (e != hipSuccess) return e;
    if (g) {
        e = hipGraphLaunch(g->exec, st.stream);
    } else {
        blast_cl_args a = launch_args(S, st, b, G);
        if (blast::forward(S->plan, &a, st.stream) != BLAST_OK) return hipErrorLaunchFailure;
    }
    const size_t c_req = (size_t)npairs(G, S->d.max_s, p->types) * p->n_ell * sizeof(double);
    if (e == hipSuccess)
        e = hipMemcpyAsync(st.C_host, st.arena + L.C, c_req * n, hipMemcpyDeviceToHost, st.stream);
    if (e == hipSuccess) e = hipEventRecord(st.done, st.stream);
    st.run_batch = b;
    st.run_G = G;
    return e;
}

void finish(blast_server *S, const Req &q, blast_status status, Clock::time_point now) {
    const double ms = std::chrono::duration<double, std::milli>(now - q.t_submit).count();
    S->done[q.id] = Done{status, ms};
    if (status == BLAST_OK) {
        S->lat.push_back(ms);
        S->completed++;
    }
}

void complete_set(blast_server *S, Set &st, blast_status status) {
    const blast_plan *p = S->plan;
    const uint32_t types = p->types;
    const int G = st.run_G, Sn = S->d.max_s;
    const size_t c_req = (size_t)npairs(G, Sn, types) * p->n_ell;
    const Clock::time_point now = Clock::now();
    for (size_t k = 0; k < st.slots.size(); ++k) {
        Req &q = st.slots[k];
        const blast_request &r = q.r;
        if (status == BLAST_OK) {
            const double *Cs = st.C_host + k * c_req;
            const int nl = (int)q.ell_idx.size();
            int pr = 0;
            auto put = [&](int t, int i, int j) {
                const int pp = padded_pair(types, G, Sn, t, i, j);
                for (int l = 0; l < nl; ++l) r.C_out[(size_t)pr * nl + l] = Cs[(size_t)pp * p->n_ell + q.ell_idx[l]];
                ++pr;
            };
            if (types & BLAST_GG)
                for (int i = 0; i < r.n_g; ++i)
                    for (int j = i; j < r.n_g; ++j) put(BLAST_GG, i, j);
            if (types & BLAST_GS)
                for (int i = 0; i < r.n_g; ++i)
                    for (int j = 0; j < r.n_s; ++j) put(BLAST_GS, i, j);
            if (types & BLAST_SS)
                for (int i = 0; i < r.n_s; ++i)
                    for (int j = i; j < r.n_s; ++j) put(BLAST_SS, i, j);
        }
        finish(S, q, status, now);
    }
    S->t_last = now;
    st.slots.clear();
    st.G = 0;
    st.in_flight = false;
    S->cv_done.notify_all();
}

void scheduler(blast_server *S) {
    (void)hipSetDevice(S->plan->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = false;
        // completions
        for (Set &st : S->sets) {
            if (!st.in_flight) continue;
            const hipError_t q = hipEventQuery(st.done);
            if (q == hipSuccess) {
                complete_set(S, st, BLAST_OK);
                progress = true;
            } else if (q != hipErrorNotReady) {
                S->fatal = BLAST_E_HIP;
                complete_set(S, st, BLAST_E_HIP);
                progress = true;
            }
        }
        if (S->fatal != BLAST_OK) {
            const Clock::time_point now = Clock::now();
            while (!S->queue.empty()) {
                finish(S, S->queue.front(), S->fatal, now);
                S->queue.pop_front();
            }
            if (S->forming >= 0) {
                for (const Req &q : S->sets[S->forming].slots) finish(S, q, S->fatal, now);
                S->sets[S->forming].slots.clear();
                S->forming = -1;
            }
            S->cv_done.notify_all();
        }
        // admission into a free set, in arrival order, while the launch still fits its arena
        if (S->forming < 0) {
            for (size_t i = 0; i < S->sets.size(); ++i)
                if (!S->sets[i].in_flight && S->sets[i].slots.empty()) {
                    S->forming = (int)i;
                    break;
                }
        }
        int running = 0;
        for (const Set &st : S->sets) running += st.in_flight ? 1 : 0;
        if (S->forming >= 0) {
            Set &st = S->sets[S->forming];
            bool next_fits = true;
            while (!S->queue.empty()) {
                const int G = std::max(st.G, bucket_of(S, S->queue.front().r.n_g));
                if ((int)st.slots.size() + 1 > S->bmax[G]) {
                    next_fits = false;
                    break;
                }
                st.slots.push_back(std::move(S->queue.front()));
                S->queue.pop_front();
                st.G = G;
                progress = true;
            }
            const bool full = !next_fits || (!st.slots.empty() && (int)st.slots.size() >= S->bmax[st.G]);
            const bool waited =
                !st.slots.empty() && std::chrono::duration<double, std::milli>(Clock::now() - st.slots[0].t_submit)
                                             .count() >= S->d.max_wait_ms;
            if (!st.slots.empty() && (full || running == 0 || waited || S->stop)) {
                S->forming = -1;
                st.in_flight = true;
                S->launches++;
                S->fill_sum += (int64_t)st.slots.size();
                S->max_sets_in_flight = std::max<int64_t>(S->max_sets_in_flight, running + 1);
                lk.unlock();
                const hipError_t e = launch_set(S, st);
                lk.lock();
                if (e != hipSuccess) {
                    S->fatal = BLAST_E_HIP;
                    complete_set(S, st, BLAST_E_HIP);
                }
                continue;
            }
        }
        if (S->stop && S->queue.empty()) {
            bool busy = false;
            for (const Set &st : S->sets) busy |= st.in_flight || !st.slots.empty();
            if (!busy) break;
        }
        if (!progress) S->cv_sched.wait_for(lk, std::chrono::microseconds(50));
    }
}

void free_sets(blast_server *S) {
    for (Set &st : S->sets) {
        for (Graph &g : st.graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.g) (void)hipGraphDestroy(g.g);
        }
        if (st.arena) (void)hipFree(st.arena);
        if (st.C_host) (void)hipHostFree(st.C_host);
        if (st.done) (void)hipEventDestroy(st.done);
        if (st.stream) (void)hipStreamDestroy(st.stream);
    }
    S->sets.clear();
}

}  // namespace

extern "C" blast_status blast_server_create(blast_plan *plan, const blast_server_desc *d, blast_server **out) {
    blast::clear_error();
    if (!plan || !d || !out) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    *out = nullptr;
    if (d->batch < 1 || d->batch > 1024 || d->max_g < 0 || d->max_s < 0 || d->max_g + d->max_s < 1 ||
        d->max_g + d->max_s > blast::kMaxBins || d->n_sets < 0 || d->n_sets > 4 || d->p_dtype < 0 ||
        d->p_dtype > 1 || d->max_wait_ms < 0 || d->precision < 0 || d->precision > 4)
        return blast::set_error("bad server descriptor"), BLAST_E_INVALID;
    if (d->precision == BLAST_FP16X3 && d->max_g + d->max_s > 20)
        return blast::set_error("FP16X3 takes at most 20 bins"), BLAST_E_UNSUPPORTED;
    blast_server *S = new (std::nothrow) blast_server();
    if (!S) return blast::set_error("host allocation failed"), BLAST_E_OOM;
    S->plan = plan;
    S->d = *d;
    if (!S->d.max_queue) S->d.max_queue = 4096;
    const size_t budget = d->hbm_budget ? d->hbm_budget : (size_t)8 << 30;
    S->p_elem = d->p_dtype == 0 ? 8 : 4;
    S->P_slot = (size_t)plan->NP * plan->n_cheb * S->p_elem;
    for (int n = d->max_s ? 0 : 1; n <= d->max_g; ++n) {
        const int b = bucket_of(S, n);
        if (S->buckets.empty() || S->buckets.back() != b) S->buckets.push_back(b);
    }
    // sets: each an arena for `batch` requests of the largest bucket, or the budget's share
    const size_t full = lay_of(S, d->batch, d->max_g).total;
    int nsets = d->n_sets ? d->n_sets : (int)std::max<size_t>(1, std::min<size_t>(4, budget / full));
    S->set_bytes = std::min(full, budget / nsets);
    for (int G : S->buckets) {
        int b = 0;
        while (b < d->batch && lay_of(S, b + 1, G).total <= S->set_bytes) ++b;
        S->bmax[G] = b;
    }
    if (S->bmax[S->buckets.front()] < 1) {
        blast::set_error("an HBM budget of %zu bytes in %d sets holds no request (one needs %zu bytes)", budget, nsets,
                         lay_of(S, 1, S->buckets.front()).total);
        delete S;
        return BLAST_E_OOM;
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(plan->device);
    S->sets.resize(nsets);
    const size_t c_host = (size_t)d->batch * npairs(d->max_g, d->max_s, plan->types) * plan->n_ell * sizeof(double);
    hipError_t e = hipSuccess;
    for (Set &st : S->sets) {
        if (e == hipSuccess) e = hipStreamCreate(&st.stream);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc((void **)&st.arena, S->set_bytes);
        if (e == hipSuccess) e = hipHostMalloc((void **)&st.C_host, c_host, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMemset(st.arena, 0, S->set_bytes);
    }
    blast_status bst = BLAST_OK;
    if (e != hipSuccess) {
        blast::set_error("server buffers: %s", hipGetErrorString(e));
        bst = e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP;
    }
    // one uncaptured forward per set (first-use setup), then a graph per (bucket, batch size)
    for (Set &st : S->sets) {
        if (bst != BLAST_OK) break;
        int G0 = S->buckets.front();
        for (int G : S->buckets)
            if (S->bmax[G] >= 1) G0 = G;
        {
            blast_cl_args a = launch_args(S, st, S->bmax[G0], G0);
            bst = blast::forward(plan, &a, st.stream);
            if (bst == BLAST_OK && hipStreamSynchronize(st.stream) != hipSuccess) bst = BLAST_E_HIP;
        }
        if (bst != BLAST_OK || !d->use_graphs) continue;
        for (int G : S->buckets) {
            const int bm = S->bmax[G];
            std::vector<int> sizes;
            for (int b = 1; b < bm; b *= 2) sizes.push_back(b);
            if (bm >= 1) sizes.push_back(bm);
            for (int b : sizes) {
                Graph g;
                g.batch = b;
                g.G = G;
                blast_cl_args a = launch_args(S, st, b, G);
                e = hipStreamBeginCapture(st.stream, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) break;
                const blast_status fs = blast::forward(plan, &a, st.stream);
                e = hipStreamEndCapture(st.stream, &g.g);
                if (fs != BLAST_OK) {
                    bst = fs;
                    break;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.g, nullptr, nullptr, 0);
                if (e != hipSuccess) break;
                st.graphs.push_back(g);
            }
            if (e != hipSuccess || bst != BLAST_OK) break;
        }
        if (e != hipSuccess && bst == BLAST_OK) {
            blast::set_error("graph capture: %s", hipGetErrorString(e));
            bst = BLAST_E_HIP;
        }
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    if (bst != BLAST_OK) {
        free_sets(S);
        delete S;
        return bst;
    }
    S->th = std::thread(scheduler, S);
    *out = S;
    return BLAST_OK;
}

extern "C" blast_status blast_server_footprint(const blast_server *S, int32_t n_g, int32_t n_s, int32_t count,
                                               size_t *bytes, size_t *set_bytes) {
    if (!S || !bytes) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    if (n_g < 0 || n_s < 0 || n_g > S->d.max_g || n_s > S->d.max_s || n_g + n_s < 1 || count < 1 ||
        count > S->d.batch)
        return blast::set_error("bins or count outside the server's limits"), BLAST_E_INVALID;
    *bytes = lay_of(S, count, bucket_of(S, n_g)).total;
    if (set_bytes) *set_bytes = S->set_bytes;
    return BLAST_OK;
}

extern "C" blast_status blast_server_submit(blast_server *S, const blast_request *r, uint64_t *ticket) {
    if (!S || !r || !ticket) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    const blast_plan *p = S->plan;
    if (!r->P || r->n_g < 0 || r->n_s < 0 || r->n_g > S->d.max_g || r->n_s > S->d.max_s || r->n_g + r->n_s < 1 ||
        !r->K_chi || !r->K_chi2 || !r->C_out || r->n_ell < 1 || r->n_ell > p->n_ell || !r->ell_idx ||
        npairs(r->n_g, r->n_s, p->types) < 1) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->rejected++;
        return blast::set_error("malformed request"), BLAST_E_INVALID;
    }
    for (int i = 0; i < r->n_ell; ++i)
        if (r->ell_idx[i] < 0 || r->ell_idx[i] >= p->n_ell || (i && r->ell_idx[i] <= r->ell_idx[i - 1])) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->rejected++;
            return blast::set_error("ell_idx must be increasing plan indices"), BLAST_E_INVALID;
        }
    Req q;
    q.r = *r;
    q.ell_idx.assign(r->ell_idx, r->ell_idx + r->n_ell);
    q.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->fatal != BLAST_OK) return blast::set_error("server failed earlier"), S->fatal;
        const int G = bucket_of(S, r->n_g);
        if (S->bmax[G] < 1) {
            S->rejected++;
            return blast::set_error("a request with %d clustering bins needs %zu bytes; a set holds %zu", r->n_g,
                                    lay_of(S, 1, G).total, S->set_bytes),
                   BLAST_E_OOM;
        }
        if ((int)S->queue.size() >= S->d.max_queue) {
            S->rejected++;
            return blast::set_error("queue full"), BLAST_E_BUSY;
        }
        q.id = S->next_id++;
        *ticket = q.id;
        if (!S->have_first) {
            S->t_first = q.t_submit;
            S->have_first = true;
        }
        S->submitted++;
        S->queue.push_back(std::move(q));
    }
    S->cv_sched.notify_one();
    return BLAST_OK;
}

extern "C" blast_status blast_server_cancel(blast_server *S, uint64_t ticket) {
    if (!S) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    const Clock::time_point now = Clock::now();
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
        if (it->id == ticket) {
            finish(S, *it, BLAST_E_CANCELLED, now);
            S->queue.erase(it);
            S->cancelled++;
            S->cv_done.notify_all();
            return BLAST_OK;
        }
    if (S->forming >= 0) {
        Set &st = S->sets[S->forming];
        for (auto it = st.slots.begin(); it != st.slots.end(); ++it)
            if (it->id == ticket) {
                finish(S, *it, BLAST_E_CANCELLED, now);
                st.slots.erase(it);
                st.G = 0;
                for (const Req &q : st.slots) st.G = std::max(st.G, bucket_of(S, q.r.n_g));
                S->cancelled++;
                S->cv_done.notify_all();
                return BLAST_OK;
            }
    }
    for (const Set &st : S->sets)
        if (st.in_flight)
            for (const Req &q : st.slots)
                if (q.id == ticket) return blast::set_error("request %llu is running", (unsigned long long)ticket), BLAST_E_BUSY;
    return blast::set_error("ticket %llu is not pending", (unsigned long long)ticket), BLAST_E_INVALID;
}

static blast_status take_done(blast_server *S, uint64_t ticket, blast_status *req_status, double *latency_ms) {
    const Done d = S->done[ticket];
    S->done.erase(ticket);
    if (req_status) *req_status = d.st;
    if (latency_ms) *latency_ms = d.lat_ms;
    return BLAST_OK;
}

extern "C" blast_status blast_server_wait(blast_server *S, uint64_t ticket, int32_t timeout_ms,
                                          blast_status *req_status, double *latency_ms) {
    if (!S) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] { return S->done.count(ticket) > 0; };
    if (timeout_ms < 0)
        S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        return blast::set_error("timeout"), BLAST_E_BUSY;
    return take_done(S, ticket, req_status, latency_ms);
}

extern "C" blast_status blast_server_poll(blast_server *S, uint64_t ticket, int32_t *done, blast_status *req_status,
                                          double *latency_ms) {
    if (!S || !done) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    *done = S->done.count(ticket) > 0 ? 1 : 0;
    if (!*done) return BLAST_OK;
    return take_done(S, ticket, req_status, latency_ms);
}

extern "C" blast_status blast_server_stats_get(blast_server *S, blast_server_stats *o) {
    if (!S || !o) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    o->submitted = S->submitted;
    o->completed = S->completed;
    o->rejected = S->rejected;
    o->launches = S->launches;
    o->queued = (int64_t)S->queue.size();
    int64_t inf = 0;
    for (const Set &st : S->sets) inf += st.in_flight ? (int64_t)st.slots.size() : 0;
    o->in_flight = inf;
    o->mean_fill = S->launches ? (double)S->fill_sum / S->launches : 0.0;
    std::vector<double> v = S->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
        if (v.empty()) return 0.0;
        const size_t i = std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5));
        return v[i];
    };
    o->p50_ms = pct(0.50);
    o->p99_ms = pct(0.99);
    o->span_ms = S->have_first ? std::chrono::duration<double, std::milli>(S->t_last - S->t_first).count() : 0.0;
    o->cancelled = S->cancelled;
    o->max_sets_in_flight = S->max_sets_in_flight;
    o->n_sets = (int64_t)S->sets.size();
    o->set_bytes = (int64_t)S->set_bytes;
    return BLAST_OK;
}

extern "C" blast_status blast_server_destroy(blast_server *S) {
    if (!S) return BLAST_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_sched.notify_all();
    if (S->th.joinable()) S->th.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->plan->device);
    for (Set &st : S->sets)
        if (st.stream) (void)hipStreamSynchronize(st.stream);
    free_sets(S);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete S;
    return BLAST_OK;
}
