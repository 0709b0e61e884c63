// Continuous-batching server: independent single-cosmology requests -> batched forward calls.
//
// Slot-sets own fixed device buffers (inputs, outputs, workspace) and a stream each.  A
// scheduler thread fills the free set with queued requests, launches it (H2D copies of the
// requests' inputs, one replay of the captured hipGraph for the smallest captured batch that
// holds them, D2H copy of C, an event), and completes requests when their set's event fires.
// Sets launched while others run overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
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
    int batch = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct Set {
    hipStream_t stream = nullptr;
    void *P = nullptr;
    double *K1 = nullptr, *K2 = nullptr, *C = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    double *C_host = nullptr;  // pinned
    std::vector<Graph> graphs;
    hipEvent_t done = nullptr;
    std::vector<Req> slots;
    bool in_flight = false;
};

int npairs(int ng, int ns, uint32_t t) {
    int n = 0;
    if (t & BLAST_GG) n += ng * (ng + 1) / 2;
    if (t & BLAST_GS) n += ng * ns;
    if (t & BLAST_SS) n += ns * (ns + 1) / 2;
    return n;
}

}  // namespace

struct blast_server {
    blast_plan *plan = nullptr;
    blast_server_desc d{};
    int bins = 0, npairs_pad = 0;
    size_t p_elem = 0, P_slot = 0, K1_slot = 0, K2_slot = 0, C_slot = 0;
    std::vector<Set> sets;
    int forming = -1;
    std::deque<Req> queue;
    std::unordered_map<uint64_t, Done> done;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::thread th;
    bool stop = false;
    uint64_t next_id = 1;
    int64_t submitted = 0, completed = 0, rejected = 0, launches = 0, fill_sum = 0;
    std::vector<double> lat;
    Clock::time_point t_first, t_last;
    bool have_first = false;
    blast_status fatal = BLAST_OK;
};

namespace {

// position of a request's pair (t, i, j) (its own bin numbering) in the padded pair list
int padded_pair(const blast_server *S, int t, int i, int j) {
    const int G = S->d.max_g, Sn = S->d.max_s;
    const uint32_t types = S->plan->types;
    int off = 0;
    if (t == BLAST_GG) return i * G - i * (i - 1) / 2 + (j - i);
    if (types & BLAST_GG) off += G * (G + 1) / 2;
    if (t == BLAST_GS) return off + i * Sn + j;
    if (types & BLAST_GS) off += G * Sn;
    return off + i * Sn - i * (i - 1) / 2 + (j - i);
}

blast_cl_args set_args(blast_server *S, Set &st, int batch) {
    blast_cl_args a{};
    a.batch = batch;
    a.precision = S->d.precision;
    a.p_dtype = S->d.p_dtype;
    a.p_kind = 0;
    a.P = st.P;
    a.n_g = S->d.max_g;
    a.n_s = S->d.max_s;
    a.K_chi = st.K1;
    a.K_chi2 = st.K2;
    a.types = S->plan->types;
    a.n_ell_out = 0;
    a.ell_idx = nullptr;
    a.C = st.C;
    a.w_save = nullptr;
    a.workspace = st.ws;
    a.workspace_bytes = st.ws_bytes;
    return a;
}

hipError_t launch_set(blast_server *S, Set &st) {
    const int n = (int)st.slots.size();
    const blast_plan *p = S->plan;
    hipError_t e = hipSuccess;
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        const blast_request &r = st.slots[k].r;
        char *P = (char *)st.P + (size_t)k * S->P_slot;
        e = hipMemcpyAsync(P, r.P, S->P_slot, hipMemcpyHostToDevice, st.stream);
        double *K1 = st.K1 + (size_t)k * S->bins * p->n_chi;
        double *K2 = st.K2 + (size_t)k * S->bins * p->NP;
        if (e == hipSuccess) e = hipMemsetAsync(K1, 0, S->K1_slot, st.stream);
        if (e == hipSuccess) e = hipMemsetAsync(K2, 0, S->K2_slot, st.stream);
        // clustering bins at 0..n_g-1, shear bins at max_g..max_g+n_s-1
        if (e == hipSuccess && r.n_g)
            e = hipMemcpyAsync(K1, r.K_chi, sizeof(double) * r.n_g * p->n_chi, hipMemcpyHostToDevice, st.stream);
        if (e == hipSuccess && r.n_s)
            e = hipMemcpyAsync(K1 + (size_t)S->d.max_g * p->n_chi, r.K_chi + (size_t)r.n_g * p->n_chi,
                               sizeof(double) * r.n_s * p->n_chi, hipMemcpyHostToDevice, st.stream);
        if (e == hipSuccess && r.n_g)
            e = hipMemcpyAsync(K2, r.K_chi2, sizeof(double) * r.n_g * p->NP, hipMemcpyHostToDevice, st.stream);
        if (e == hipSuccess && r.n_s)
            e = hipMemcpyAsync(K2 + (size_t)S->d.max_g * p->NP, r.K_chi2 + (size_t)r.n_g * p->NP,
                               sizeof(double) * r.n_s * p->NP, hipMemcpyHostToDevice, st.stream);
    }
    if (e != hipSuccess) return e;
    // smallest captured batch that holds the requests
    const Graph *g = nullptr;
    for (const Graph &gr : st.graphs)
        if (gr.batch >= n) {
            g = &gr;
            break;
        }
    int run_batch = g ? g->batch : S->d.batch;
    if (S->d.use_graphs && g) {
        e = hipGraphLaunch(g->exec, st.stream);
    } else {
        blast_cl_args a = set_args(S, st, run_batch);
        if (blast::forward(S->plan, &a, st.stream) != BLAST_OK) return hipErrorLaunchFailure;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(st.C_host, st.C, S->C_slot * n, hipMemcpyDeviceToHost, st.stream);
    if (e == hipSuccess) e = hipEventRecord(st.done, st.stream);
    return e;
}

void complete_set(blast_server *S, Set &st, blast_status status) {
    const blast_plan *p = S->plan;
    const uint32_t types = p->types;
    const Clock::time_point now = Clock::now();
    for (size_t k = 0; k < st.slots.size(); ++k) {
        Req &q = st.slots[k];
        const blast_request &r = q.r;
        if (status == BLAST_OK) {
            const double *Cs = (const double *)((const char *)st.C_host + k * S->C_slot);
            const int nl = (int)q.ell_idx.size();
            int pr = 0;
            auto put = [&](int t, int i, int j) {
                const int pp = padded_pair(S, t, i, j);
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
        const double ms = std::chrono::duration<double, std::milli>(now - q.t_submit).count();
        S->done[q.id] = Done{status, ms};
        if (status == BLAST_OK) {
            S->lat.push_back(ms);
            S->completed++;
        }
    }
    S->t_last = now;
    st.slots.clear();
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
            while (!S->queue.empty()) {
                S->done[S->queue.front().id] = Done{S->fatal, 0.0};
                S->queue.pop_front();
            }
            S->cv_done.notify_all();
        }
        // admission into a free set
        if (S->forming < 0) {
            for (size_t i = 0; i < S->sets.size(); ++i)
                if (!S->sets[i].in_flight && S->sets[i].slots.empty()) {
                    S->forming = (int)i;
                    break;
                }
        }
        bool any_running = false;
        for (const Set &st : S->sets) any_running |= st.in_flight;
        if (S->forming >= 0) {
            Set &st = S->sets[S->forming];
            while ((int)st.slots.size() < S->d.batch && !S->queue.empty()) {
                st.slots.push_back(std::move(S->queue.front()));
                S->queue.pop_front();
                progress = true;
            }
            const bool full = (int)st.slots.size() == S->d.batch;
            const bool waited =
                !st.slots.empty() && std::chrono::duration<double, std::milli>(Clock::now() - st.slots[0].t_submit)
                                             .count() >= S->d.max_wait_ms;
            if (!st.slots.empty() && (full || !any_running || waited || S->stop)) {
                S->forming = -1;
                st.in_flight = true;
                S->launches++;
                S->fill_sum += (int64_t)st.slots.size();
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
        if (st.P) (void)hipFree(st.P);
        if (st.K1) (void)hipFree(st.K1);
        if (st.K2) (void)hipFree(st.K2);
        if (st.C) (void)hipFree(st.C);
        if (st.ws) (void)hipFree(st.ws);
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
        d->p_dtype > 1 || d->max_wait_ms < 0)
        return blast::set_error("bad server descriptor"), BLAST_E_INVALID;
    blast_server *S = new (std::nothrow) blast_server();
    if (!S) return blast::set_error("host allocation failed"), BLAST_E_OOM;
    S->plan = plan;
    S->d = *d;
    if (!S->d.max_queue) S->d.max_queue = 4096;
    const size_t budget = d->hbm_budget ? d->hbm_budget : (size_t)8 << 30;
    S->bins = d->max_g + d->max_s;
    if (d->precision == BLAST_FP16X3 && S->bins > 20) {
        delete S;
        return blast::set_error("FP16X3 takes at most 20 bins"), BLAST_E_UNSUPPORTED;
    }
    S->npairs_pad = npairs(d->max_g, d->max_s, plan->types);
    S->p_elem = d->p_dtype == 0 ? 8 : 4;
    S->P_slot = (size_t)plan->NP * plan->n_cheb * S->p_elem;
    S->K1_slot = sizeof(double) * S->bins * plan->n_chi;
    S->K2_slot = sizeof(double) * S->bins * plan->NP;
    S->C_slot = sizeof(double) * S->npairs_pad * plan->n_ell;
    size_t ws = 0;
    if (blast_cl_workspace_bytes(plan, d->batch, d->precision, S->bins, &ws) != BLAST_OK) {
        delete S;
        return BLAST_E_INVALID;
    }
    const size_t per_set = (S->P_slot + S->K1_slot + S->K2_slot + S->C_slot) * d->batch + ws;
    int nsets = d->n_sets ? d->n_sets : (int)std::min<size_t>(4, budget / per_set);
    if (nsets < 1 || per_set * nsets > budget) {
        blast::set_error("HBM budget of %zu bytes holds no set of %zu bytes", budget, per_set);
        delete S;
        return BLAST_E_OOM;
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(plan->device);
    S->sets.resize(nsets);
    hipError_t e = hipSuccess;
    for (Set &st : S->sets) {
        if (e == hipSuccess) e = hipStreamCreate(&st.stream);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&st.P, S->P_slot * d->batch);
        if (e == hipSuccess) e = hipMalloc((void **)&st.K1, S->K1_slot * d->batch);
        if (e == hipSuccess) e = hipMalloc((void **)&st.K2, S->K2_slot * d->batch);
        if (e == hipSuccess) e = hipMalloc((void **)&st.C, S->C_slot * d->batch);
        if (e == hipSuccess) e = hipMalloc(&st.ws, ws);
        st.ws_bytes = ws;
        if (e == hipSuccess) e = hipHostMalloc((void **)&st.C_host, S->C_slot * d->batch, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMemset(st.P, 0, S->P_slot * d->batch);
        if (e == hipSuccess) e = hipMemset(st.K1, 0, S->K1_slot * d->batch);
        if (e == hipSuccess) e = hipMemset(st.K2, 0, S->K2_slot * d->batch);
    }
    blast_status bst = BLAST_OK;
    if (e != hipSuccess) {
        blast::set_error("server buffers: %s", hipGetErrorString(e));
        bst = e == hipErrorOutOfMemory ? BLAST_E_OOM : BLAST_E_HIP;
    }
    // one uncaptured forward per set (first-use setup), then graphs for batches 1, 2, 4, ..., batch
    for (Set &st : S->sets) {
        if (bst != BLAST_OK) break;
        blast_cl_args a = set_args(S, st, d->batch);
        bst = blast::forward(plan, &a, st.stream);
        if (bst == BLAST_OK && hipStreamSynchronize(st.stream) != hipSuccess) bst = BLAST_E_HIP;
        if (bst != BLAST_OK || !d->use_graphs) continue;
        std::vector<int> sizes;
        for (int b = 1; b < d->batch; b *= 2) sizes.push_back(b);
        sizes.push_back(d->batch);
        for (int b : sizes) {
            Graph g;
            g.batch = b;
            a = set_args(S, st, b);
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

extern "C" blast_status blast_server_wait(blast_server *S, uint64_t ticket, int32_t timeout_ms,
                                          blast_status *req_status, double *latency_ms) {
    if (!S) return blast::set_error("NULL argument"), BLAST_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] { return S->done.count(ticket) > 0; };
    if (timeout_ms < 0)
        S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        return blast::set_error("timeout"), BLAST_E_BUSY;
    const Done d = S->done[ticket];
    S->done.erase(ticket);
    if (req_status) *req_status = d.st;
    if (latency_ms) *latency_ms = d.lat_ms;
    return BLAST_OK;
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
