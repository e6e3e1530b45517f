// Host side of the batched sparse solver (kernel: gd_batch.hip).
//
// Ingest: per instance, couplings from a dense matrix or CSR, validated
// (finite, exactly symmetric, diagonal dropped), packed into one ELL list of
// dmax neighbours per spin; per-instance coupling scale s_k and field term
// h_1 = -g sqrt(rho_th) / s_k.  Run: items (instance, slice of T trajectories)
// are bin-packed onto as many workgroups as the GPU holds at once (longest
// processing time first, deterministic), the kernel variant is chosen by
// timing the candidates on the live state with dt = 0 (state unchanged), and
// the launch for a chunk of steps is captured once in a hipGraph and replayed.
#include "gd_batch_rt.h"
#include "gd_internal.h"
#include "gd_relabel.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <queue>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

namespace gd {

namespace {

#define GD_TRY(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return gd_fail(e_ == hipErrorOutOfMemory ? GD_E_OOM : GD_E_DEVICE,           \
                           (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

template <class T>
int dmalloc(T **p, size_t count) {
    *p = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return gd_fail(e == hipErrorOutOfMemory ? GD_E_OOM : GD_E_DEVICE, hipGetErrorString(e));
    }
    return GD_OK;
}

template <class T>
int upload(T **p, const std::vector<T> &v) {
    int rc = dmalloc(p, v.size());
    if (rc != GD_OK) return rc;
    if (!v.empty()) GD_TRY(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return GD_OK;
}

std::mutex g_btune_mu;
// (K, R, nmax, dmax, total, packed form + 2 uniform rates) -> cfg
std::map<std::tuple<int, int, int, int, long long, int>, int> g_btune;

}  // namespace

struct BatchSolver {
    int K = 0, dmax = 0, nmax = 0;
    gd_params prm{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<int> n;               // per instance
    std::vector<long long> spin_off;  // per instance, prefix sums of n
    std::vector<float> inv_s;
    std::vector<double> scale;
    long long total = 0;              // sum of n
    std::vector<float> eps_host;      // [total]
    // device constants
    int *d_n = nullptr;
    long long *d_spin = nullptr, *d_state = nullptr;
    float *d_inv_s = nullptr, *d_w = nullptr, *d_eps = nullptr, *d_h1 = nullptr, *d_g = nullptr;
    int *d_idx = nullptr;
    // packed neighbours (dmax <= 3, one coupling magnitude per instance):
    // [total][2] words and [K] magnitudes, or null when the batch does not qualify
    unsigned int *d_pack = nullptr;
    float *d_wmag = nullptr;
    bool packable = false;
    std::vector<unsigned int> pack_host;
    // spin labels of the per-instance-width variants, per (instance, groups
    // per gather instruction), computed once
    std::map<std::pair<int, int>, std::vector<int>> labels;
    bool no_field = true;             // every g_i = 0
    // state
    int R = 0;
    bool have_state = false;
    float *d_x = nullptr, *d_gam = nullptr, *d_D = nullptr;
    double *d_E = nullptr;
    double *d_best_E = nullptr;   // running best of a run's checks (no targets)
    int *d_best_r = nullptr;
    int *d_flags = nullptr;
    int8_t *d_spins = nullptr;
    // schedule
    BatchConfig cfg{};
    int nwg = 0;
    int *d_wg_off = nullptr, *d_items = nullptr;
    int *d_tlog = nullptr;            // per-instance item widths (variants with traj = 0)
    // their spin labels (kept across schedules; tw_key: the groups per gather
    // instruction of each instance they were made for)
    int *d_tw_label = nullptr, *d_tw_spin = nullptr;
    unsigned int *d_tw_pack = nullptr;
    std::vector<int> tw_key;
    hipGraphExec_t graph = nullptr;
    int graph_steps = -1;
    // stats
    int64_t steps_done = 0, spin_updates = 0;
    double run_seconds = 0.0;
    int diverged = 0;
    std::vector<double> targets;      // per instance (empty: none)
    std::vector<double> ttt;          // per instance seconds, < 0 if not reached
    std::vector<int64_t> ttt_steps;
    std::vector<double> best_E;
    std::vector<int> best_r;
    // time to target: device time of the gd_run calls since the last set-up
    // (an event at the start of each call, one after each check, one at the end)
    hipEvent_t ev_run0 = nullptr, ev_chk = nullptr, ev_end = nullptr;
    double clock_s = 0.0;
    // GD_F_PROFILE: an event pair around every persistent launch
    std::vector<hipEvent_t> prof_ev;
    double kernel_ms = 0.0;
    int64_t kernel_launches = 0;
};

namespace {

void free_schedule(BatchSolver *b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_steps = -1;
    if (b->d_wg_off) (void)hipFree(b->d_wg_off);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_tlog) (void)hipFree(b->d_tlog);
    b->d_wg_off = b->d_items = b->d_tlog = nullptr;
    b->nwg = 0;
}

void free_labels(BatchSolver *b) {
    if (b->d_tw_label) (void)hipFree(b->d_tw_label);
    if (b->d_tw_spin) (void)hipFree(b->d_tw_spin);
    if (b->d_tw_pack) (void)hipFree(b->d_tw_pack);
    b->d_tw_label = b->d_tw_spin = nullptr;
    b->d_tw_pack = nullptr;
    b->tw_key.clear();
}

void free_state(BatchSolver *b) {
    free_schedule(b);
    void *ps[] = {b->d_x, b->d_gam, b->d_D, b->d_E, b->d_best_E, b->d_best_r, b->d_flags, b->d_spins};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    b->d_x = b->d_gam = b->d_D = nullptr;
    b->d_E = b->d_best_E = nullptr;
    b->d_best_r = nullptr;
    b->d_flags = nullptr;
    b->d_spins = nullptr;
    b->have_state = false;
    b->R = 0;
}

BatchArgs make_args(BatchSolver *b, int steps, float dt) {
    BatchArgs a{};
    a.inst_n = b->d_n;
    a.inst_spin = b->d_spin;
    a.inst_state = b->d_state;
    a.inst_inv_s = b->d_inv_s;
    a.ell_idx = b->d_idx;
    a.ell_w = b->d_w;
    a.ell_pack = b->d_pack;
    a.inst_wmag = b->d_wmag;
    a.inst_tlog = b->d_tlog;
    a.tw_label = b->d_tw_label;
    a.tw_spin = b->d_tw_spin;
    a.tw_pack = b->d_tw_pack;
    a.eps = b->d_eps;
    a.h1 = b->d_h1;
    a.g = b->d_g;
    a.x = b->d_x;
    a.gam = b->d_gam;
    a.E = b->d_E;
    a.flags = b->d_flags;
    a.wg_off = b->d_wg_off;
    a.items = b->d_items;
    a.nslices = b->cfg.traj ? b->R / b->cfg.traj : 0;
    a.R = b->R;
    a.dmax = b->dmax;
    a.nmax = b->nmax;
    a.steps = steps;
    a.dt = dt;
    a.gamma_c = float(b->prm.gamma_c);
    a.rho_th = float(b->prm.rho_th);
    a.eps0 = b->eps_host.empty() ? 0.0f : b->eps_host[0];
    return a;
}

// one eps for every spin and no field: the variants without per-spin constants apply
bool uniform_rates(const BatchSolver *b) {
    if (!b->no_field || b->eps_host.empty()) return false;
    for (float e : b->eps_host)
        if (std::memcmp(&e, &b->eps_host[0], sizeof(float)) != 0) return false;
    return true;
}

// per-instance item width of the traj = 0 variants: the widest T = 2^t <= 64
// dividing R with T (n + 1) <= E NT + 64 and T n <= E NT (-1: none fits)
int width_log2(const BatchConfig &c, int n, int R) {
    const long long cap = batch_item_capacity(c);
    for (int t = 6; t >= 0; --t) {
        const long long T = 1LL << t;
        if (R % T == 0 && T * (n + 1) <= cap + 64 && T * n <= cap) return t;
    }
    return -1;
}

bool config_fits(const BatchSolver *b, const BatchConfig &c) {
    if (c.packed && !b->packable) return false;
    if (c.uniform && !uniform_rates(b)) return false;
    if (c.traj == 0) {
        if (width_log2(c, b->nmax, b->R) < 0) return false;
    } else {
        if (b->R % c.traj) return false;
        if ((long long)b->nmax * c.traj > (long long)c.slots * c.threads) return false;
    }
    return batch_lds_bytes(c, b->nmax, b->dmax) <= 160 * 1024;
}

// Spin labels of the per-instance-width variants (gather_relabel, per
// instance with G = 64 / T_k groups per gather instruction; the identity
// when G <= 2 or with GD_BATCH_RELABEL=0), computed on host threads, and the
// device arrays made from them: label of each spin, spin of each label, and
// the packed neighbour words in label order with labels as indices.
int build_labels(BatchSolver *b, const std::vector<int> &tl) {
    const char *env = std::getenv("GD_BATCH_RELABEL");
    const bool on = !(env && std::strcmp(env, "0") == 0);
    std::vector<int> key(b->K);
    for (int k = 0; k < b->K; ++k) key[k] = on ? 64 >> tl[k] : 1;
    if (b->d_tw_label && key == b->tw_key) return GD_OK;
    std::vector<std::pair<int, int>> todo;
    for (int k = 0; k < b->K; ++k)
        if (!b->labels.count({k, key[k]})) todo.push_back({k, key[k]});
    std::vector<std::vector<int>> got(todo.size());
    std::atomic<size_t> next{0};
    std::atomic<bool> failed{false};
    auto work = [&]() {
        for (size_t q; (q = next.fetch_add(1)) < todo.size();) {
            // an exception must not leave a worker thread (host memory)
            try {
                const int k = todo[q].first, g = todo[q].second, n = b->n[k];
                std::vector<int> nb((size_t)3 * n);
                for (int i = 0; i < n; ++i) {
                    const unsigned int *w = &b->pack_host[(size_t)(b->spin_off[k] + i) * 2];
                    nb[3 * i] = int(w[0] & 0xFFFFu);
                    nb[3 * i + 1] = int(w[0] >> 16);
                    nb[3 * i + 2] = int(w[1] & 0xFFFFu);
                }
                // blocks of G / 2 labels: the rows of one 32-lane pass of a gather
                got[q] = gather_relabel(n, nb, g, g / 2, uint64_t(k) * 64 + uint64_t(g), 12LL * n).label;
            } catch (...) {
                failed = true;
            }
        }
    };
    // up to 15 helper threads; the calling thread works too, and takes what
    // is left when no thread can be started
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const size_t nth = std::min<size_t>(hw, todo.size());
    std::vector<std::thread> pool;
    for (size_t t = 1; t < nth; ++t) {
        try {
            pool.emplace_back(work);
        } catch (...) {
            break;
        }
    }
    work();
    for (auto &t : pool) t.join();
    if (failed) return gd_fail(GD_E_OOM, "spin relabeling ran out of host memory");
    for (size_t q = 0; q < todo.size(); ++q) b->labels[todo[q]] = std::move(got[q]);
    std::vector<int> label(b->total), spin(b->total);
    std::vector<unsigned int> tpack((size_t)b->total * 2);
    for (int k = 0; k < b->K; ++k) {
        const std::vector<int> &L = b->labels[{k, on ? 64 >> tl[k] : 1}];
        const int n = b->n[k];
        const long long off = b->spin_off[k];
        auto relab = [&](unsigned int j) { return j < (unsigned)n ? (unsigned)L[j] : j; };   // n: the zero row
        for (int i = 0; i < n; ++i) {
            const int p = L[i];
            label[off + i] = p;
            spin[off + p] = i;
            const unsigned int *w = &b->pack_host[(size_t)(off + i) * 2];
            tpack[(size_t)(off + p) * 2] = relab(w[0] & 0xFFFFu) | (relab(w[0] >> 16) << 16);
            tpack[(size_t)(off + p) * 2 + 1] = relab(w[1] & 0xFFFFu) | (w[1] & 0xE0000000u);
        }
    }
    free_labels(b);
    int rc = upload(&b->d_tw_label, label);
    if (rc == GD_OK) rc = upload(&b->d_tw_spin, spin);
    if (rc == GD_OK) rc = upload(&b->d_tw_pack, tpack);
    if (rc == GD_OK) b->tw_key = key;
    return rc;
}

// Longest processing time first: items sorted by cost, each to the least
// loaded workgroup (ties -> lowest workgroup id).  Deterministic.
int build_schedule(BatchSolver *b, const BatchConfig &c) {
    free_schedule(b);
    b->cfg = c;
    int dev = 0, cus = 0, occ = 0;
    GD_TRY(hipGetDevice(&dev));
    GD_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GD_TRY(prepare_batch(c, b->nmax, b->dmax));
    // resident workgroups per CU (registers, LDS, threads), so that the bin
    // packing below spreads the items over workgroups that run at once
    occ = batch_occupancy(c, b->nmax, b->dmax);
    // items: (instance, slice of T trajectories); fixed T: item = k nslices + slice,
    // cost n_k; per-instance T_k: item = k R + first trajectory, cost T_k n_k
    std::vector<int> order;
    std::vector<long long> costs;
    if (c.traj) {
        const int nslices = b->R / c.traj;
        for (int k = 0; k < b->K; ++k)
            for (int sl = 0; sl < nslices; ++sl) {
                order.push_back(k * nslices + sl);
                costs.push_back(b->n[k]);
            }
    } else {
        std::vector<int> tl(b->K);
        for (int k = 0; k < b->K; ++k) {
            tl[k] = width_log2(c, b->n[k], b->R);
            if (tl[k] < 0) return gd_fail(GD_E_UNSUPPORTED, "instance too large for the batch kernel variant");
            for (int r0 = 0; r0 < b->R; r0 += 1 << tl[k]) {
                order.push_back(k * b->R + r0);
                costs.push_back((long long)b->n[k] << tl[k]);
            }
        }
        if (int rc = upload(&b->d_tlog, tl); rc != GD_OK) return rc;
        if (int rc = build_labels(b, tl); rc != GD_OK) return rc;
    }
    const long long nitems = (long long)order.size();
    int nwg = int(std::min<long long>((long long)cus * occ, nitems));
    // positions sorted by cost (longest first; stable, so deterministic)
    std::vector<long long> cost_of(order.size());
    {
        std::vector<int> pos(order.size());
        std::iota(pos.begin(), pos.end(), 0);
        std::stable_sort(pos.begin(), pos.end(), [&](int x, int y) { return costs[x] > costs[y]; });
        std::vector<int> sorted(order.size());
        for (size_t q = 0; q < pos.size(); ++q) {
            sorted[q] = order[pos[q]];
            cost_of[q] = costs[pos[q]];
        }
        order.swap(sorted);
    }
    typedef std::pair<long long, int> LW;   // (load, wg)
    std::priority_queue<LW, std::vector<LW>, std::greater<LW>> heap;
    for (int w = 0; w < nwg; ++w) heap.push({0, w});
    std::vector<std::vector<int>> lists(nwg);
    for (size_t q = 0; q < order.size(); ++q) {
        LW top = heap.top();
        heap.pop();
        lists[top.second].push_back(order[q]);
        heap.push({top.first + cost_of[q], top.second});
    }
    std::vector<int> off(nwg + 1, 0), items;
    items.reserve(nitems);
    for (int w = 0; w < nwg; ++w) {
        off[w] = int(items.size());
        items.insert(items.end(), lists[w].begin(), lists[w].end());
    }
    off[nwg] = int(items.size());
    int rc = upload(&b->d_wg_off, off);
    if (rc == GD_OK) rc = upload(&b->d_items, items);
    if (rc != GD_OK) return rc;
    b->nwg = nwg;
    return GD_OK;
}

int choose_config(BatchSolver *b) {
    std::vector<int> cands;
    for (int id = 0; id < batch_config_count(); ++id)
        if (config_fits(b, batch_config(id))) cands.push_back(id);
    if (cands.empty()) return gd_fail(GD_E_UNSUPPORTED, "no batch kernel variant fits this batch");
    if (const char *env = std::getenv("GD_BATCH_CONFIG")) {
        const int id = std::atoi(env);
        if (std::find(cands.begin(), cands.end(), id) == cands.end())
            return gd_fail(GD_E_INVALID_ARG, "GD_BATCH_CONFIG does not fit this batch");
        return build_schedule(b, batch_config(id));
    }
    auto key = std::make_tuple(b->K, b->R, b->nmax, b->dmax, b->total, int(b->packable) + 2 * int(uniform_rates(b)));
    const std::vector<long long> fkey{b->K, b->R, b->nmax, b->dmax, b->total,
                                      int(b->packable) + 2 * int(uniform_rates(b))};
    auto is_cand = [&](int id) { return std::find(cands.begin(), cands.end(), id) != cands.end(); };
    {
        // the cache file first (GD_AUTOTUNE_CACHE), then this process's table
        const int fid = tune_cache_lookup("batch", fkey);
        if (fid >= 0 && is_cand(fid)) {
            std::lock_guard<std::mutex> lk(g_btune_mu);
            g_btune[key] = fid;
            return build_schedule(b, batch_config(fid));
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_btune_mu);
        auto it = g_btune.find(key);
        if (it != g_btune.end() && is_cand(it->second)) return build_schedule(b, batch_config(it->second));
    }
    int best = cands[0];
    if (cands.size() > 1 && b->total * (long long)b->R >= (1 << 16)) {
        hipEvent_t e0, e1;
        GD_TRY(hipEventCreate(&e0));
        GD_TRY(hipEventCreate(&e1));
        float best_ms = 1e30f;
        for (int id : cands) {
            int rc = build_schedule(b, batch_config(id));
            if (rc != GD_OK) return rc;
            const BatchArgs a = make_args(b, 20, 0.0f);   // dt = 0: state unchanged
            GD_TRY(launch_batch(b->cfg, b->nwg, a, b->stream));
            // the fastest of three timed launches (variants a few per cent
            // apart swap places in single timings)
            for (int rep = 0; rep < 3; ++rep) {
                GD_TRY(hipEventRecord(e0, b->stream));
                GD_TRY(launch_batch(b->cfg, b->nwg, a, b->stream));
                GD_TRY(hipEventRecord(e1, b->stream));
                GD_TRY(hipEventSynchronize(e1));
                float ms = 0.0f;
                GD_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_ms) { best_ms = ms; best = id; }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    {
        std::lock_guard<std::mutex> lk(g_btune_mu);
        g_btune[key] = best;
    }
    tune_cache_store("batch", fkey, best);
    return build_schedule(b, batch_config(best));
}

bool finite_all(const float *p, size_t m) {
    for (size_t i = 0; i < m; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// caller buffer (host or device) -> host vector
int fetch(const BatchSolver *b, const float *src, size_t count, std::vector<float> &dst) {
    dst.resize(count);
    if (!count) return GD_OK;
    if (b->prm.flags & GD_F_DEVICE_PTRS) GD_TRY(hipMemcpy(dst.data(), src, count * 4, hipMemcpyDeviceToHost));
    else std::memcpy(dst.data(), src, count * 4);
    return GD_OK;
}

int alloc_state(BatchSolver *b, int R) {
    free_state(b);
    b->R = R;
    const size_t st = (size_t)b->total * R;
    int rc = dmalloc(&b->d_x, st);
    if (rc == GD_OK) rc = dmalloc(&b->d_gam, st);
    if (rc == GD_OK) rc = dmalloc(&b->d_D, st);
    if (rc == GD_OK) rc = dmalloc(&b->d_spins, st);
    if (rc == GD_OK) rc = dmalloc(&b->d_E, (size_t)b->K * R);
    if (rc == GD_OK) rc = dmalloc(&b->d_best_E, (size_t)b->K);
    if (rc == GD_OK) rc = dmalloc(&b->d_best_r, (size_t)b->K);
    if (rc == GD_OK) rc = dmalloc(&b->d_flags, (size_t)b->K * R);
    if (rc != GD_OK) {
        free_state(b);
        return rc;
    }
    std::vector<long long> soff(b->K);
    for (int k = 0; k < b->K; ++k) soff[k] = b->spin_off[k] * R;
    if (b->d_state) (void)hipFree(b->d_state);
    b->d_state = nullptr;
    if ((rc = upload(&b->d_state, soff)) != GD_OK) return rc;
    GD_TRY(hipMemset(b->d_flags, 0, (size_t)b->K * R * sizeof(int)));
    b->have_state = true;
    return GD_OK;
}

void reset_stats(BatchSolver *b) {
    b->steps_done = b->spin_updates = 0;
    b->run_seconds = 0.0;
    b->clock_s = 0.0;
    b->kernel_ms = 0.0;
    b->kernel_launches = 0;
    b->diverged = 0;
    b->ttt.assign(b->K, -1.0);
    b->ttt_steps.assign(b->K, -1);
    b->best_E.assign(b->K, HUGE_VAL);
    b->best_r.assign(b->K, -1);
}

int upload_state(BatchSolver *b, const float *psi, const float *gam) {
    const size_t st = (size_t)b->total * b->R;
    const hipMemcpyKind kind = (b->prm.flags & GD_F_DEVICE_PTRS) ? hipMemcpyDeviceToDevice
                                                                 : hipMemcpyHostToDevice;
    GD_TRY(hipMemcpy(b->d_x, psi, st * 4, kind));
    if (gam) {
        GD_TRY(hipMemcpy(b->d_gam, gam, st * 4, kind));
    } else {
        std::vector<float> g0(st, float(b->prm.gamma0));
        GD_TRY(hipMemcpy(b->d_gam, g0.data(), st * 4, hipMemcpyHostToDevice));
    }
    return GD_OK;
}

// energies of the current state (a launch with zero steps), per-instance best
int energies_now(BatchSolver *b, std::vector<double> &E) {
    const BatchArgs a = make_args(b, 0, float(b->prm.dt));
    GD_TRY(launch_batch(b->cfg, b->nwg, a, b->stream));
    E.resize((size_t)b->K * b->R);
    GD_TRY(hipMemcpyAsync(E.data(), b->d_E, E.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    GD_TRY(hipStreamSynchronize(b->stream));
    return GD_OK;
}

}  // namespace

int batch_create(BatchSolver **out, int count, const gd_instance *inst, int model, const gd_params *p) {
    *out = nullptr;
    if (count < 1 || !inst) return gd_fail(GD_E_INVALID_ARG, "count must be >= 1 and inst non-NULL");
    if (model != GD_ISING) return gd_fail(GD_E_UNSUPPORTED, "batched solver integrates the Ising model");
    if (p->integrator != GD_EULER) return gd_fail(GD_E_UNSUPPORTED, "batched solver uses Euler steps");
    if (p->precision != GD_PREC_FP32) return gd_fail(GD_E_UNSUPPORTED, "batched solver is FP32");
    if (p->noise_D != 0.0) return gd_fail(GD_E_UNSUPPORTED, "batched solver has no noise term");
    BatchSolver *b = new (std::nothrow) BatchSolver();
    if (!b) return gd_fail(GD_E_OOM, "host allocation failed");
    b->K = count;
    b->prm = *p;
    auto bail = [&](int rc) { batch_destroy(b); return rc; };
    // CSR per instance -> ELL
    std::vector<std::vector<std::pair<int, float>>> rows;
    std::vector<int> inst_of_row;
    std::vector<float> gvec;
    for (int k = 0; k < count; ++k) {
        const gd_instance &I = inst[k];
        const int n = I.n;
        if (n < 1 || n > 65535) return bail(gd_fail(GD_E_INVALID_ARG, "instance n out of range [1, 65535]"));
        std::vector<std::vector<std::pair<int, float>>> R(n);
        std::vector<float> tmp;
        if (I.J) {
            if (fetch(b, I.J, (size_t)n * n, tmp) != GD_OK) return bail(GD_E_DEVICE);
            if (!finite_all(tmp.data(), tmp.size())) return bail(gd_fail(GD_E_NONFINITE, "J has non-finite entries"));
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    if (i != j && tmp[(size_t)i * n + j] != 0.0f) R[i].push_back({j, tmp[(size_t)i * n + j]});
        } else {
            if (!I.row_ptr || !I.col || !I.val) return bail(gd_fail(GD_E_INVALID_ARG, "instance has neither J nor CSR"));
            if (b->prm.flags & GD_F_DEVICE_PTRS) return bail(gd_fail(GD_E_UNSUPPORTED, "CSR input must be host memory"));
            if (I.row_ptr[0] != 0) return bail(gd_fail(GD_E_INVALID_ARG, "CSR row_ptr[0] != 0"));
            for (int i = 0; i < n; ++i) {
                if (I.row_ptr[i + 1] < I.row_ptr[i]) return bail(gd_fail(GD_E_INVALID_ARG, "CSR row_ptr not monotone"));
                for (int q = I.row_ptr[i]; q < I.row_ptr[i + 1]; ++q) {
                    const int j = I.col[q];
                    const float v = I.val[q];
                    if (j < 0 || j >= n) return bail(gd_fail(GD_E_INVALID_ARG, "CSR column out of range"));
                    if (!std::isfinite(v)) return bail(gd_fail(GD_E_NONFINITE, "CSR value non-finite"));
                    if (j != i && v != 0.0f) R[i].push_back({j, v});
                }
            }
        }
        // symmetric, no duplicate columns
        std::map<std::pair<int, int>, float> m;
        for (int i = 0; i < n; ++i) {
            std::sort(R[i].begin(), R[i].end(), [](auto &x, auto &y) { return x.first < y.first; });
            for (size_t q = 0; q < R[i].size(); ++q) {
                if (q && R[i][q].first == R[i][q - 1].first)
                    return bail(gd_fail(GD_E_INVALID_ARG, "duplicate CSR column"));
                m[{i, R[i][q].first}] = R[i][q].second;
            }
        }
        double ss = 0.0;
        for (auto &kv : m) {
            auto it = m.find({kv.first.second, kv.first.first});
            if (it == m.end() || it->second != kv.second)
                return bail(gd_fail(GD_E_NOT_SYMMETRIC, "instance couplings are not symmetric"));
            ss += double(kv.second) * kv.second;
        }
        double s = p->j_scale > 0 ? p->j_scale : std::sqrt(ss / n);
        if (!(s > 0)) s = 1.0;
        b->scale.push_back(s);
        b->inv_s.push_back(float(1.0 / s));
        b->n.push_back(n);
        b->spin_off.push_back(b->total);
        b->total += n;
        b->nmax = std::max(b->nmax, n);
        for (int i = 0; i < n; ++i) {
            b->dmax = std::max<int>(b->dmax, int(R[i].size()));
            rows.push_back(std::move(R[i]));
        }
        std::vector<float> gk;
        if (I.g) {
            if (fetch(b, I.g, (size_t)n, gk) != GD_OK) return bail(GD_E_DEVICE);
            if (!finite_all(gk.data(), gk.size())) return bail(gd_fail(GD_E_NONFINITE, "g has non-finite entries"));
        } else {
            gk.assign(n, 0.0f);
        }
        for (float v : gk) b->no_field = b->no_field && v == 0.0f;
        gvec.insert(gvec.end(), gk.begin(), gk.end());
    }
    b->dmax = std::max(b->dmax, 1);
    std::vector<int> idx((size_t)b->total * b->dmax, 0);
    std::vector<float> w((size_t)b->total * b->dmax, 0.0f), h1(b->total);
    for (long long i = 0; i < b->total; ++i)
        for (size_t d = 0; d < rows[i].size(); ++d) {
            idx[(size_t)i * b->dmax + d] = rows[i][d].first;
            w[(size_t)i * b->dmax + d] = rows[i][d].second;
        }
    for (int k = 0; k < count; ++k)
        for (int i = 0; i < b->n[k]; ++i) {
            const long long q = b->spin_off[k] + i;
            h1[q] = float(-double(gvec[q]) * std::sqrt(p->rho_th) / b->scale[k]);
        }
    // packed neighbours: at most 3 per spin, indices below 2^16 - 1 and every
    // nonzero coupling of an instance of one magnitude (e.g. +-1 max-cut
    // couplings); each coupling becomes a neighbour index and a sign bit, a
    // missing one the index n_k of an all-zero amplitude row (one past the
    // instance's spins)
    std::vector<unsigned int> pack;
    std::vector<float> wmag(count, 1.0f);
    b->packable = b->dmax <= 3 && b->nmax < 65535;
    for (int k = 0; k < count && b->packable; ++k) {
        float mag = 0.0f;
        for (int i = 0; i < b->n[k] && b->packable; ++i)
            for (int d = 0; d < b->dmax; ++d) {
                const float v = w[(size_t)(b->spin_off[k] + i) * b->dmax + d];
                if (v == 0.0f) continue;
                if (mag == 0.0f) mag = std::fabs(v);
                else if (std::fabs(v) != mag) b->packable = false;
            }
        if (mag > 0.0f) wmag[k] = mag;
    }
    if (b->packable) {
        pack.assign((size_t)b->total * 2, 0u);
        for (int k = 0; k < count; ++k)
            for (int i = 0; i < b->n[k]; ++i) {
                const long long q = b->spin_off[k] + i;
                const unsigned int zero_row = (unsigned int)b->n[k];
                unsigned int id[3] = {zero_row, zero_row, zero_row}, neg[3] = {0u, 0u, 0u};
                for (int d = 0; d < b->dmax; ++d) {
                    const float v = w[(size_t)q * b->dmax + d];
                    if (v == 0.0f) continue;
                    id[d] = (unsigned int)idx[(size_t)q * b->dmax + d];
                    neg[d] = v < 0.0f ? 1u : 0u;
                }
                pack[(size_t)q * 2] = id[0] | (id[1] << 16);
                pack[(size_t)q * 2 + 1] = id[2] | (neg[2] << 29) | (neg[1] << 30) | (neg[0] << 31);
            }
    }
    b->eps_host.assign(b->total, float(p->eps));
    if (p->stream) {
        b->stream = static_cast<hipStream_t>(p->stream);
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(gd_fail(GD_E_DEVICE, "hipStreamCreate failed"));
        b->own_stream = true;
    }
    int rc = upload(&b->d_n, b->n);
    if (rc == GD_OK) rc = upload(&b->d_spin, b->spin_off);
    if (rc == GD_OK) rc = upload(&b->d_inv_s, b->inv_s);
    if (rc == GD_OK) rc = upload(&b->d_idx, idx);
    if (rc == GD_OK) rc = upload(&b->d_w, w);
    if (rc == GD_OK && b->packable) rc = upload(&b->d_pack, pack);
    b->pack_host = std::move(pack);
    if (rc == GD_OK && b->packable) rc = upload(&b->d_wmag, wmag);
    if (rc == GD_OK) rc = upload(&b->d_eps, b->eps_host);
    if (rc == GD_OK) rc = upload(&b->d_h1, h1);
    if (rc == GD_OK) rc = upload(&b->d_g, gvec);
    if (rc != GD_OK) return bail(rc);
    reset_stats(b);
    *out = b;
    return GD_OK;
}

void batch_destroy(BatchSolver *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_state(b);
    free_labels(b);
    void *ps[] = {b->d_n, b->d_spin, b->d_state, b->d_inv_s, b->d_w, b->d_eps, b->d_h1, b->d_g, b->d_idx,
                  b->d_pack, b->d_wmag};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    for (hipEvent_t e : {b->ev_run0, b->ev_chk, b->ev_end})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->prof_ev) (void)hipEventDestroy(e);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int batch_set_init(BatchSolver *b, int R, const float *psi0, const float *gamma0, const float *eps) {
    if (R < 1 || R > (1 << 16)) return gd_fail(GD_E_INVALID_ARG, "batch out of range");
    const size_t st = (size_t)b->total * R;
    std::vector<float> chk;
    int rc;
    if (eps) {
        if ((rc = fetch(b, eps, (size_t)b->total, chk)) != GD_OK) return rc;
        if (!finite_all(chk.data(), chk.size())) return gd_fail(GD_E_NONFINITE, "eps has non-finite entries");
        b->eps_host = chk;
    } else {
        b->eps_host.assign(b->total, float(b->prm.eps));
    }
    GD_TRY(hipMemcpy(b->d_eps, b->eps_host.data(), b->total * 4, hipMemcpyHostToDevice));
    if (psi0 && (rc = fetch(b, psi0, st, chk)) == GD_OK && !finite_all(chk.data(), chk.size()))
        return gd_fail(GD_E_NONFINITE, "psi0 has non-finite entries");
    if (gamma0 && (rc = fetch(b, gamma0, st, chk)) == GD_OK && !finite_all(chk.data(), chk.size()))
        return gd_fail(GD_E_NONFINITE, "gamma0 has non-finite entries");
    if ((rc = alloc_state(b, R)) != GD_OK) return rc;
    reset_stats(b);
    if (psi0) {
        if ((rc = upload_state(b, psi0, gamma0)) != GD_OK) return rc;
    } else {
        // default initial amplitudes U(-a, a) from SplitMix64 keyed by (seed, instance, r, i)
        std::vector<float> h(st);
        for (int k = 0; k < b->K; ++k)
            for (int r = 0; r < R; ++r)
                for (int i = 0; i < b->n[k]; ++i) {
                    uint64_t z = b->prm.seed ^ (0x9E3779B97F4A7C15ull * (uint64_t(k) * 1000003ull + 1));
                    z += 0x9E3779B97F4A7C15ull * (uint64_t(r) * 65537ull + uint64_t(i) + 1);
                    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                    z ^= z >> 31;
                    const double u = double(z >> 11) * (1.0 / 9007199254740992.0);
                    h[(size_t)b->spin_off[k] * R + (size_t)r * b->n[k] + i] = float(b->prm.init_amp * (2 * u - 1));
                }
        const uint32_t saved = b->prm.flags;
        b->prm.flags &= ~GD_F_DEVICE_PTRS;
        rc = upload_state(b, h.data(), nullptr);
        b->prm.flags = saved;
        if (rc == GD_OK && gamma0) {
            const hipMemcpyKind kind = (b->prm.flags & GD_F_DEVICE_PTRS) ? hipMemcpyDeviceToDevice
                                                                         : hipMemcpyHostToDevice;
            GD_TRY(hipMemcpy(b->d_gam, gamma0, st * 4, kind));
        }
        if (rc != GD_OK) return rc;
    }
    return choose_config(b);
}

int batch_run(BatchSolver *b, int R, int64_t steps) {
    if (steps < 0) return gd_fail(GD_E_INVALID_ARG, "steps must be >= 0");
    int rc;
    if (!b->have_state) {
        if ((rc = batch_set_init(b, R, nullptr, nullptr, nullptr)) != GD_OK) return rc;
    } else if (R != b->R) {
        return gd_fail(GD_E_INVALID_ARG, "batch differs from the current number of trajectories");
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int ci = b->prm.check_interval;
    const bool track = !b->targets.empty();
    const bool clocked = track && ci > 0;
    if (clocked) {
        for (hipEvent_t *e : {&b->ev_run0, &b->ev_chk, &b->ev_end})
            if (!*e) GD_TRY(hipEventCreate(e));
        GD_TRY(hipEventRecord(b->ev_run0, b->stream));
    }
    const double clock0 = b->clock_s;
    // Without targets (no time to record) the best of the checks is kept on
    // the device and read back once, at the end of the run.
    const bool deferred = ci > 0 && !track;
    if (deferred) {
        GD_TRY(hipMemcpyAsync(b->d_best_E, b->best_E.data(), b->K * sizeof(double), hipMemcpyHostToDevice,
                              b->stream));
        GD_TRY(hipMemcpyAsync(b->d_best_r, b->best_r.data(), b->K * sizeof(int), hipMemcpyHostToDevice,
                              b->stream));
    }
    const bool timed = (b->prm.flags & GD_F_PROFILE) != 0;
    size_t nprof = 0;   // event pairs used by this call
    int64_t done = 0;
    std::vector<double> E;
    while (done < steps) {
        const int64_t chunk = (ci > 0) ? std::min<int64_t>(ci, steps - done) : steps - done;
        const int cs = int(std::min<int64_t>(chunk, 1 << 30));
        if (b->graph_steps != cs) {
            // capture the persistent launch for `cs` steps once, replay it per chunk
            if (b->graph) (void)hipGraphExecDestroy(b->graph);
            b->graph = nullptr;
            hipGraph_t g = nullptr;
            GD_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            const BatchArgs a = make_args(b, cs, float(b->prm.dt));
            hipError_t le = launch_batch(b->cfg, b->nwg, a, b->stream);
            hipError_t ce = hipStreamEndCapture(b->stream, &g);
            if (le != hipSuccess || ce != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return gd_fail(GD_E_DEVICE, hipGetErrorString(le != hipSuccess ? le : ce));
            }
            hipError_t ie = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) return gd_fail(GD_E_DEVICE, hipGetErrorString(ie));
            b->graph_steps = cs;
        }
        if (timed) {
            while (b->prof_ev.size() < 2 * nprof + 2) {
                hipEvent_t e;
                GD_TRY(hipEventCreate(&e));
                b->prof_ev.push_back(e);
            }
            GD_TRY(hipEventRecord(b->prof_ev[2 * nprof], b->stream));
        }
        GD_TRY(hipGraphLaunch(b->graph, b->stream));
        if (timed) GD_TRY(hipEventRecord(b->prof_ev[2 * nprof++ + 1], b->stream));
        done += cs;
        b->steps_done += cs;
        b->spin_updates += (int64_t)b->total * b->R * cs;
        if (deferred) {
            GD_TRY(launch_batch_best(b->d_E, b->K, b->R, b->d_best_E, b->d_best_r, b->stream));
        } else if (ci > 0) {
            E.resize((size_t)b->K * b->R);
            GD_TRY(hipMemcpyAsync(E.data(), b->d_E, E.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  b->stream));
            if (clocked) GD_TRY(hipEventRecord(b->ev_chk, b->stream));
            GD_TRY(hipStreamSynchronize(b->stream));
            float ms = 0.0f;
            if (clocked) GD_TRY(hipEventElapsedTime(&ms, b->ev_run0, b->ev_chk));
            const double now = clock0 + ms * 1e-3;
            bool all = true;
            for (int k = 0; k < b->K; ++k) {
                for (int r = 0; r < b->R; ++r) {
                    const double e = E[(size_t)k * b->R + r];
                    if (e < b->best_E[k]) { b->best_E[k] = e; b->best_r[k] = r; }
                }
                if (track) {
                    if (b->ttt[k] < 0 && b->best_E[k] <= b->targets[k]) {
                        b->ttt[k] = now;
                        b->ttt_steps[k] = b->steps_done;
                    }
                    all = all && b->ttt[k] >= 0;
                }
            }
            if (track && all && b->prm.has_target) break;   // every instance reached its target
        }
    }
    if (deferred) {
        GD_TRY(hipMemcpyAsync(b->best_E.data(), b->d_best_E, b->K * sizeof(double), hipMemcpyDeviceToHost,
                              b->stream));
        GD_TRY(hipMemcpyAsync(b->best_r.data(), b->d_best_r, b->K * sizeof(int), hipMemcpyDeviceToHost,
                              b->stream));
    }
    if (clocked) GD_TRY(hipEventRecord(b->ev_end, b->stream));
    GD_TRY(hipStreamSynchronize(b->stream));
    b->run_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (clocked) {
        float ms = 0.0f;
        GD_TRY(hipEventElapsedTime(&ms, b->ev_run0, b->ev_end));
        b->clock_s += ms * 1e-3;
    }
    for (size_t q = 0; q < nprof; ++q) {
        float ms = 0.0f;
        GD_TRY(hipEventElapsedTime(&ms, b->prof_ev[2 * q], b->prof_ev[2 * q + 1]));
        b->kernel_ms += ms;
        b->kernel_launches += 1;
    }
    std::vector<int> fl((size_t)b->K * b->R);
    GD_TRY(hipMemcpy(fl.data(), b->d_flags, fl.size() * sizeof(int), hipMemcpyDeviceToHost));
    b->diverged = int(std::count_if(fl.begin(), fl.end(), [](int v) { return v != 0; }));
    if (b->diverged) return gd_fail(GD_E_DIVERGED, "trajectories became non-finite");
    return GD_OK;
}

int batch_energy(BatchSolver *b, double *E, int32_t *best) {
    if (!b->have_state) return gd_fail(GD_E_STATE, "no state: call gd_set_init or gd_run first");
    if (!E) return gd_fail(GD_E_INVALID_ARG, "E is NULL");
    std::vector<double> h;
    int rc = energies_now(b, h);
    if (rc != GD_OK) return rc;
    if (b->prm.flags & GD_F_DEVICE_PTRS) GD_TRY(hipMemcpy(E, b->d_E, h.size() * 8, hipMemcpyDeviceToDevice));
    else std::memcpy(E, h.data(), h.size() * 8);
    if (best) {
        std::vector<int32_t> bi(b->K);
        for (int k = 0; k < b->K; ++k) {
            int arg = 0;
            for (int r = 1; r < b->R; ++r)
                if (h[(size_t)k * b->R + r] < h[(size_t)k * b->R + arg]) arg = r;
            bi[k] = arg;
        }
        if (b->prm.flags & GD_F_DEVICE_PTRS) GD_TRY(hipMemcpy(best, bi.data(), b->K * 4, hipMemcpyHostToDevice));
        else std::memcpy(best, bi.data(), b->K * 4);
    }
    return GD_OK;
}

int batch_spins(BatchSolver *b, void *out, int fmt) {
    if (!b->have_state) return gd_fail(GD_E_STATE, "no state");
    if (fmt != GD_SPINS_I8) return gd_fail(GD_E_UNSUPPORTED, "batched solver returns int8 spins");
    const long long st = b->total * b->R;
    // one plane of st spins: discretise as a single trajectory of length st
    std::vector<int> dummy(1, 0);
    int *d_flag = nullptr;
    int rc = dmalloc(&d_flag, 1);
    if (rc != GD_OK) return rc;
    hipError_t e = launch_discretise(b->d_x, b->d_D, nullptr, OP_F32, RO_SIGN, 0, b->d_spins, nullptr,
                                     nullptr, d_flag, int(st), 1, int(st), 1, 1, st, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, b->d_spins, st, (b->prm.flags & GD_F_DEVICE_PTRS) ? hipMemcpyDeviceToDevice
                                                                                 : hipMemcpyDeviceToHost,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d_flag);
    if (e != hipSuccess) return gd_fail(GD_E_DEVICE, hipGetErrorString(e));
    return GD_OK;
}

int batch_get_state(BatchSolver *b, float *psi, float *gamma, int64_t *step) {
    if (!b->have_state) return gd_fail(GD_E_STATE, "no state");
    const size_t st = (size_t)b->total * b->R;
    const hipMemcpyKind kind = (b->prm.flags & GD_F_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    GD_TRY(hipStreamSynchronize(b->stream));
    if (psi) GD_TRY(hipMemcpy(psi, b->d_x, st * 4, kind));
    if (gamma) GD_TRY(hipMemcpy(gamma, b->d_gam, st * 4, kind));
    if (step) *step = b->steps_done;
    return GD_OK;
}

int batch_set_state(BatchSolver *b, int R, const float *psi, const float *gamma, int64_t step) {
    if (!psi || !gamma) return gd_fail(GD_E_INVALID_ARG, "psi and gamma are required");
    if (R < 1 || R > (1 << 16) || step < 0) return gd_fail(GD_E_INVALID_ARG, "bad batch or step");
    const size_t st = (size_t)b->total * R;
    std::vector<float> chk;
    int rc;
    if ((rc = fetch(b, psi, st, chk)) != GD_OK) return rc;
    if (!finite_all(chk.data(), chk.size())) return gd_fail(GD_E_NONFINITE, "psi has non-finite entries");
    if ((rc = fetch(b, gamma, st, chk)) != GD_OK) return rc;
    if (!finite_all(chk.data(), chk.size())) return gd_fail(GD_E_NONFINITE, "gamma has non-finite entries");
    if (!b->have_state || R != b->R) {
        if ((rc = alloc_state(b, R)) != GD_OK) return rc;
        reset_stats(b);
        if ((rc = upload_state(b, psi, gamma)) != GD_OK) return rc;
        if ((rc = choose_config(b)) != GD_OK) return rc;
    } else if ((rc = upload_state(b, psi, gamma)) != GD_OK) {
        return rc;
    }
    GD_TRY(hipMemset(b->d_flags, 0, (size_t)b->K * R * sizeof(int)));
    b->steps_done = step;
    return GD_OK;
}

int batch_trajectory_status(BatchSolver *b, int32_t *out, int64_t count) {
    if (b->R < 1) return gd_fail(GD_E_STATE, "no state: call gd_set_init first");
    if (count != (int64_t)b->K * b->R)
        return gd_fail(GD_E_INVALID_ARG, "count must be instances x trajectories");
    static_assert(sizeof(int) == sizeof(int32_t), "flag words are 32-bit");
    GD_TRY(hipStreamSynchronize(b->stream));
    GD_TRY(hipMemcpy(out, b->d_flags, (size_t)count * sizeof(int), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < count; ++i) out[i] = out[i] != 0;
    return GD_OK;
}

int batch_stats(BatchSolver *b, gd_run_stats *out) {
    out->batch = b->R;
    out->steps_done = b->steps_done;
    out->spin_updates = b->spin_updates;
    out->run_seconds = b->run_seconds;
    out->kernel_ms = b->kernel_ms;
    out->kernel_launches = b->kernel_launches;
    out->diverged = b->diverged;
    int reached = !b->targets.empty();
    double t = 0.0;
    int64_t s = 0;
    for (int k = 0; k < b->K && reached; ++k) {
        if (b->ttt[k] < 0) reached = 0;
        t = std::max(t, b->ttt[k]);
        s = std::max(s, b->ttt_steps[k]);
    }
    out->target_reached = reached;
    out->ttt_seconds = reached ? t : 0.0;
    out->ttt_steps = reached ? s : 0;
    double be = HUGE_VAL;
    int bi = -1;
    for (int k = 0; k < b->K; ++k)
        if (b->best_E[k] < be) { be = b->best_E[k]; bi = b->best_r[k]; }
    out->best_energy = be;
    out->best_index = bi;
    out->kernel_config = b->cfg.id;
    return GD_OK;
}

int batch_set_targets(BatchSolver *b, const double *targets) {
    if (!targets) {
        b->targets.clear();
        return GD_OK;
    }
    b->targets.assign(targets, targets + b->K);
    b->ttt.assign(b->K, -1.0);
    b->ttt_steps.assign(b->K, -1);
    return GD_OK;
}

int batch_ttt(BatchSolver *b, double *seconds, int64_t *steps, double *best_energy) {
    for (int k = 0; k < b->K; ++k) {
        if (seconds) seconds[k] = b->ttt.empty() ? -1.0 : b->ttt[k];
        if (steps) steps[k] = b->ttt_steps.empty() ? -1 : b->ttt_steps[k];
        if (best_energy) best_energy[k] = b->best_E[k];
    }
    return GD_OK;
}

int batch_count(const BatchSolver *b) { return b->K; }

int batch_view(BatchSolver *b, BatchView *v) {
    v->K = b->K;
    v->dmax = b->dmax;
    v->nmax = b->nmax;
    v->R = b->R;
    v->total = b->total;
    v->d_n = b->d_n;
    v->d_spin = b->d_spin;
    v->d_state = b->d_state;
    v->d_inv_s = b->d_inv_s;
    v->d_idx = b->d_idx;
    v->d_w = b->d_w;
    v->d_eps = b->d_eps;
    v->d_x = b->d_x;
    v->d_gam = b->d_gam;
    v->stream = b->stream;
    v->eps0 = b->prm.eps;
    v->gamma0 = b->prm.gamma0;
    v->amp = b->prm.init_amp;
    return GD_OK;
}

int batch_prepare_state(BatchSolver *b, int R) {
    if (R < 1 || R > (1 << 16)) return gd_fail(GD_E_INVALID_ARG, "batch out of range");
    int rc = alloc_state(b, R);
    if (rc != GD_OK) return rc;
    reset_stats(b);
    return GD_OK;
}

int batch_finish_init(BatchSolver *b) {
    GD_TRY(hipStreamSynchronize(b->stream));
    GD_TRY(hipMemcpy(b->eps_host.data(), b->d_eps, b->total * 4, hipMemcpyDeviceToHost));
    return choose_config(b);
}
double batch_scale(const BatchSolver *b, int k) { return b->scale[k]; }

}  // namespace gd
