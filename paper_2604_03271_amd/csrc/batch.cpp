// batch.cpp -- the batched path (many spectra, every K, advancing together) and
// the served path (continuous batching of a request stream).
//
// Both keep a pool of (spectrum, K) groups on the device.  Per tempering stage
// the pool issues one stage launch for every group and one move launch per tile
// bucket (groups with the same peak kind, noise kind and tile).  A spectrum's
// tile depends on its own shape only, and its random streams on its own seed and
// uid, so a spectrum gets bit-identical results alone, in a batch, or in the
// server's mix.  The batched path captures the launches of one stage in a
// hipGraph and replays it; finished groups turn into no-ops inside the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "host_common.hpp"

namespace smc {
namespace {

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// First-fit allocator of offsets inside one device allocation.
struct BlockAllocator {
    size_t size = 0;
    std::map<size_t, size_t> free_list;  // offset -> bytes
    void init(size_t n) {
        size = n;
        free_list.clear();
        if (n) free_list[0] = n;
    }
    bool alloc(size_t n, size_t& off) {
        n = align256(n);
        for (auto it = free_list.begin(); it != free_list.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_list.erase(it);
                if (rest) free_list[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align256(n);
        auto it = free_list.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_list.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_list.erase(next);
        }
        if (it != free_list.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_list.erase(it);
            }
        }
    }
};

// One spectrum of the pool with all its candidate K.
struct Entry {
    uint64_t id = 0;
    Spectrum spec;
    smc_options opt{};
    Tile tile{};
    double econst = 0.0;
    int ng = 0;
    size_t off = 0, bytes = 0;          // device block
    GroupState* d_states = nullptr;
    std::vector<GroupDesc> groups;      // host copies
    std::chrono::steady_clock::time_point t_submit;
    bool started = false;               // stage 0 launched
};

size_t entry_bytes(const smc_problem& p, const smc_options& o) {
    const int ng = p.k_max - p.k_min + 1;
    return spectrum_bytes(p, o) + align256(sizeof(GroupState) * ng) + 4096;
}

// Lay out one entry inside [base, base + bytes): states first (or at `states`, a slot of a
// table outside the block), then the spectrum's buffers.
bool carve_entry(Entry& e, const smc_options& o, void* base, GroupState* states = nullptr) {
    Arena a{base, e.bytes, 0};
    e.d_states = states ? states : static_cast<GroupState*>(a.take(sizeof(GroupState) * e.ng));
    if (!e.d_states) return false;
    std::vector<PendingCopy> copies;
    e.groups.clear();
    if (!describe_spectrum(e.spec, o, a, e.d_states, 0, e.groups, copies)) return false;
    return true;
}

hipError_t upload_entry(const Entry& e, hipStream_t s, std::vector<std::vector<char>>& keep) {
    hipError_t err = hipMemcpyAsync(const_cast<float*>(e.groups[0].x), e.spec.xf.data(),
                                    sizeof(float) * e.spec.prob.n_points, hipMemcpyHostToDevice, s);
    if (err != hipSuccess) return err;
    err = hipMemcpyAsync(const_cast<float*>(e.groups[0].y), e.spec.yf.data(), sizeof(float) * e.spec.prob.n_points,
                         hipMemcpyHostToDevice, s);
    if (err != hipSuccess) return err;
    if (!e.spec.mref_f.empty()) {   // XRD reference positions
        err = hipMemcpyAsync(const_cast<float*>(e.groups[0].mu_ref), e.spec.mref_f.data(),
                             sizeof(float) * e.spec.mref_f.size(), hipMemcpyHostToDevice, s);
        if (err != hipSuccess) return err;
    }
    std::vector<GroupState> zero(e.ng);
    keep.emplace_back(reinterpret_cast<const char*>(zero.data()),
                      reinterpret_cast<const char*>(zero.data()) + sizeof(GroupState) * e.ng);
    err = hipMemcpyAsync(e.d_states, keep.back().data(), sizeof(GroupState) * e.ng, hipMemcpyHostToDevice, s);
    if (err != hipSuccess) return err;
    return upload_group_tables(e.spec, e.groups, 0, e.groups.size(), s, keep);
}

struct Bucket {
    int pk = 0, nz = 0;
    Tile tile{};
    int work_off = 0, work_cnt = 0;
    size_t lds_move = 0, lds_energy = 0;
};

// Device-side view of the pool: descriptors of every group and the move work of every bucket.
struct PoolView {
    std::vector<GroupDesc> groups;
    std::vector<int> group_entry;
    std::vector<int> group_bucket;
    std::vector<Bucket> buckets;
    std::vector<MoveWork> work;
    GroupDesc* d_groups = nullptr;
    MoveWork* d_work = nullptr;
    size_t cap_groups = 0, cap_work = 0;

    void release() {
        if (d_groups) (void)hipFree(d_groups);
        if (d_work) (void)hipFree(d_work);
        d_groups = nullptr;
        d_work = nullptr;
        cap_groups = cap_work = 0;
    }

    // Rebuild from the entries (heaviest buckets and groups first) and upload.  With `keep`
    // (one flag per group of the entries, in order) only the flagged groups enter the pool.
    smc_status rebuild(const std::vector<Entry*>& entries, hipStream_t s, const std::vector<char>* keep = nullptr) {
        groups.clear();
        group_entry.clear();
        group_bucket.clear();
        buckets.clear();
        work.clear();
        std::map<std::tuple<int, int, int, int>, std::vector<int>> by_tile;
        size_t flat = 0;
        for (size_t ei = 0; ei < entries.size(); ++ei) {
            const Entry& e = *entries[ei];
            for (int k = 0; k < e.ng; ++k) {
                if (keep && !(*keep)[flat++]) continue;
                const int gi = static_cast<int>(groups.size());
                groups.push_back(e.groups[k]);
                group_entry.push_back(static_cast<int>(ei));
                by_tile[{e.spec.prob.peak_kind, e.spec.prob.noise_kind, e.tile.lc, e.tile.pi}].push_back(gi);
            }
        }
        for (auto& kv : by_tile) {
            Bucket b;
            b.pk = std::get<0>(kv.first);
            b.nz = std::get<1>(kv.first);
            const Entry& e0 = *entries[group_entry[kv.second.front()]];
            b.tile = e0.tile;
            std::vector<int> gs = kv.second;
            // heaviest first: cost ~ chains * d * points
            std::stable_sort(gs.begin(), gs.end(), [&](int a, int c) {
                const GroupDesc &ga = groups[a], &gc = groups[c];
                return static_cast<double>(ga.M) * ga.d * ga.n > static_cast<double>(gc.M) * gc.d * gc.n;
            });
            std::vector<int> chains(groups.size(), 0);
            int dmax = 1;
            for (int g : gs) {
                chains[g] = groups[g].M;
                dmax = std::max(dmax, groups[g].d);
            }
            b.work_off = static_cast<int>(work.size());
            build_work(gs, chains, b.tile, work);
            b.work_cnt = static_cast<int>(work.size()) - b.work_off;
            b.lds_move = move_lds_bytes(b.tile, dmax, b.pk, b.nz);
            b.lds_energy = energy_lds_bytes(b.tile, dmax);
            buckets.push_back(b);
        }
        group_bucket.assign(groups.size(), -1);
        for (size_t bi = 0; bi < buckets.size(); ++bi)
            for (int q = buckets[bi].work_off; q < buckets[bi].work_off + buckets[bi].work_cnt; ++q)
                group_bucket[work[q].group] = static_cast<int>(bi);
        if (groups.size() > cap_groups) {
            if (d_groups) (void)hipFree(d_groups);
            cap_groups = std::max<size_t>(groups.size() * 2, 64);
            if (hipMalloc(&d_groups, sizeof(GroupDesc) * cap_groups) != hipSuccess) return SMC_ENOMEM;
        }
        if (work.size() > cap_work) {
            if (d_work) (void)hipFree(d_work);
            cap_work = std::max<size_t>(work.size() * 2, 256);
            if (hipMalloc(&d_work, sizeof(MoveWork) * cap_work) != hipSuccess) return SMC_ENOMEM;
        }
        if (!groups.empty() &&
            hipMemcpyAsync(d_groups, groups.data(), sizeof(GroupDesc) * groups.size(), hipMemcpyHostToDevice, s) !=
                hipSuccess)
            return SMC_EDEVICE;
        if (!work.empty() &&
            hipMemcpyAsync(d_work, work.data(), sizeof(MoveWork) * work.size(), hipMemcpyHostToDevice, s) != hipSuccess)
            return SMC_EDEVICE;
        return SMC_OK;
    }

    // Stage 0 of the groups whose entry index is in `fresh` (draws, then energies per bucket).
    smc_status stage0(const std::vector<char>& fresh, hipStream_t s, std::vector<MoveWork>& scratch,
                      MoveWork*& d_scratch, size_t& cap_scratch) {
        scratch.clear();
        std::vector<std::pair<int, int>> energy_ranges;  // per bucket: [off, cnt) in scratch
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            if (!fresh[group_entry[gi]]) continue;
            const GroupDesc& g = groups[gi];
            const int64_t n = static_cast<int64_t>(g.P) * g.d;
            for (int64_t t0 = 0; t0 < n; t0 += 256)
                scratch.push_back(
                    MoveWork{static_cast<int>(gi), static_cast<int>(t0), static_cast<int>(std::min<int64_t>(256, n - t0)), 0});
        }
        const int n_draw = static_cast<int>(scratch.size());
        std::vector<int> chains(groups.size(), 0);
        for (size_t gi = 0; gi < groups.size(); ++gi) chains[gi] = groups[gi].P;
        for (size_t bi = 0; bi < buckets.size(); ++bi) {
            std::vector<int> mine;
            for (size_t gi = 0; gi < groups.size(); ++gi)
                if (fresh[group_entry[gi]] && group_bucket[gi] == static_cast<int>(bi)) mine.push_back(static_cast<int>(gi));
            const int off = static_cast<int>(scratch.size());
            build_work(mine, chains, buckets[bi].tile, scratch);
            energy_ranges.emplace_back(off, static_cast<int>(scratch.size()) - off);
        }
        if (scratch.empty()) return SMC_OK;
        if (scratch.size() > cap_scratch) {
            if (d_scratch) (void)hipFree(d_scratch);
            cap_scratch = scratch.size() * 2;
            if (hipMalloc(&d_scratch, sizeof(MoveWork) * cap_scratch) != hipSuccess) return SMC_ENOMEM;
        }
        if (hipMemcpyAsync(d_scratch, scratch.data(), sizeof(MoveWork) * scratch.size(), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            launch_draw_items(d_groups, d_scratch, n_draw, s) != hipSuccess)
            return SMC_EDEVICE;
        for (size_t bi = 0; bi < buckets.size(); ++bi) {
            const Bucket& b = buckets[bi];
            const void* efn = kernels().energy[b.pk][b.nz][b.tile.lc][b.tile.pi];
            if (launch_tiled(efn, b.tile, energy_ranges[bi].second, b.lds_energy, d_groups,
                             d_scratch + energy_ranges[bi].first, s) != hipSuccess)
                return SMC_EDEVICE;
        }
        // the scratch list must stay valid until the launches have read it
        return hipStreamSynchronize(s) == hipSuccess ? SMC_OK : SMC_EDEVICE;
    }

    // One tempering stage of every group.
    hipError_t launch_stage_all(hipStream_t s) const {
        if (groups.empty()) return hipSuccess;
        int max_p = 1, max_m = 1, max_d = 1;
        for (const GroupDesc& g : groups) {
            max_p = std::max(max_p, g.P);
            max_m = std::max(max_m, g.M);
            max_d = std::max(max_d, g.d);
        }
        hipError_t e = launch_stage(StageLaunch{d_groups, static_cast<int>(groups.size()), max_p, max_m, max_d}, s);
        if (e != hipSuccess) return e;
        for (const Bucket& b : buckets) {
            const void* mfn = kernels().move[b.pk][b.nz][b.tile.lc][b.tile.pi];
            e = launch_tiled(mfn, b.tile, b.work_cnt, b.lds_move, d_groups, d_work + b.work_off, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

// Copy every group's state to the host: one transfer per entry (its states are contiguous),
// in the pool's group order.
hipError_t copy_states(const PoolView& view, const std::vector<Entry*>& entries, std::vector<GroupState>& out,
                       hipStream_t s) {
    out.resize(view.groups.size());
    size_t gi = 0;
    for (const Entry* e : entries) {
        hipError_t err = hipMemcpyAsync(&out[gi], e->d_states, sizeof(GroupState) * e->ng, hipMemcpyDeviceToHost, s);
        if (err != hipSuccess) return err;
        gi += e->ng;
    }
    return hipSuccess;
}

Tile entry_tile(const smc_problem& p, const smc_options& o) {
    const int M = o.waste_free ? o.n_particles / o.n_moves : o.n_particles;
    const int64_t chains = static_cast<int64_t>(p.k_max - p.k_min + 1) * M;
    return choose_tile(p, chains, o.lanes_per_chain);
}

}  // namespace
}  // namespace smc

using namespace smc;

// ============================================================================ batched path

extern "C" smc_status smc_batch_run(const smc_problem* probs, int32_t n, const smc_options* opt, double* logz_out) {
    if (!probs || n < 1 || !opt || !logz_out) return SMC_EINVAL;
    for (int i = 0; i < n; ++i) {
        const smc_status st = validate(&probs[i], opt);
        if (st != SMC_OK) return st;
        if (!tile_has_kernels(probs[i], entry_tile(probs[i], *opt))) return SMC_EINVAL;
    }
    if (!device_ok()) return SMC_EDEVICE;

    hipStream_t s = static_cast<hipStream_t>(opt->hip_stream);
    bool own = false;
    if (!s) {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return SMC_EDEVICE;
        own = true;
    }
    // one device block: the state table of every group (entries in order, so one copy reads
    // them all), then the entries
    std::vector<std::unique_ptr<Entry>> entries(n);
    size_t ngroups = 0;
    for (int i = 0; i < n; ++i) ngroups += probs[i].k_max - probs[i].k_min + 1;
    size_t total = align256(sizeof(GroupState) * ngroups);
    for (int i = 0; i < n; ++i) {
        entries[i] = std::make_unique<Entry>();
        Entry& e = *entries[i];
        e.opt = *opt;
        e.spec.assign(probs[i]);
        e.ng = probs[i].k_max - probs[i].k_min + 1;
        e.tile = entry_tile(probs[i], *opt);
        e.econst = energy_constant(e.spec.prob);
        e.bytes = align256(entry_bytes(probs[i], *opt));
        e.off = total;
        total += e.bytes;
    }
    void* dmem = nullptr;
    PoolView view;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    MoveWork* d_scratch = nullptr;
    size_t cap_scratch = 0;
    smc_status status = SMC_OK;
    auto drop_graph = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    };
    auto cleanup = [&]() {
        drop_graph();
        (void)hipStreamSynchronize(s);
        view.release();
        if (d_scratch) (void)hipFree(d_scratch);
        if (dmem) (void)hipFree(dmem);
        if (own) (void)hipStreamDestroy(s);
    };
    if (hipMalloc(&dmem, total) != hipSuccess) {
        cleanup();
        return SMC_ENOMEM;
    }
    GroupState* d_states = static_cast<GroupState*>(dmem);
    std::vector<Entry*> ptrs;
    std::vector<std::vector<char>> keep;
    size_t first = 0;
    for (auto& e : entries) {
        if (!carve_entry(*e, *opt, static_cast<char*>(dmem) + e->off, d_states + first) ||
            upload_entry(*e, s, keep) != hipSuccess) {
            cleanup();
            return SMC_EDEVICE;
        }
        first += e->ng;
        ptrs.push_back(e.get());
    }
    status = view.rebuild(ptrs, s);
    std::vector<MoveWork> scratch;
    if (status == SMC_OK) status = view.stage0(std::vector<char>(n, 1), s, scratch, d_scratch, cap_scratch);
    keep.clear();
    if (status != SMC_OK) {
        cleanup();
        return status;
    }

    // One stage of the pool (the stage pipeline over every group, one move launch per tile
    // bucket) captured in a graph and replayed; after every few replays one copy reads all
    // the states, and when groups have finished the pool is rebuilt without them and the
    // stage captured again, so the tail of long runs launches only the groups still running.
    auto capture = [&]() -> smc_status {
        drop_graph();
        smc_status cs = SMC_OK;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return SMC_EDEVICE;
        if (view.launch_stage_all(s) != hipSuccess) cs = SMC_EDEVICE;
        if (hipStreamEndCapture(s, &graph) != hipSuccess && cs == SMC_OK) cs = SMC_EDEVICE;
        if (cs == SMC_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) cs = SMC_EDEVICE;
        return cs;
    };
    status = capture();
    if (status != SMC_OK) {
        cleanup();
        return status;
    }

    std::vector<GroupState> states(ngroups);
    std::vector<char> running(ngroups, 1);
    size_t n_running = ngroups;
    const int replays_between_checks = 4;
    bool all_done = false;
    for (int round = 0; !all_done && round <= opt->max_stages + 2; round += replays_between_checks) {
        for (int r = 0; r < replays_between_checks; ++r)
            if (hipGraphLaunch(exec, s) != hipSuccess) {
                cleanup();
                return SMC_EDEVICE;
            }
        if (hipMemcpyAsync(states.data(), d_states, sizeof(GroupState) * ngroups, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            cleanup();
            return SMC_EDEVICE;
        }
        all_done = true;
        size_t still = 0;
        for (size_t gi = 0; gi < ngroups; ++gi) {
            const GroupState& st = states[gi];
            if (st.status != SMC_OK) status = st.status;
            all_done = all_done && st.done;
            running[gi] = st.done ? 0 : 1;
            still += running[gi];
        }
        if (status != SMC_OK) break;
        if (!all_done && still < n_running) {
            n_running = still;
            status = view.rebuild(ptrs, s, &running);
            if (status == SMC_OK) status = capture();
            if (status != SMC_OK) break;
        }
    }
    if (status == SMC_OK && !all_done) status = SMC_ENUMERIC;
    size_t o = 0;
    for (const auto& e : entries)
        for (int k = 0; k < e->ng; ++k, ++o) logz_out[o] = states[o].logz - states[o].beta * e->econst;
    cleanup();
    return status;
}

// ============================================================================ served path

struct smc_server {
    smc_options opt{};
    uint64_t budget = 0;
    hipStream_t stream = nullptr;
    void* dmem = nullptr;
    BlockAllocator alloc;
    PoolView view;
    MoveWork* d_scratch = nullptr;
    size_t cap_scratch = 0;
    int device = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<Entry>> queue;   // submitted, not admitted
    std::vector<std::unique_ptr<Entry>> active;
    std::deque<smc_result> results;
    bool stop = false;
    smc_status fatal = SMC_OK;
    std::thread worker;

    void run();
    smc_status tick();
};

namespace {

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// Admit queued requests that fit (in arrival order), run one stage of every active group,
// retire finished requests.  Called by the worker thread only.
smc_status smc_server::tick() {
    std::vector<char> fresh;
    bool changed = false;
    {
        std::lock_guard<std::mutex> lk(mu);
        while (!queue.empty()) {
            Entry& e = *queue.front();
            size_t off = 0;
            if (!alloc.alloc(e.bytes, off)) break;
            e.off = off;
            if (!carve_entry(e, e.opt, static_cast<char*>(dmem) + off)) {
                alloc.release(off, e.bytes);
                smc_result r{};
                r.request_id = e.id;
                r.status = SMC_ENOMEM;
                results.push_back(r);
                queue.pop_front();
                continue;
            }
            active.push_back(std::move(queue.front()));
            queue.pop_front();
            changed = true;
        }
    }
    if (changed) {
        std::vector<std::vector<char>> keep;
        std::vector<Entry*> ptrs;
        fresh.assign(active.size(), 0);
        for (size_t i = 0; i < active.size(); ++i) {
            ptrs.push_back(active[i].get());
            if (!active[i]->started) {
                if (upload_entry(*active[i], stream, keep) != hipSuccess) return SMC_EDEVICE;
                fresh[i] = 1;
                active[i]->started = true;
            }
        }
        smc_status st = view.rebuild(ptrs, stream);
        if (st != SMC_OK) return st;
        std::vector<MoveWork> scratch;
        st = view.stage0(fresh, stream, scratch, d_scratch, cap_scratch);
        if (st != SMC_OK) return st;
    }
    if (active.empty()) return SMC_OK;
    if (view.launch_stage_all(stream) != hipSuccess) return SMC_EDEVICE;
    std::vector<GroupState> states(view.groups.size());
    std::vector<Entry*> cur;
    for (auto& ep : active) cur.push_back(ep.get());
    if (copy_states(view, cur, states, stream) != hipSuccess) return SMC_EDEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return SMC_EDEVICE;

    // retire requests whose every group is done
    std::vector<std::unique_ptr<Entry>> keep_active;
    bool retired = false;
    size_t gi = 0;
    for (auto& ep : active) {
        Entry& e = *ep;
        bool done = true;
        smc_status est = SMC_OK;
        for (int k = 0; k < e.ng; ++k) {
            const GroupState& st = states[gi + k];
            done = done && st.done;
            if (st.status != SMC_OK) est = st.status;
        }
        if (done || est != SMC_OK) {
            smc_result r{};
            r.request_id = e.id;
            r.status = est;
            r.k_min = e.spec.prob.k_min;
            r.k_max = e.spec.prob.k_max;
            double best = -__builtin_inf();
            int stages = 0;
            for (int k = 0; k < e.ng; ++k) {
                const GroupState& st = states[gi + k];
                r.logz[k] = st.logz - st.beta * e.econst;
                stages = std::max(stages, st.stage);
                if (r.logz[k] > best) {
                    best = r.logz[k];
                    r.best_k = e.spec.prob.k_min + k;
                }
            }
            r.n_stages = stages;
            r.latency_s = seconds_since(e.t_submit);
            {
                std::lock_guard<std::mutex> lk(mu);
                results.push_back(r);
                alloc.release(e.off, e.bytes);
            }
            retired = true;
        } else {
            keep_active.push_back(std::move(ep));
        }
        gi += e.ng;
    }
    active.swap(keep_active);  // every still-running entry was moved into keep_active
    if (retired) {
        cv_done.notify_all();
        std::vector<Entry*> ptrs;
        for (auto& ep : active) ptrs.push_back(ep.get());
        smc_status st = view.rebuild(ptrs, stream);
        if (st != SMC_OK) return st;
        // admission may have been blocked by memory: let the loop retry at once
    }
    return SMC_OK;
}

void smc_server::run() {
    if (hipSetDevice(device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = SMC_EDEVICE;
        cv_done.notify_all();
        return;
    }
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop) return;
        }
        const smc_status st = tick();
        if (st != SMC_OK) {
            std::lock_guard<std::mutex> lk(mu);
            fatal = st;
            cv_done.notify_all();
            return;
        }
    }
}

extern "C" uint64_t smc_server_request_bytes(const smc_problem* p, const smc_options* o) {
    if (!p || !o || validate(p, o) != SMC_OK) return 0;
    return align256(entry_bytes(*p, *o));
}

extern "C" smc_status smc_server_create(smc_server** out, uint64_t mem_budget_bytes, const smc_options* defaults) {
    if (!out || !defaults || mem_budget_bytes < 4096) return SMC_EINVAL;
    *out = nullptr;
    if (defaults->n_particles < 2 || defaults->n_moves < 1 ||
        (defaults->waste_free && defaults->n_particles % defaults->n_moves))
        return SMC_EINVAL;
    if (!device_ok()) return SMC_EDEVICE;
    smc_server* sv = new (std::nothrow) smc_server();
    if (!sv) return SMC_ENOMEM;
    sv->opt = *defaults;
    sv->budget = mem_budget_bytes;
    if (hipGetDevice(&sv->device) != hipSuccess || hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
        delete sv;
        return SMC_EDEVICE;
    }
    if (hipMalloc(&sv->dmem, mem_budget_bytes) != hipSuccess) {
        (void)hipStreamDestroy(sv->stream);
        delete sv;
        return SMC_ENOMEM;
    }
    sv->alloc.init(mem_budget_bytes);
    sv->worker = std::thread([sv] { sv->run(); });
    *out = sv;
    return SMC_OK;
}

extern "C" smc_status smc_server_submit(smc_server* sv, const smc_problem* prob, const smc_options* opt,
                                        uint64_t request_id) {
    if (!sv || !prob) return SMC_EINVAL;
    smc_options o = opt ? *opt : sv->opt;
    o.hip_stream = nullptr;
    o.plain = 0;
    o.profile = 0;
    smc_status st = validate(prob, &o);
    if (st != SMC_OK) return st;
    if (prob->k_max - prob->k_min + 1 > 32) return SMC_EINVAL;
    if (!tile_has_kernels(*prob, entry_tile(*prob, o))) return SMC_EINVAL;
    auto e = std::make_unique<Entry>();
    e->id = request_id;
    e->opt = o;
    e->spec.assign(*prob);
    e->ng = prob->k_max - prob->k_min + 1;
    e->tile = entry_tile(*prob, o);
    e->econst = energy_constant(e->spec.prob);
    e->bytes = align256(entry_bytes(*prob, o));
    e->t_submit = std::chrono::steady_clock::now();
    if (e->bytes > sv->budget) return SMC_EBUDGET;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->fatal != SMC_OK) return sv->fatal;
        sv->queue.push_back(std::move(e));
    }
    sv->cv_work.notify_one();
    return SMC_OK;
}

extern "C" smc_status smc_server_poll(smc_server* sv, smc_result* out, int32_t cap, int32_t* n_out, int32_t wait_ms) {
    if (!sv || !n_out || (cap > 0 && !out)) return SMC_EINVAL;
    *n_out = 0;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->results.empty() && wait_ms > 0)
        sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms),
                             [&] { return !sv->results.empty() || sv->fatal != SMC_OK; });
    int n = 0;
    while (n < cap && !sv->results.empty()) {
        out[n++] = sv->results.front();
        sv->results.pop_front();
    }
    *n_out = n;
    if (sv->fatal != SMC_OK) return sv->fatal;
    return n > 0 ? SMC_OK : SMC_EAGAIN;
}

extern "C" void smc_server_destroy(smc_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    (void)hipStreamSynchronize(sv->stream);
    sv->view.release();
    if (sv->d_scratch) (void)hipFree(sv->d_scratch);
    if (sv->dmem) (void)hipFree(sv->dmem);
    (void)hipStreamDestroy(sv->stream);
    delete sv;
}
