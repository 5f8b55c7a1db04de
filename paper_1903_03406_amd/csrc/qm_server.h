// qm_server.h -- served form of the refinement: a job queue admitted against
// a device-memory budget, run by worker threads that each own a HIP stream.
//
// Host code only (no kernels).  A job is one qm_refine call (the round loop
// of paper, Section 2) on the server's device; the server copies the job's
// host arrays at submission, so the caller's buffers are free again when
// qm_server_submit returns.  Admission: a job is taken when its byte
// estimate fits in the budget minus the estimates of the jobs already
// admitted and not finished; otherwise submission returns QM_EAGAIN and the
// caller retries later.  Workers take admitted jobs first come, first served;
// a finished job's estimate is released before its result is handed out.
//
// Stepped form (created with no workers): continuous batching.  The jobs
// form SRV_GROUPS lockstep batches, each on a stream and a persistent host
// thread of its own (a new job joins the batch with the fewest resident
// input tets): each qm_server_step sets up the jobs admitted since the last
// step, then every batch runs one round of each of its resident jobs, each
// phase of the round one launch over all of them, the batches at the same
// time; jobs join and leave at round boundaries and their meshes stay on
// the device in between.
//
// Eviction (both forms): qm_server_evict takes a job off the device at a
// round boundary.  Its output mesh and refinement state (qm_result_state)
// become a host checkpoint, and its estimate leaves the budget.
// qm_server_readmit admits it again, and it resumes from the checkpoint
// (qm_refine_resume).  The result it finally returns holds the round records
// and statistics of every segment, and equals the uninterrupted refinement.
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <unordered_map>

namespace {

using srv_clock = std::chrono::steady_clock;

struct SrvJob {
    uint64_t ticket = 0;
    size_t est = 0;
    std::vector<double> xyz;
    std::vector<int32_t> tet, sf, sff, ss, ssg, seg, ftri, ftrif;
    qm_plc plc{};
    qm_mesh mesh{};
    qm_options opt{};
    srv_clock::time_point t_sub;
    // eviction: the checkpoint (the mesh above is then the output it
    // resumes from), and what the job's earlier segments recorded
    std::vector<uint8_t> tfl, sfl, ssl;
    qm_state state{};
    bool has_state = false;
    std::vector<int32_t> hist_rounds;
    qm_stats hist{};
    int segments = 0;
    std::atomic<bool> stop{false};     // worker form: end at the next round boundary
    double wait_s = -1.0;              // queued time before the first segment started
};

// the job's options for its next segment: the round limit less the rounds
// its earlier segments ran
qm_options srv_seg_opt(const SrvJob& J) {
    qm_options o = J.opt;
    if (J.has_state) o.max_rounds = std::max(0, J.opt.max_rounds - J.state.rounds);
    return o;
}

void srv_add_stats(qm_stats& a, const qm_stats& b) {
    a.rounds += b.rounds;
    for (int c = 0; c < 3; ++c) a.inserted[c] += b.inserted[c];
    a.candidates += b.candidates;
    a.mis_passes += b.mis_passes;
    a.deferred += b.deferred;
    a.device_bytes_peak = std::max(a.device_bytes_peak, b.device_bytes_peak);
    a.seconds_setup += b.seconds_setup;
    a.seconds_refine += b.seconds_refine;
    a.seconds_total += b.seconds_total;
}

// an evicted segment's host result becomes the job's checkpoint
void srv_checkpoint(SrvJob& J, qm_result* r) {
    J.xyz = std::move(r->xyz); J.tet = std::move(r->tets);
    J.sf = std::move(r->sf); J.sff = std::move(r->sff);
    J.ss = std::move(r->ss); J.ssg = std::move(r->ssg);
    J.tfl = std::move(r->st_tfl); J.sfl = std::move(r->st_sfl); J.ssl = std::move(r->st_ssl);
    J.mesh = qm_mesh{(int32_t)(J.xyz.size() / 3), J.xyz.data(), (int32_t)(J.tet.size() / 4), J.tet.data(),
                     (int32_t)J.sff.size(), J.sf.data(), J.sff.data(), (int32_t)J.ssg.size(), J.ss.data(),
                     J.ssg.data()};
    J.state = qm_state{r->st_hmin2, r->st_rounds, r->st_next, (int32_t)J.tfl.size(), (int32_t)J.sfl.size(),
                       (int32_t)J.ssl.size(), J.tfl.data(), J.sfl.data(), J.ssl.data()};
    J.has_state = true;
    J.hist_rounds.insert(J.hist_rounds.end(), r->rounds.begin(), r->rounds.end());
    srv_add_stats(J.hist, r->stats);
    ++J.segments;
    qm_result_free(r);
}

// the last segment's result completed with the earlier segments' records
void srv_merge(const SrvJob& J, qm_result* r) {
    if (!r || !J.segments) return;
    r->rounds.insert(r->rounds.begin(), J.hist_rounds.begin(), J.hist_rounds.end());
    // counters summed over the segments; the output's own figures are the
    // last segment's
    qm_stats s = J.hist;
    srv_add_stats(s, r->stats);
    r->stats.rounds = s.rounds;
    for (int c = 0; c < 3; ++c) r->stats.inserted[c] = s.inserted[c];
    r->stats.candidates = s.candidates;
    r->stats.mis_passes = s.mis_passes;
    r->stats.deferred = s.deferred;
    r->stats.device_bytes_peak = s.device_bytes_peak;
    r->stats.seconds_setup = s.seconds_setup;
    r->stats.seconds_refine = s.seconds_refine;
    r->stats.seconds_total = s.seconds_total;
}

struct SrvDone {
    qm_result* res = nullptr;
    int code = QM_EINTERNAL;
    std::string msg;
    double wait_s = 0, total_s = 0;
};

// copy n*cols elements of a borrowed host array; false when a non-empty
// array has no pointer
template <class T>
bool srv_copy(std::vector<T>& dst, const T* src, long n, int cols) {
    if (n < 0) return false;
    if (n == 0) return true;
    if (!src) return false;
    dst.assign(src, src + n * (long)cols);
    return true;
}

}  // namespace

struct qm_server {
    int dev = 0;
    size_t budget = 0, resident = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<SrvJob>> queue;
    std::unordered_map<uint64_t, SrvDone> done;
    std::unordered_map<uint64_t, int> live;   // admitted and not yet collected
    uint64_t next_ticket = 1;
    bool stop = false;
    int running = 0;
    int64_t admitted = 0, refused = 0, completed = 0, evictions = 0;
    std::unordered_map<uint64_t, SrvJob*> running_jobs;             // worker form: jobs being refined
    std::unordered_map<uint64_t, std::unique_ptr<SrvJob>> parked;   // evicted jobs (host checkpoints)
    std::vector<std::thread> workers;
    bool stepped = false;                                  // no workers: qm_server_step drives the jobs
    // stepped form: lockstep batches of resident jobs, each with its stream,
    // resident input tets and step thread, and what the server keeps of each
    // resident job (its estimate, batch and times)
    struct Group {
        hipStream_t st = nullptr;
        std::unique_ptr<Lockstep> batch;
        int64_t load = 0;
        int code = 0;
        std::string msg;
    };
    std::vector<Group> groups;
    std::vector<std::thread> group_threads;
    std::mutex gmu;
    std::condition_variable gcv, gdone;
    uint64_t gen = 0;
    int gpending = 0;
    bool gstop = false;
    std::unordered_map<uint64_t, std::unique_ptr<SrvJob>> in_batch;
    std::unordered_map<uint64_t, srv_clock::time_point> t_added;
    std::unordered_map<uint64_t, int> group_of;
    std::mutex step_mu;                                    // steps take turns
    int live_jobs() const {
        int n = 0;
        for (auto& g : groups) n += g.batch ? g.batch->live() : 0;
        return n;
    }
};

namespace {
constexpr int SRV_GROUPS = 4;      // lockstep batches of the stepped form

// a step thread: runs its batch's round whenever the step counter moves on
void srv_group_run(qm_server* S, int g) {
    (void)hipSetDevice(S->dev);
    uint64_t seen = 0;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->gmu);
            S->gcv.wait(lk, [&] { return S->gstop || S->gen != seen; });
            if (S->gstop) return;
            seen = S->gen;
        }
        auto& G = S->groups[g];
        try {
            if (G.batch->live() > 0) G.batch->step();
        } catch (const QmError& e) {
            G.code = e.code;
            G.msg = e.what();
        } catch (const std::exception& e) {
            G.code = QM_EINTERNAL;
            G.msg = e.what();
        }
        std::lock_guard<std::mutex> lk(S->gmu);
        if (--S->gpending == 0) S->gdone.notify_all();
    }
}
}  // namespace

namespace {

void srv_worker(qm_server* S) {
    hipStream_t st = nullptr;
    bool ok = hipSetDevice(S->dev) == hipSuccess &&
              hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
        std::unique_ptr<SrvJob> J;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->stop) break;
            J = std::move(S->queue.front());
            S->queue.pop_front();
            ++S->running;
            S->running_jobs[J->ticket] = J.get();
        }
        const auto t_start = srv_clock::now();
        if (J->wait_s < 0) J->wait_s = std::chrono::duration<double>(t_start - J->t_sub).count();
        SrvDone d;
        if (ok) {
            const qm_options o = srv_seg_opt(*J);
            d.code = refine_within(&J->plc, &J->mesh, &o, st, &d.res, J->est, J->has_state ? &J->state : nullptr,
                                   &J->stop);
            if (d.code != QM_OK && d.code != QM_EROUNDS) d.msg = qm_last_error();
        } else {
            d.code = QM_EDEVICE;
            d.msg = "server worker has no HIP stream";
        }
        const bool evicted = d.code == QM_OK && d.res && d.res->stats.status == 2;
        if (evicted) srv_checkpoint(*J, d.res);
        else srv_merge(*J, d.res);
        const auto t_end = srv_clock::now();
        d.wait_s = J->wait_s;
        d.total_s = std::chrono::duration<double>(t_end - J->t_sub).count();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->resident -= J->est;
            --S->running;
            S->running_jobs.erase(J->ticket);
            if (evicted) {
                J->stop = false;
                ++S->evictions;
                const uint64_t t = J->ticket;
                S->parked[t] = std::move(J);
            } else {
                ++S->completed;
                S->done[J->ticket] = std::move(d);
            }
        }
        S->cv_done.notify_all();
    }
    if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
}

}  // namespace

extern "C" {

size_t qm_estimate_bytes(const qm_plc* plc, const qm_mesh* in, const qm_options* opt) {
    if (!plc || !in || !opt || in->nt < 0 || in->nv < 0) return 0;
    // Measured peaks of single refinements (qm_stats.device_bytes_peak) stay
    // below 8 KB per input tet at B >= 1.6 and 16 KB at tighter bounds once
    // the slab tiles are held to a quarter of the budget: the mesh grows 2-4x (7x at
    // B = 1.4), and a bad-tet round's candidate arrays, result pools and
    // selection words dominate.  320 MiB covers the fixed buffers; a served
    // job runs with its estimate as its budget.
    const double per_tet = opt->B < 1.6 ? 16384.0 : 8192.0;
    return (size_t)((double)in->nt * per_tet) + ((size_t)320 << 20);
}

int qm_server_create(size_t hbm_budget_bytes, int32_t nworkers, qm_server** out) {
    g_err.clear();
    if (!out || nworkers < 0 || nworkers > 64 || hbm_budget_bytes == 0) {
        g_err = "bad server arguments";
        return QM_EINVAL;
    }
    *out = nullptr;
    auto S = std::make_unique<qm_server>();
    if (hipGetDevice(&S->dev) != hipSuccess) { g_err = "no HIP device"; return QM_EDEVICE; }
    S->budget = hbm_budget_bytes;
    S->stepped = nworkers == 0;
    try {
        if (S->stepped) {
            S->groups.resize(SRV_GROUPS);
            for (auto& G : S->groups) {
                if (hipStreamCreateWithFlags(&G.st, hipStreamNonBlocking) != hipSuccess) {
                    for (auto& H : S->groups)
                        if (H.st) (void)hipStreamDestroy(H.st);
                    g_err = "no HIP stream for the stepped server";
                    return QM_EDEVICE;
                }
                G.batch = std::make_unique<Lockstep>(G.st);
            }
            for (int g = 0; g < SRV_GROUPS; ++g) S->group_threads.emplace_back(srv_group_run, S.get(), g);
        }
        for (int i = 0; i < nworkers; ++i) S->workers.emplace_back(srv_worker, S.get());
    } catch (const std::exception& e) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        for (auto& t : S->workers) t.join();
        {
            std::lock_guard<std::mutex> lk(S->gmu);
            S->gstop = true;
        }
        S->gcv.notify_all();
        for (auto& t : S->group_threads) t.join();
        for (auto& G : S->groups) {
            G.batch.reset();
            if (G.st) (void)hipStreamDestroy(G.st);
        }
        g_err = e.what();
        return QM_ENOMEM;
    }
    *out = S.release();
    return QM_OK;
}

int qm_server_submit(qm_server* S, const qm_plc* plc, const qm_mesh* in, const qm_options* opt,
                     size_t est_bytes, uint64_t* ticket) {
    g_err.clear();
    if (!S || !plc || !in || !opt || !ticket) { g_err = "null argument"; return QM_EINVAL; }
    if (opt->flags & QM_INPUT_DEVICE) { g_err = "server jobs take host arrays"; return QM_EINVAL; }
    const size_t est = est_bytes ? est_bytes : qm_estimate_bytes(plc, in, opt);
    if (est > S->budget) {
        g_err = "job estimate " + std::to_string(est) + " B exceeds the server budget";
        return QM_ENOMEM;
    }
    auto J = std::make_unique<SrvJob>();
    try {
        if (!srv_copy(J->xyz, in->xyz, in->nv, 3) || !srv_copy(J->tet, in->tet, in->nt, 4) ||
            !srv_copy(J->sf, in->sf, in->nsf, 3) || !srv_copy(J->sff, in->sf_facet, in->nsf, 1) ||
            !srv_copy(J->ss, in->ss, in->nss, 2) || !srv_copy(J->ssg, in->ss_seg, in->nss, 1) ||
            !srv_copy(J->seg, plc->seg, plc->nseg, 2) || !srv_copy(J->ftri, plc->ftri, plc->nftri, 3) ||
            !srv_copy(J->ftrif, plc->ftri_facet, plc->nftri, 1)) {
            g_err = "negative count or missing array";
            return QM_EINVAL;
        }
    } catch (const std::bad_alloc&) {
        g_err = "host copy of the job failed";
        return QM_ENOMEM;
    }
    J->plc = qm_plc{plc->nv, plc->nseg, J->seg.data(), plc->nftri, J->ftri.data(), J->ftrif.data()};
    J->mesh = qm_mesh{in->nv, J->xyz.data(), in->nt, J->tet.data(), in->nsf, J->sf.data(), J->sff.data(),
                      in->nss, J->ss.data(), J->ssg.data()};
    J->opt = *opt;
    J->est = est;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->resident + est > S->budget) {
            ++S->refused;
            g_err = "over the server budget (resident " + std::to_string(S->resident) + " B)";
            return QM_EAGAIN;
        }
        S->resident += est;
        J->ticket = S->next_ticket++;
        J->t_sub = srv_clock::now();
        *ticket = J->ticket;
        S->live[J->ticket] = 1;
        ++S->admitted;
        S->queue.push_back(std::move(J));
    }
    S->cv_work.notify_one();
    return QM_OK;
}

int qm_server_poll(qm_server* S, uint64_t ticket, int32_t wait_ms, qm_result** out, int32_t* code,
                   double* seconds) {
    g_err.clear();
    if (!S || !out || !code) { g_err = "null argument"; return QM_EINVAL; }
    std::unique_lock<std::mutex> lk(S->mu);
    if (!S->live.count(ticket)) { g_err = "unknown ticket"; return QM_EINVAL; }
    auto ready = [&] { return S->done.count(ticket) > 0 || S->parked.count(ticket) > 0; };
    if (!ready()) {
        if (wait_ms < 0) S->cv_done.wait(lk, ready);
        else if (wait_ms > 0) S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    }
    if (!S->done.count(ticket)) {
        if (S->parked.count(ticket)) g_err = "the job is evicted (qm_server_readmit brings it back)";
        return QM_EAGAIN;
    }
    auto it = S->done.find(ticket);
    SrvDone d = std::move(it->second);
    S->done.erase(it);
    S->live.erase(ticket);
    *out = d.res;
    *code = d.code;
    if (seconds) { seconds[0] = d.wait_s; seconds[1] = d.total_s; }
    g_err = d.msg;
    return QM_OK;
}

}  // extern "C"

namespace {
// stepped form: jobs that left their batches (finished, failed, or evicted
// with a checkpoint) leave the budget; called with step_mu held
void srv_collect(qm_server* S, std::vector<LsDone>& finished) {
    const auto now = srv_clock::now();
    for (auto& d : finished) {
        auto it = S->in_batch.find(d.tag);
        auto go = S->group_of.find(d.tag);
        if (go != S->group_of.end()) {
            if (it != S->in_batch.end()) S->groups[go->second].load -= it->second->mesh.nt;
            S->group_of.erase(go);
        }
        std::unique_ptr<SrvJob> J;
        if (it != S->in_batch.end()) {
            J = std::move(it->second);
            S->in_batch.erase(it);
        }
        const bool evicted = J && d.code == QM_OK && d.res && d.res->stats.status == 2;
        SrvDone out;
        if (J && !evicted) {
            srv_merge(*J, d.res);
            out.wait_s = J->wait_s;
            out.total_s = std::chrono::duration<double>(now - J->t_sub).count();
        }
        if (evicted) srv_checkpoint(*J, d.res);
        out.res = evicted ? nullptr : d.res;
        out.code = d.code;
        out.msg = d.msg;
        const size_t est = J ? J->est : 0;
        S->t_added.erase(d.tag);
        std::lock_guard<std::mutex> lk(S->mu);
        S->resident -= est;
        if (evicted) {
            ++S->evictions;
            S->parked[d.tag] = std::move(J);
        } else {
            ++S->completed;
            S->done[d.tag] = std::move(out);
        }
    }
}

// a job waiting in the queue leaves it for the parked set (called with mu
// held); false when it is not queued
bool srv_park_queued(qm_server* S, uint64_t t) {
    for (auto q = S->queue.begin(); q != S->queue.end(); ++q) {
        if ((*q)->ticket != t) continue;
        S->resident -= (*q)->est;
        ++S->evictions;
        S->parked[t] = std::move(*q);
        S->queue.erase(q);
        return true;
    }
    return false;
}
}  // namespace

extern "C" {

int qm_server_evict(qm_server* S, uint64_t t) {
    g_err.clear();
    if (!S) { g_err = "null argument"; return QM_EINVAL; }
    auto known = [&]() {
        if (!S->live.count(t) || S->done.count(t) || S->parked.count(t)) {
            g_err = "unknown, finished or already evicted ticket";
            return false;
        }
        return true;
    };
    try {
        if (S->stepped) {
            std::lock_guard<std::mutex> step_lock(S->step_mu);   // the batches are idle between steps
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (!known()) return QM_EINVAL;
                if (srv_park_queued(S, t)) { S->cv_done.notify_all(); return QM_OK; }
            }
            auto go = S->group_of.find(t);
            if (go == S->group_of.end()) { g_err = "the job is not resident"; return QM_EINVAL; }
            if (hipSetDevice(S->dev) != hipSuccess) throw QmError(QM_EDEVICE, "cannot select the server's device");
            auto& G = S->groups[go->second];
            G.batch->evict_now(t);
            std::vector<LsDone> finished = G.batch->take_done();
            srv_collect(S, finished);
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->running = S->live_jobs();
            }
            S->cv_done.notify_all();
            std::lock_guard<std::mutex> lk(S->mu);
            return S->parked.count(t) ? QM_OK : QM_EAGAIN;
        }
        std::unique_lock<std::mutex> lk(S->mu);
        if (!known()) return QM_EINVAL;
        if (srv_park_queued(S, t)) { S->cv_done.notify_all(); return QM_OK; }
        auto r = S->running_jobs.find(t);
        if (r == S->running_jobs.end()) { g_err = "the job is not resident"; return QM_EINVAL; }
        r->second->stop = true;                   // the worker ends the job at its next round boundary
        S->cv_done.wait(lk, [&] { return S->parked.count(t) > 0 || S->done.count(t) > 0; });
        if (S->parked.count(t)) return QM_OK;
        g_err = "the job finished before it could be evicted";
        return QM_EAGAIN;
    } catch (const QmError& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return QM_EINTERNAL;
    }
}

int qm_server_readmit(qm_server* S, uint64_t t) {
    g_err.clear();
    if (!S) { g_err = "null argument"; return QM_EINVAL; }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->parked.find(t);
        if (it == S->parked.end()) { g_err = "the ticket is not an evicted job"; return QM_EINVAL; }
        if (S->resident + it->second->est > S->budget) {
            ++S->refused;
            g_err = "over the server budget (resident " + std::to_string(S->resident) + " B)";
            return QM_EAGAIN;
        }
        S->resident += it->second->est;
        S->queue.push_back(std::move(it->second));
        S->parked.erase(it);
    }
    S->cv_work.notify_one();
    return QM_OK;
}

int qm_server_step(qm_server* S, int32_t* nresident) {
    g_err.clear();
    if (!S) { g_err = "null argument"; return QM_EINVAL; }
    if (!S->stepped) { g_err = "this server runs its jobs with its own workers"; return QM_EINVAL; }
    std::lock_guard<std::mutex> step_lock(S->step_mu);
    try {
        if (hipSetDevice(S->dev) != hipSuccess) throw QmError(QM_EDEVICE, "cannot select the server's device");
        // jobs admitted since the last step join the batch (set-up on the device)
        std::vector<std::unique_ptr<SrvJob>> fresh;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            while (!S->queue.empty()) {
                fresh.push_back(std::move(S->queue.front()));
                S->queue.pop_front();
            }
        }
        for (auto& J : fresh) {
            const uint64_t t = J->ticket;
            int g = 0;
            for (int k = 1; k < (int)S->groups.size(); ++k)
                if (S->groups[k].load < S->groups[g].load) g = k;
            S->t_added[t] = srv_clock::now();
            if (J->wait_s < 0) J->wait_s = std::chrono::duration<double>(S->t_added[t] - J->t_sub).count();
            S->groups[g].load += J->mesh.nt;
            S->group_of[t] = g;
            const qm_options o = srv_seg_opt(*J);
            S->groups[g].batch->add(&J->plc, &J->mesh, &o, t, J->has_state ? &J->state : nullptr);
            S->in_batch[t] = std::move(J);
        }
        // one round of every resident job: the batches at the same time, each
        // phase one launch over a batch's jobs
        {
            std::unique_lock<std::mutex> lk(S->gmu);
            S->gpending = (int)S->groups.size();
            ++S->gen;
            S->gcv.notify_all();
            S->gdone.wait(lk, [&] { return S->gpending == 0; });
        }
        for (auto& G : S->groups)
            if (G.code) {
                const int c = G.code;
                G.code = 0;
                throw QmError(c, G.msg);
            }
        std::vector<LsDone> finished;
        for (auto& G : S->groups)
            for (auto& d : G.batch->take_done()) finished.push_back(std::move(d));
        srv_collect(S, finished);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->running = S->live_jobs();
        }
        S->cv_done.notify_all();
        if (nresident) *nresident = (int32_t)S->live_jobs();
        return QM_OK;
    } catch (const QmError& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return QM_EINTERNAL;
    }
}

int qm_server_info(qm_server* S, qm_server_stats* info) {
    g_err.clear();
    if (!S || !info) { g_err = "null argument"; return QM_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    info->budget = S->budget;
    info->resident = S->resident;
    info->queued = (int32_t)S->queue.size();
    info->running = S->running;
    info->admitted = S->admitted;
    info->refused = S->refused;
    info->completed = S->completed;
    info->evictions = S->evictions;
    info->parked = (int32_t)S->parked.size();
    return QM_OK;
}

void qm_server_destroy(qm_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (auto& J : S->queue) S->resident -= J->est;
        S->queue.clear();
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    if (S->stepped) {                        // stepped form: resident jobs end with their batches
        {
            std::lock_guard<std::mutex> lk(S->gmu);
            S->gstop = true;
        }
        S->gcv.notify_all();
        for (auto& t : S->group_threads) t.join();
        (void)hipSetDevice(S->dev);
        for (auto& G : S->groups) {
            G.batch.reset();
            if (G.st) (void)hipStreamDestroy(G.st);
        }
    }
    for (auto& kv : S->done) qm_result_free(kv.second.res);
    delete S;
}

}  // extern "C"
