// qm_lockstep.h -- lockstep batched form: independent refinements advance
// round by round together, and each phase of a round is one launch over the
// work of every instance that takes part in it.
//
// The round is the paper's (Section 2: classify, split, locate, grow and
// validate, select, insert); each instance runs exactly the rounds it runs
// alone and ends with the same output bits.  What changes is the launch
// shape: a batched launch carries a part table (the instances it covers and
// each one's first workgroup), every workgroup finds its part with two wave
// ballots and runs the single-instance kernel body on that instance's arrays
// with its workgroup index inside the part.  Per-instance pointers and
// counts sit in a device table of `LsInst` records that the host refreshes
// (one copy) whenever one of them changes.  Each instance still picks its
// own class, so a round mixes subsegment, subface and tet work of different
// instances in one launch.  Work whose size makes launch cost irrelevant
// (radix sorts of more than 4096 candidates, device-wide scans of more than
// 32768, renumbering tet slots) runs per instance.
#pragma once

namespace qm {

// device view of one instance in a batched launch
struct LsInst {
    Mesh M;
    Cands C;
    Pools PL;
    BfPool BP;
    int* ctr;
    int* c_elem0;
    unsigned long long* c_key0;
    int4* c_tup0;
    double4* c_p0;
    int *c_st0, *c_reason0;
    int *olist, *glist, *sk, *st_, *ss_, *kept, *ulist0, *ulist1;
    unsigned long long* mark;
    int* owner;
    unsigned char *mis_drop, *mis_lose;
    unsigned long long key_mask;
    unsigned pass;
    int cls, ncand, ncl, nkept, min_tier, nover, nbig, nv0, nt0, nss0;
};

// Parts of one batched launch, passed by value: part k covers workgroups
// [pre[k], pre[k+1]) and instance table entry map[k].
constexpr int LS_PARTS = 256;
struct LsParts {
    int np;
    int pre[LS_PARTS + 1];
    int map[LS_PARTS];
};

// the part of workgroup b: the last k with pre[k] <= b (parts are never
// empty), searched 64 parts at a time by wave ballots (np <= 4096)
QMD int ls_find_part(const LsParts& P, int b) {
    const int lane = threadIdx.x & 63;
    const int step = (P.np + 63) >> 6;
    int j = lane * step;
    unsigned long long m = __ballot(j < P.np && P.pre[j] <= b);
    const int base = (63 - __clzll((long long)m)) * step;
    j = base + lane;
    m = __ballot(lane < step && j < P.np && P.pre[j] <= b);
    return base + (63 - __clzll((long long)m));
}

template <int NT, class F>
__global__ __launch_bounds__(NT) void k_each(const LsInst* __restrict__ D, const LsParts P, const F f) {
    const int k = ls_find_part(P, (int)blockIdx.x);
    f(D[P.map[k]], k, (int)blockIdx.x - P.pre[k], P.pre[k + 1] - P.pre[k]);
}

// ---- per-phase bodies (instance record, part index, workgroup, workgroups)
struct FReset {                 // k_round_reset
    QMD void operator()(const LsInst& d, int, int, int) const {
        const int i = threadIdx.x;
        if (i < 48 && (i < 11 || i >= 15)) d.ctr[i] = 0;
    }
};
// classification: each workgroup takes `tiles` consecutive 256-element
// tiles of its instance (one part lookup for all of them)
// (each body starts from local copies of the record's fields: stores of the
// body cannot then force the record to be read again)
struct FClassifySS {
    int tiles;
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        const Mesh M = d.M;
        int* const cand = d.c_elem0;
        int* const cnt = d.ctr + 8;
        for (int v = 0; v < tiles; ++v) d_classify_ss(M, cand, cnt, b * tiles + v, g * tiles);
    }
};
struct FClassifySF {
    int tiles;
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        int* const cnt = d.ctr + 8;
        if (cnt[CLS_SS] > 0) return;                 // an earlier class has candidates
        const Mesh M = d.M;
        int* const cand = d.c_elem0;
        for (int v = 0; v < tiles; ++v) d_classify_sf(M, cand, cnt, b * tiles + v, g * tiles);
    }
};
struct FClassifyTet {
    int tiles;
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        int* const cnt = d.ctr + 8;
        if (cnt[CLS_SS] > 0 || cnt[CLS_SF] > 0) return;
        const Mesh M = d.M;
        int* const cand = d.c_elem0;
        for (int v = 0; v < tiles; ++v) d_classify_tet(M, cand, cnt, b * tiles + v, g * tiles);
    }
};
struct FGather {                // counters of each part, side by side
    int* out;
    QMD void operator()(const LsInst& d, int k, int, int) const {
        for (int i = threadIdx.x; i < 48; i += blockDim.x) out[48 * k + i] = d.ctr[i];
    }
};
struct FSplit {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        d_split(d.M, d.cls, d.ncand, d.c_elem0, d.c_key0, d.c_tup0, d.c_p0, d.c_st0, d.c_reason0, d.key_mask, b, g);
    }
};
struct FOrderSmall {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        d_order_small(d.ncand, d.c_elem0, d.c_key0, d.c_tup0, d.c_p0, d.c_st0, d.c_reason0, d.C, b, g);
    }
};
constexpr int LS_ORDER_CAP = 4096;    // one 1024-lane workgroup ranks at most this many candidates
struct FOrderMid {
    QMD void operator()(const LsInst& d, int, int, int) const {
        d_order_rank<1024, LS_ORDER_CAP>(d.ncand, d.c_elem0, d.c_key0, d.c_tup0, d.c_p0, d.c_st0, d.c_reason0, d.C);
    }
};
struct FLocate {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        const Mesh M = d.M;
        const Cands C = d.C;
        d_locate(M, d.cls, C, b, g);
    }
};
struct FResetPools {            // k_round_reset_pools
    QMD void operator()(const LsInst& d, int, int, int) const {
        if (threadIdx.x < 8) d.ctr[threadIdx.x] = 0;
    }
};
struct FGrowSmall {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        const Mesh M = d.M;
        const Cands C = d.C;
        const Pools PL = d.PL;
        const BfPool BP = d.BP;
        d_grow_lds<QM_TILES_SMALL>(M, d.cls, C, PL, BP, nullptr, 0, nullptr, d.min_tier, b, g);
    }
};
struct FListReset {             // re-run list counts [32..35) and [36]
    QMD void operator()(const LsInst& d, int, int, int) const {
        const int i = threadIdx.x;
        if (i < 5 && i != 3) d.ctr[32 + i] = 0;
    }
};
struct FOverflowList {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        d_overflow_list(d.C, d.olist, d.glist, d.ctr + 32, b, g);
    }
};
struct FGrowHybrid {            // workgroup w of the launch uses block w of the shared slab
    GrowTiles T;
    char* slab;
    size_t block;
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        const Mesh M = d.M;
        const Cands C = d.C;
        const Pools PL = d.PL;
        const BfPool BP = d.BP;
        d_grow_hybrid<H_LANES, H_HCAP, H_RFHCAP, H_QHCAP>(M, d.cls, C, PL, BP, d.olist, d.nover, T,
                                                          slab + block * blockIdx.x, b, g);
    }
};
struct FGrowGlobal {
    GrowTiles T;
    char* slab;
    size_t block;
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        const Mesh M = d.M;
        const Cands C = d.C;
        const Pools PL = d.PL;
        const BfPool BP = d.BP;
        d_grow_global<B_LANES>(M, d.cls, C, PL, BP, d.glist, d.nbig, T, slab + block * blockIdx.x, b, g);
    }
};
struct FVerdicts {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        const Mesh M = d.M;
        const Cands C = d.C;
        const Pools PL = d.PL;
        d_verdicts(M, d.cls, C, PL, d.ctr + 16, b, g);
    }
};
struct FMisSmall {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        d_mis_small(d.ncl, d.PL.cl, d.PL.clc, d.ncand, d.C.state, d.mark, d.owner, d.mis_drop, d.mis_lose, d.pass,
                    MIS_SMALL_PASSES, d.ctr + 38, b, g);
    }
};
// selection passes over several workgroups per instance (claims or
// candidates beyond one workgroup): pass b of a batch of MIS_BATCH, pass p
// of the round (its parity picks the undecided lists)
struct FUndecReset {
    QMD void operator()(const LsInst& d, int, int, int) const {
        if (threadIdx.x < MIS_BATCH) d.ctr[40 + threadIdx.x] = 0;
    }
};
struct FMisMark {
    int b;
    QMD void operator()(const LsInst& d, int, int x, int g) const {
        d_mis_mark(d.ncl, d.PL.cl, d.PL.clc, d.C.state, d.mark, d.pass + (unsigned)b, nullptr, x, g);
    }
};
struct FMisCheck {
    int b;
    QMD void operator()(const LsInst& d, int, int x, int g) const {
        d_mis_check(d.ncl, d.PL.cl, d.PL.clc, d.C.state, d.mark, d.owner, d.pass + (unsigned)b, d.mis_drop,
                    d.mis_lose, nullptr, x, g);
    }
};
struct FMisDecide {
    int b;
    QMD void operator()(const LsInst& d, int, int x, int g) const {
        d_mis_decide(d.ncand, d.C.state, d.mis_drop, d.mis_lose, d.ctr + 40 + b, nullptr, d.ulist0, d.ctr + 46, x, g);
    }
};
struct FMisCommit {
    QMD void operator()(const LsInst& d, int, int x, int g) const {
        d_mis_commit(d.ncl, d.PL.cl, d.PL.clc, d.C.state, d.owner, nullptr, x, g);
    }
};
struct FMisMarkList {
    int b, p;
    QMD void operator()(const LsInst& d, int, int x, int g) const {
        const int* u_in = (p & 1) ? d.ulist0 : d.ulist1;
        d_mis_mark_list(u_in, d.ctr + 46 + ((p - 1) & 1), d.C, d.PL.cl, d.mark, d.pass + (unsigned)b,
                        d.ctr + 46 + (p & 1), x, g);
    }
};
struct FMisCheckList {
    int b, p;
    QMD void operator()(const LsInst& d, int, int x, int g) const {
        const int* u_in = (p & 1) ? d.ulist0 : d.ulist1;
        d_mis_check_list(u_in, d.ctr + 46 + ((p - 1) & 1), d.C, d.PL.cl, d.mark, d.owner, d.pass + (unsigned)b,
                         d.mis_drop, d.mis_lose, x, g);
    }
};
struct FMisDecideList {
    int b, p;
    QMD void operator()(const LsInst& d, int, int x, int g) const {
        const int* u_in = (p & 1) ? d.ulist0 : d.ulist1;
        int* u_out = (p & 1) ? d.ulist1 : d.ulist0;
        d_mis_decide_list(u_in, d.ctr + 46 + ((p - 1) & 1), d.C.state, d.mis_drop, d.mis_lose, d.ctr + 40 + b, u_out,
                          d.ctr + 46 + (p & 1), x, g);
    }
};
struct FMisCommitList {
    int p;
    QMD void operator()(const LsInst& d, int, int x, int g) const {
        const int* u_in = (p & 1) ? d.ulist0 : d.ulist1;
        d_mis_commit_list(u_in, d.ctr + 46 + ((p - 1) & 1), d.C, d.PL.cl, d.C.state, d.owner, x, g);
    }
};
struct FScanSmall {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        d_scan_small(d.C, d.cls, d.ncand, d.sk, d.st_, d.ss_, d.ctr + 11, b, g);
    }
};
struct FKeptList {
    QMD void operator()(const LsInst& d, int, int b, int g) const { d_kept_list(d.C, d.sk, d.kept, b, g); }
};
struct FInsert {
    QMD void operator()(const LsInst& d, int, int b, int g) const {
        const Mesh M = d.M;
        const Cands C = d.C;
        const Pools PL = d.PL;
        const BfPool BP = d.BP;
        d_insert(M, d.cls, C, PL, BP, d.kept, d.nkept, d.sk, d.st_, d.ss_, d.nv0, d.nt0, d.nss0, d.ctr + 14, b, g);
    }
};
struct FMisRelease {
    QMD void operator()(const LsInst& d, int, int b, int g) const { d_mis_release(d.ncl, d.PL.cl, d.PL.clc, d.owner, b, g); }
};

}  // namespace qm

namespace {

using namespace qm;

// host and device halves of the staging ring for the instance tables.  A
// region of the pinned half is the source of a copy that runs in stream
// order, so it may be written again only once that copy has run: the ring
// restarts only right after a stream synchronisation (synced(), called by
// the code that synchronised) or when it is full (put() synchronises).
struct LsStage {
    char* h = nullptr;
    DBuf<char> d;
    size_t cap = 0, off = 0;
    hipStream_t s;
    explicit LsStage(hipStream_t st) : s(st) {}
    ~LsStage() {
        if (h) (void)hipHostFree(h);
        d.release(s);
    }
    void reserve(size_t bytes) {
        if (bytes <= cap) return;
        HIPCK(hipStreamSynchronize(s));
        if (h) (void)hipHostFree(h);
        h = nullptr;
        cap = std::max(bytes, (size_t)4 << 20);
        HIPCK(hipHostMalloc((void**)&h, cap, hipHostMallocDefault));
        d.ensure_exact(cap, s);
        off = 0;
    }
    // copy n records to the device; returns their device address
    template <class T>
    const T* put(const T* src, size_t n) {
        const size_t bytes = ((n * sizeof(T)) + 255) & ~(size_t)255;
        if (off + bytes > cap) {            // full: wait for the copies in flight
            HIPCK(hipStreamSynchronize(s));
            off = 0;
            reserve(bytes);
        }
        std::memcpy(h + off, src, n * sizeof(T));
        HIPCK(hipMemcpyAsync(d.p + off, h + off, n * sizeof(T), hipMemcpyHostToDevice, s));
        const T* r = reinterpret_cast<const T*>(d.p + off);
        off += bytes;
        return r;
    }
    void synced() { off = 0; }
};

// One instance of a lockstep batch: its engine (all device buffers), result
// and round state.
struct LsJob {
    uint64_t tag = 0;
    const qm_options* opt = nullptr;
    qm_options opt_copy{};
    std::unique_ptr<Engine> E;
    std::unique_ptr<qm_result> R;
    qm_stats ST{};
    int round = 0, status = 0, last_ncand = 0;
    int round0 = 0;                 // rounds run before this set-up (a resumed refinement)
    int cls = CLS_NONE, ncand = 0, ncl = 0, nkept = 0, newt = 0, newss = 0, nover = 0, nbig = 0;
    int passes = 0, ncl_final = 0;
    int undecided = 0;              // selection: undecided candidates after the last batch
    bool small_sel = false, pool_done = false, sel_done = false;
    unsigned long long key_mask = ~0ull;
    int min_tier = 0;
    const int* hc = nullptr;        // its counters at the last gather
    std::chrono::steady_clock::time_point t_add, t_ready;
};

struct LsDone {
    uint64_t tag;
    qm_result* res;
    int code;
    std::string msg;
};

// launch-shape knobs of a lockstep batch (qm_lockstep_tune); none of them
// changes a result
struct LsTune {
    int classify_tiles = 8;       // 256-element tiles per classification workgroup
    int rank_max = LS_ORDER_CAP;  // candidates ordered in one workgroup (more: radix sort)
    int select_one_wg = MIS_SMALL;  // claims and candidates selected in one workgroup
    int hybrid_wgs = 1024;        // hybrid-tier workgroups over all instances
    int global_wgs = 256;         // global-tier workgroups over all instances
};

class Lockstep {
public:
    explicit Lockstep(hipStream_t s, const LsTune& t = LsTune()) : s_(s), stage_(s), tune_(t) {}
    ~Lockstep() {
        for (auto& d : done_) qm_result_free(d.res);
        jobs_.clear();
        hslab_.release(s_); gslab_.release(s_); gath_.release(s_);
        if (hgath_) (void)hipHostFree(hgath_);
        (void)hipStreamSynchronize(s_);
    }
    int live() const { return (int)jobs_.size(); }
    // Set an instance up on the device (resumed from `st` when given); it
    // takes part from the next step.  A failing set-up (or refused options)
    // ends it at once, in take_done().
    void add(const qm_plc* plc, const qm_mesh* in, const qm_options* opt, uint64_t tag,
             const qm_state* st = nullptr) {
        auto J = std::make_unique<LsJob>();
        J->tag = tag;
        J->t_add = std::chrono::steady_clock::now();
        try {
            if (!plc || !in || !opt) throw QmError(QM_EINVAL, "null argument");
            if (!(opt->B > 0.0) || !(opt->hmin_factor >= 0.0) || opt->max_rounds < 0)
                throw QmError(QM_EINVAL, "B must be > 0, hmin_factor >= 0, max_rounds >= 0");
            if (in->nv < 8 || in->nt < 1 || in->nsf < 0 || in->nss < 0 || plc->nftri < 0 || plc->nseg < 0)
                throw QmError(QM_EINVAL, "bad counts");
            if (in->nv >= (1 << 21)) throw QmError(QM_EINVAL, "input vertex count must be below 2^21");
            if (opt->flags & (QM_PROFILE | QM_PROFILE_GROW | QM_EARLY_STOP | QM_SUBPHASE_ROUNDS) || opt->max_kept > 0)
                throw QmError(QM_EINVAL, "the lockstep form takes no profiling, non-parity mode or insertion cap");
            J->opt_copy = *opt;
            J->opt = &J->opt_copy;
            J->key_mask = (opt->flags & QM_TEST_KEY_COLLIDE) ? 0xE000000000000000ull : ~0ull;
            J->min_tier = (opt->flags & QM_TEST_TIER2) ? 2 : (opt->flags & QM_TEST_TIER1) ? 1 : 0;
            if (st) check_state(in, st);
            J->round0 = st ? st->rounds : 0;
            J->E = std::make_unique<Engine>(s_);
            J->R = std::make_unique<qm_result>();
            setup_mesh(*J->E, plc, in, J->opt, nullptr, nullptr, st);
            J->t_ready = std::chrono::steady_clock::now();
            jobs_.push_back(std::move(J));
        } catch (const QmError& e) {
            fail(*J, e.code, e.what());
        } catch (const std::exception& e) {
            fail(*J, QM_EINTERNAL, e.what());
        }
    }
    // One round of every live instance; instances that finish (no candidate
    // left, round limit, failure) move to take_done().
    void step();
    // Between steps: take instance `tag` off the device.  Its mesh and state
    // go to a host result with status 2 in take_done(), a checkpoint that
    // add() resumes from.  False when no live instance has that tag.
    bool evict_now(uint64_t tag) {
        for (auto& P : jobs_) {
            if (!P->E || P->tag != tag) continue;
            LsJob& J = *P;
            int hc[48];
            HIPCK(hipMemcpyAsync(hc, J.E->ctr.p, sizeof hc, hipMemcpyDeviceToHost, s_));
            HIPCK(hipStreamSynchronize(s_));
            J.hc = hc;
            patch_last_record(J);
            J.hc = nullptr;
            J.status = 2;
            finish(J);
            compact();
            return true;
        }
        return false;
    }
    std::vector<LsDone> take_done() { return std::exchange(done_, {}); }

private:
    hipStream_t s_;
    LsStage stage_;
    LsTune tune_;
    std::vector<std::unique_ptr<LsJob>> jobs_;
    std::vector<LsDone> done_;
    std::vector<LsInst> table_;
    const LsInst* dtab_ = nullptr;
    DBuf<int> gath_;
    int* hgath_ = nullptr;
    size_t hgath_cap_ = 0;
    DBuf<char> hslab_, gslab_;

    void fail(LsJob& J, int code, const std::string& msg) {
        J.E.reset();                         // frees its buffers in stream order
        done_.push_back({J.tag, nullptr, code, msg});
    }
    // current device view of every live instance (one copy)
    void upload() {
        table_.resize(jobs_.size());
        for (size_t i = 0; i < jobs_.size(); ++i) {
            LsJob& J = *jobs_[i];
            if (!J.E) continue;                  // ended this step (never listed again)
            Engine& E = *J.E;
            LsInst& t = table_[i];
            t.M = E.M; t.C = E.C; t.PL = E.PL; t.BP = E.BP;
            t.ctr = E.ctr.p;
            t.c_elem0 = E.c_elem0.p; t.c_key0 = E.c_key0.p; t.c_tup0 = E.c_tup0.p; t.c_p0 = E.c_p0.p;
            t.c_st0 = E.c_st0.p; t.c_reason0 = E.c_reason0.p;
            t.olist = E.olist.p; t.glist = E.glist.p; t.sk = E.sk.p; t.st_ = E.st_.p; t.ss_ = E.ss_.p;
            t.kept = E.kept.p; t.ulist0 = E.ulist0.p; t.ulist1 = E.ulist1.p; t.mark = E.mark.p; t.owner = E.owner.p;
            t.mis_drop = E.mis_drop.p; t.mis_lose = E.mis_lose.p;
            t.key_mask = J.key_mask; t.pass = E.pass;
            t.cls = J.cls; t.ncand = J.ncand; t.ncl = J.ncl; t.nkept = J.nkept; t.min_tier = J.min_tier;
            t.nover = J.nover; t.nbig = J.nbig; t.nv0 = E.M.nv; t.nt0 = E.M.nt; t.nss0 = E.M.nss;
        }
        stage_.reserve(sizeof(LsInst) * table_.size() + 256);
        dtab_ = stage_.put(table_.data(), table_.size());
    }
    // one batched launch over the instances `idx` (indices into jobs_) with
    // blocks(i) workgroups each (instances with none are left out), in
    // launches of at most LS_PARTS parts
    template <int NT, class F, class B>
    void launch(const std::vector<int>& idx, B blocks, const F& f) {
        LsParts P;
        P.np = 0;
        P.pre[0] = 0;
        auto go = [&]() {
            if (!P.np) return;
            k_each<NT, F><<<P.pre[P.np], NT, 0, s_>>>(dtab_, P, f);
            P.np = 0;
            P.pre[0] = 0;
        };
        for (int i : idx) {
            const long nb = blocks(*jobs_[i]);
            if (nb <= 0) continue;
            if (P.np == LS_PARTS || (long)P.pre[P.np] + nb > (1L << 30)) go();
            P.map[P.np] = i;
            P.pre[P.np + 1] = P.pre[P.np] + (int)nb;
            ++P.np;
        }
        go();
    }
    // the counters of the instances `idx` to the host (one copy, one
    // synchronisation); J.hc points at each one's 48 values
    void gather(const std::vector<int>& idx) {
        const size_t n = idx.size();
        gath_.ensure(48 * std::max<size_t>(n, 1), s_, false);
        if (48 * n > hgath_cap_) {
            HIPCK(hipStreamSynchronize(s_));
            if (hgath_) (void)hipHostFree(hgath_);
            hgath_ = nullptr;
            hgath_cap_ = 48 * std::max<size_t>(n, 64);
            HIPCK(hipHostMalloc((void**)&hgath_, sizeof(int) * hgath_cap_, hipHostMallocDefault));
        }
        // parts in idx order: part k of chunk c is entry c * LS_PARTS + k
        for (size_t c = 0; c < n; c += LS_PARTS) {
            std::vector<int> sub(idx.begin() + c, idx.begin() + std::min(n, c + LS_PARTS));
            FGather g{gath_.p + 48 * c};
            launch<64>(sub, [](const LsJob&) { return 1L; }, g);
        }
        HIPCK(hipMemcpyAsync(hgath_, gath_.p, sizeof(int) * 48 * n, hipMemcpyDeviceToHost, s_));
        HIPCK(hipStreamSynchronize(s_));
        stage_.synced();
        for (size_t k = 0; k < n; ++k) jobs_[idx[k]]->hc = hgath_ + 48 * k;
    }
    void finish(LsJob& J);
    void patch_last_record(LsJob& J) {
        if (J.R->rounds.empty()) return;
        J.E->dead = J.hc[14];
        J.R->rounds[J.R->rounds.size() - QM_ROUND_FIELDS + 16] = J.E->M.nt - (int)J.E->dead;
    }
    void scans_large(LsJob& J);
    void sort_large(LsJob& J);
    // run fn on each listed job; a job whose host logic throws ends with
    // that error (its device work so far is harmless: nothing reads it)
    template <class Fn>
    void each(std::vector<int>& idx, Fn fn) {
        bool dropped = false;
        for (int i : idx) {
            LsJob& J = *jobs_[i];
            if (!J.E) continue;
            try {
                fn(J);
            } catch (const QmError& e) {
                fail(J, e.code, e.what());
                dropped = true;
            } catch (const std::exception& e) {
                fail(J, QM_EINTERNAL, e.what());
                dropped = true;
            }
        }
        if (dropped) idx.erase(std::remove_if(idx.begin(), idx.end(), [&](int i) { return !jobs_[i]->E; }), idx.end());
    }
    void compact() {        // drop finished and failed jobs from the live list
        jobs_.erase(std::remove_if(jobs_.begin(), jobs_.end(), [](const std::unique_ptr<LsJob>& J) { return !J->E; }),
                    jobs_.end());
    }
};

void Lockstep::finish(LsJob& J) {
    Engine& E = *J.E;
    if (J.last_ncand > 0) read_last_round(E, J.R.get(), J.last_ncand);
    const int gerr = read1(E.M.err, s_);
    if (gerr) throw QmError(QM_EINTERNAL, "exact predicate precondition failed (code " + std::to_string(gerr) + ")");
    if (J.status == 2) J.opt_copy.flags &= ~QM_OUTPUT_DEVICE;   // a checkpoint is kept on the host
    J.ST.nt_out = emit_output(E, J.R.get(), J.opt, nullptr, nullptr);
    const auto now = std::chrono::steady_clock::now();
    J.ST.rounds = J.round;
    J.ST.status = J.status;
    J.R->st_rounds = J.round0 + J.round;
    J.ST.device_bytes_peak = (int64_t)E.acct.peak;
    J.ST.nv_out = E.M.nv;
    J.ST.seconds_setup = std::chrono::duration<double>(J.t_ready - J.t_add).count();
    J.ST.seconds_refine = std::chrono::duration<double>(now - J.t_ready).count();
    J.ST.seconds_total = std::chrono::duration<double>(now - J.t_add).count();
    J.R->stats = J.ST;
    J.E.reset();
    done_.push_back({J.tag, J.R.release(), J.status == 1 ? QM_EROUNDS : QM_OK, ""});
}

// more than 256 candidates: radix sort by key, then the tie fix
void Lockstep::sort_large(LsJob& J) {
    Engine& E = *J.E;
    const int n = J.ncand;
    k_iota<<<nblk(n), 256, 0, s_>>>(n, E.order0.p);
    E.sort_desc(E.c_key0.p, E.skey.p, E.order0.p, E.order1.p, n);
    k_fix_ties<<<nblk(n), 256, 0, s_>>>(n, E.skey.p, E.order1.p, E.c_tup0.p);
    k_permute<<<nblk(n), 256, 0, s_>>>(n, E.order1.p, E.c_elem0.p, E.c_key0.p, E.c_tup0.p, E.c_p0.p, E.c_st0.p,
                                       E.c_reason0.p, E.C);
}

// more than SCAN_SMALL candidates: device-wide scans of the three values
void Lockstep::scans_large(LsJob& J) {
    Engine& E = *J.E;
    const int n = J.ncand;
    k_scan_vals<<<nblk(n), 256, 0, s_>>>(E.C, J.cls, E.vk.p, E.vt.p, E.vs.p);
    E.exscan(E.vk.p, E.sk.p, n);
    E.exscan(E.vt.p, E.st_.p, n);
    E.exscan(E.vs.p, E.ss_.p, n);
    k_totals<<<1, 1, 0, s_>>>(n, E.sk.p, E.vk.p, E.st_.p, E.vt.p, E.ss_.p, E.vs.p, E.ctr.p + 11);
}

void Lockstep::step() {
    std::vector<int> L(jobs_.size());
    for (size_t i = 0; i < jobs_.size(); ++i) L[i] = (int)i;
    // round start: the round limit, slot renumbering, candidate space
    each(L, [&](LsJob& J) {
        Engine& E = *J.E;
        if (J.round >= J.opt->max_rounds) {
            int hc[48];
            HIPCK(hipMemcpyAsync(hc, E.ctr.p, sizeof hc, hipMemcpyDeviceToHost, s_));
            HIPCK(hipStreamSynchronize(s_));
            J.hc = hc;
            patch_last_record(J);
            J.hc = nullptr;
            J.status = 1;
            finish(J);
            return;
        }
        if (E.M.nt - E.nt_ordered > std::max(E.M.nt / 10, 65536)) E.reorder();
        E.c_elem0.ensure(std::max((size_t)E.M.nss, 4 * (size_t)E.M.nt), s_, false);
    });
    L.erase(std::remove_if(L.begin(), L.end(), [&](int i) { return !jobs_[i]->E; }), L.end());
    if (L.empty()) { compact(); return; }
    // step 1: classify (the staging ring is not rewound here: the last
    // round's insertion table may still be waiting for its copy)
    upload();
    launch<64>(L, [](const LsJob&) { return 1L; }, FReset{});
    const int ct = tune_.classify_tiles;
    launch<256>(L, [ct](const LsJob& J) { return J.E->M.nss ? (long)nblk(J.E->M.nss, 256 * ct) : 0L; },
                FClassifySS{ct});
    launch<256>(L, [ct](const LsJob& J) { return (long)nblk(J.E->M.nt, 256 * ct); }, FClassifySF{ct});
    launch<256>(L, [ct](const LsJob& J) { return (long)nblk(J.E->M.nt, 256 * ct); }, FClassifyTet{ct});
    gather(L);
    each(L, [&](LsJob& J) {
        patch_last_record(J);
        J.cls = CLS_NONE;
        J.ncand = 0;
        for (int c = CLS_SS; c <= CLS_TET && J.cls == CLS_NONE; ++c)
            if (J.hc[8 + c] > 0) { J.cls = c; J.ncand = J.hc[8 + c]; }
        if (J.cls == CLS_NONE) { finish(J); return; }
        Engine& E = *J.E;
        E.ensure_cands(J.ncand);
        E.ensure_pools(E.pool_need(1, J.ncand, J.cls), E.pool_need(2, J.ncand, J.cls), E.pool_need(3, J.ncand, J.cls),
                       E.pool_need(4, J.ncand, J.cls));
        J.pool_done = false;
        J.nover = J.nbig = 0;
    });
    L.erase(std::remove_if(L.begin(), L.end(), [&](int i) { return !jobs_[i]->E; }), L.end());
    if (L.empty()) { compact(); return; }
    // step 2: splitting points, priorities and their order
    upload();
    launch<256>(L, [](const LsJob& J) { return (long)nblk(J.ncand); }, FSplit{});
    launch<SORT_SMALL>(L, [](const LsJob& J) { return J.ncand <= SORT_SMALL ? 1L : 0L; }, FOrderSmall{});
    const int rmax = tune_.rank_max;
    launch<1024>(L, [rmax](const LsJob& J) { return J.ncand > SORT_SMALL && J.ncand <= rmax ? 1L : 0L; },
                 FOrderMid{});
    each(L, [&](LsJob& J) { if (J.ncand > SORT_SMALL && J.ncand > rmax) sort_large(J); });
    // step 3: locate
    launch<64>(L, [](const LsJob& J) { return J.cls != CLS_SS ? (long)nblk(J.ncand, 64) : 0L; }, FLocate{});
    // steps 4-5: grow and validate; a pass is repeated (with larger pools) by
    // the instances whose result pools were full
    std::vector<int> P = L;
    for (int pass = 0; !P.empty(); ++pass) {
        if (pass > 0) {
            upload();
            launch<64>(P, [](const LsJob&) { return 1L; }, FResetPools{});
        }
        launch<64>(P, [](const LsJob& J) { return (long)std::min(J.ncand, 16384); }, FGrowSmall{});
        std::vector<int> A = P;
        for (int attempt = 0; !A.empty(); ++attempt) {
            launch<64>(A, [](const LsJob&) { return 1L; }, FListReset{});
            launch<256>(A, [](const LsJob& J) { return (long)nblk(J.ncand); }, FOverflowList{});
            gather(A);
            long hyb_total = 0, big_total = 0;
            each(A, [&](LsJob& J) {
                J.nover = J.hc[32];
                J.nbig = J.hc[36];
                if (J.hc[34])
                    throw QmError(QM_ECAPACITY, "a region exceeds the largest supported size (round " +
                                                    std::to_string(J.round) + ", class " + std::to_string(J.cls) + ")");
                if (J.nover + J.nbig == 0) {            // this pass is evaluated: were the pools large enough?
                    if (!J.hc[5]) {
                        J.E->pool_seen(J.hc, J.ncand, J.cls);
                        J.ncl_final = J.hc[3];
                        J.pool_done = true;
                    } else {
                        if (pass >= 8) throw QmError(QM_ENOMEM, "result pools kept overflowing");
                        Engine& E = *J.E;
                        auto need = [](int used, size_t cap) {
                            return std::max(cap, (size_t)used + (size_t)used / 8 + 4096);
                        };
                        E.ensure_pools(need(J.hc[1], E.p_bfr.cap / BFR), need(J.hc[2], E.p_be.cap),
                                       need(J.hc[3], E.p_cl.cap), need(J.hc[4], E.p_q.cap));
                    }
                    return;
                }
                if (attempt >= 64) throw QmError(QM_EINTERNAL, "regions kept outgrowing the tiles");
                hyb_total += std::min(J.nover, 1024);
                big_total += std::min(J.nbig, 1024);
            });
            A.erase(std::remove_if(A.begin(), A.end(), [&](int i) { return !jobs_[i]->E || jobs_[i]->nover + jobs_[i]->nbig == 0; }),
                    A.end());
            if (A.empty()) break;
            upload();
            if (hyb_total > 0) {            // hybrid tier: at most 1024 workgroups over all instances
                const GrowTiles HT = hybrid_tiles();
                const size_t block = lists_slab_bytes(HT);
                const long cap = tune_.hybrid_wgs;
                auto share = [&](const LsJob& J) -> long {
                    if (J.nover <= 0) return 0L;
                    const long want = std::min(J.nover, 1024);
                    return hyb_total <= cap ? want : std::max(1L, want * cap / hyb_total);
                };
                long total = 0;
                for (int i : A) total += share(*jobs_[i]);
                hslab_.ensure(block * (size_t)std::min<long>(total, LS_PARTS * 1024L), s_, false);
                launch<H_LANES>(A, share, FGrowHybrid{HT, hslab_.p, block});
            }
            if (big_total > 0) {            // global-memory tiles: at most 256 workgroups over all instances
                GrowTiles BT{};
                BT.maxrt = B_MAXRT; BT.hcap = B_HCAP; BT.rfhcap = B_RFHCAP; BT.maxrf = B_MAXRF; BT.maxbe = B_MAXBE;
                BT.qhcap = B_QHCAP; BT.maxq = B_MAXQ; BT.maxbf = B_MAXBF; BT.maxcx = B_MAXBF; BT.tier = 2;
                BT.ehcap = 1;
                while (BT.ehcap < 2 * (3 * BT.maxbf + BT.maxbe)) BT.ehcap <<= 1;
                const size_t block = grow_slab_bytes(BT);
                const long cap = tune_.global_wgs;
                auto share = [&](const LsJob& J) -> long {
                    if (J.nbig <= 0) return 0L;
                    const long want = std::min(J.nbig, 1024);
                    return big_total <= cap ? want : std::max(1L, want * cap / big_total);
                };
                long total = 0;
                for (int i : A) total += share(*jobs_[i]);
                gslab_.ensure(block * (size_t)std::min<long>(total, LS_PARTS * 1024L), s_, false);
                launch<B_LANES>(A, share, FGrowGlobal{BT, gslab_.p, block});
            }
        }
        P.erase(std::remove_if(P.begin(), P.end(), [&](int i) { return !jobs_[i]->E || jobs_[i]->pool_done; }), P.end());
    }
    L.erase(std::remove_if(L.begin(), L.end(), [&](int i) { return !jobs_[i]->E; }), L.end());
    if (L.empty()) { compact(); return; }
    // verdicts, then step 6: selection, with the step-7 scans
    each(L, [&](LsJob& J) {
        Engine& E = *J.E;
        J.ncl = std::min(J.ncl_final, E.PL.cap_cl);
        J.small_sel = J.ncl > 0 && J.ncl <= tune_.select_one_wg && J.ncand <= tune_.select_one_wg;
        J.sel_done = false;
        J.passes = 0;
    });
    upload();
    launch<256>(L, [](const LsJob& J) { return (long)nblk(J.ncand); }, FVerdicts{});
    launch<1024>(L, [](const LsJob& J) { return J.small_sel ? 1L : 0L; }, FMisSmall{});
    // the other selections: batches of MIS_BATCH passes over several
    // workgroups per instance, one look at the undecided counts per batch
    std::vector<int> S;
    for (int i : L)
        if (jobs_[i]->ncl > 0 && !jobs_[i]->small_sel) S.push_back(i);
    for (int batch = 0; !S.empty(); ++batch) {
        if (batch > 0) {
            upload();                       // pass stamps moved on
            launch<64>(S, [](const LsJob&) { return 1L; }, FUndecReset{});
        }
        for (int b = 0; b < MIS_BATCH; ++b) {
            const int p = batch * MIS_BATCH + b;
            if (p == 0) {
                launch<256>(S, [](const LsJob& J) { return (long)nblk(J.ncl); }, FMisMark{b});
                launch<256>(S, [](const LsJob& J) { return (long)nblk(J.ncl); }, FMisCheck{b});
                launch<256>(S, [](const LsJob& J) { return (long)nblk(J.ncand); }, FMisDecide{b});
                launch<256>(S, [](const LsJob& J) { return (long)nblk(J.ncl); }, FMisCommit{});
            } else {                        // list lengths are bounded by the last undecided count
                auto wave = [](const LsJob& J) { return (long)std::min(MIS_LIST_GRID, nblk(J.undecided, 4)); };
                auto lane = [](const LsJob& J) { return (long)std::min(MIS_LIST_GRID / 4, nblk(J.undecided)); };
                launch<256>(S, wave, FMisMarkList{b, p});
                launch<256>(S, wave, FMisCheckList{b, p});
                launch<256>(S, lane, FMisDecideList{b, p});
                launch<256>(S, wave, FMisCommitList{p});
            }
            if (p == 0) for (int i : S) jobs_[i]->undecided = jobs_[i]->ncand;
        }
        gather(S);
        each(S, [&](LsJob& J) {
            for (int b = 0; b < MIS_BATCH; ++b) {
                ++J.passes;
                if (J.hc[40 + b] == 0) break;
            }
            J.E->pass += MIS_BATCH;
            J.undecided = J.hc[40 + MIS_BATCH - 1];
            J.sel_done = J.undecided == 0;
        });
        S.erase(std::remove_if(S.begin(), S.end(), [&](int i) { return !jobs_[i]->E || jobs_[i]->sel_done; }),
                S.end());
    }
    L.erase(std::remove_if(L.begin(), L.end(), [&](int i) { return !jobs_[i]->E; }), L.end());
    if (L.empty()) { compact(); return; }
    // step-7 scans (kept ids, new tet slots, new subsegment slots)
    launch<1024>(L, [](const LsJob& J) { return J.ncand <= SCAN_SMALL ? 1L : 0L; }, FScanSmall{});
    each(L, [&](LsJob& J) { if (J.ncand > SCAN_SMALL) scans_large(J); });
    gather(L);
    // step 7: insertion
    each(L, [&](LsJob& J) {
        Engine& E = *J.E;
        if (J.small_sel) {
            if (J.hc[38] < 0) throw QmError(QM_EINTERNAL, "selection did not finish");
            J.passes = J.hc[38];
            E.pass += (unsigned)J.passes;
        }
        J.nkept = J.hc[11];
        J.newt = J.hc[12];
        J.newss = J.hc[13];
        if (J.hc[16 + 13]) throw QmError(QM_EINTERNAL, "candidate left unresolved");
        if (J.nkept > 0) E.ensure_mesh(E.M.nv + J.nkept, E.M.nt + J.newt, E.M.nss + J.newss);
    });
    upload();
    launch<256>(L, [](const LsJob& J) { return J.nkept > 0 ? (long)nblk(J.ncand) : 0L; }, FKeptList{});
    launch<64>(L, [](const LsJob& J) { return (long)std::min(J.nkept, 16384); }, FInsert{});
    launch<256>(L, [](const LsJob& J) { return J.ncl > 0 ? (long)nblk(J.ncl) : 0L; }, FMisRelease{});
    each(L, [&](LsJob& J) {
        Engine& E = *J.E;
        const int* st = J.hc + 16;
        E.M.nv += J.nkept; E.M.nt += J.newt; E.M.nss += J.newss;
        int rec[QM_ROUND_FIELDS] = {J.cls, st[0], st[1], st[2], st[3], J.nkept};
        for (int r = 1; r < EX_NREASON; ++r) rec[5 + r] = st[3 + r];
        rec[15] = E.M.nv;
        rec[16] = E.M.nt - (int)E.dead;   // completed at the next synchronisation
        J.R->rounds.insert(J.R->rounds.end(), rec, rec + QM_ROUND_FIELDS);
        J.ST.inserted[J.cls] += J.nkept;
        J.last_ncand = J.ncand;
        J.ST.candidates += J.ncand;
        J.ST.mis_passes += J.passes;
        J.ST.deferred += st[14];
        ++J.round;
    });
    compact();
}

// A whole lockstep batch: instances dealt, largest input first in snake
// order, to `groups` groups (one on `s`, or each on a stream and host thread
// of its own).  Returns 0 or the first group failure (message in err).
int lockstep_run(int32_t n, const qm_plc* plcs, const qm_mesh* meshes, const qm_options* opts, hipStream_t s,
                 const LsTune& tune, int groups, qm_result** outs, int32_t* codes, std::vector<std::string>& msgs,
                 std::string& err) {
    for (int i = 0; i < n; ++i) { outs[i] = nullptr; codes[i] = QM_EINTERNAL; }
    msgs.assign(n, std::string());
    const int G = std::max(1, std::min<int>(groups, n));
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return meshes[a].nt > meshes[b].nt; });
    std::vector<std::vector<int>> part(G);
    for (int k = 0; k < n; ++k) {
        const int r = k / G, c = k % G;
        part[(r & 1) ? G - 1 - c : c].push_back(order[k]);
    }
    std::vector<int> gcode(G, QM_OK);
    std::vector<std::string> gmsg(G);
    auto run = [&](int g, hipStream_t st) {
        try {
            Lockstep B(st, tune);
            auto collect = [&]() {
                for (auto& d : B.take_done()) {
                    outs[d.tag] = d.res;
                    codes[d.tag] = d.code;
                    msgs[d.tag] = d.msg;
                }
            };
            for (int i : part[g]) B.add(&plcs[i], &meshes[i], &opts[i], (uint64_t)i);
            collect();
            while (B.live() > 0) {
                B.step();
                collect();
            }
        } catch (const QmError& e) {
            gcode[g] = e.code;
            gmsg[g] = e.what();
        } catch (const std::exception& e) {
            gcode[g] = QM_EINTERNAL;
            gmsg[g] = e.what();
        }
    };
    if (G == 1) {
        run(0, s);
    } else {                      // one stream (default priority) and one host thread per group
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) { err = "no HIP device"; return QM_EDEVICE; }
        std::vector<std::thread> th;
        for (int g = 0; g < G; ++g)
            th.emplace_back([&, g]() {
                hipStream_t st = nullptr;
                if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                    gcode[g] = QM_EDEVICE;
                    gmsg[g] = "no stream for a lockstep group";
                    return;
                }
                run(g, st);
                (void)hipStreamSynchronize(st);
                (void)hipStreamDestroy(st);
            });
        for (auto& t : th) t.join();
    }
    for (int g = 0; g < G; ++g)
        if (gcode[g] != QM_OK) {
            err = gmsg[g];
            return gcode[g];
        }
    for (int i = 0; i < n; ++i)
        if (codes[i] != QM_OK && codes[i] != QM_EROUNDS) {
            err = "instance " + std::to_string(i) + ": " + msgs[i];
            return codes[i];
        }
    return QM_OK;
}

// the library's knobs from the caller's struct (NULL: defaults), checked
int tune_from(const qm_lockstep_tune* t, LsTune& out, int& groups) {
    out = LsTune();
    groups = 1;
    if (!t) return QM_OK;
    if (t->groups < 1 || t->groups > 64 || t->classify_tiles < 1 || t->classify_tiles > 64 || t->rank_max < SORT_SMALL ||
        t->rank_max > LS_ORDER_CAP || t->select_one_wg < 0 || t->select_one_wg > (1 << 20) || t->hybrid_wgs < 16 ||
        t->hybrid_wgs > 4096 || t->global_wgs < 4 || t->global_wgs > 1024)
        return QM_EINVAL;
    groups = t->groups;
    out.classify_tiles = t->classify_tiles;
    out.rank_max = t->rank_max;
    out.select_one_wg = t->select_one_wg;
    out.hybrid_wgs = t->hybrid_wgs;
    out.global_wgs = t->global_wgs;
    return QM_OK;
}

void tune_to(const LsTune& t, int groups, qm_lockstep_tune* out) {
    out->groups = groups;
    out->classify_tiles = t.classify_tiles;
    out->rank_max = t.rank_max;
    out->select_one_wg = t.select_one_wg;
    out->hybrid_wgs = t.hybrid_wgs;
    out->global_wgs = t.global_wgs;
}

}  // namespace

extern "C" {

int qm_refine_lockstep(int32_t n, const qm_plc* plcs, const qm_mesh* meshes, const qm_options* opts,
                       void* hip_stream, const qm_lockstep_tune* tune, qm_result** outs, int32_t* codes) {
    g_err.clear();
    LsTune t;
    int groups = 1;
    if (n < 0 || (n > 0 && (!plcs || !meshes || !opts || !outs || !codes)) || tune_from(tune, t, groups) != QM_OK) {
        g_err = "bad batch arguments";
        return QM_EINVAL;
    }
    std::vector<std::string> msgs;
    std::string err;
    const int rc = lockstep_run(n, plcs, meshes, opts, (hipStream_t)hip_stream, t, groups, outs, codes, msgs, err);
    if (rc != QM_OK) g_err = err;
    return rc;
}

// Coordinate descent over the knobs on a probe batch (instances evenly
// spaced in input size): each knob in turn takes the value whose run of the
// probe is fastest (a change must gain 3%); the results of the probe runs
// are freed.
int qm_lockstep_autotune(int32_t n, const qm_plc* plcs, const qm_mesh* meshes, const qm_options* opts,
                         int32_t probe, qm_lockstep_tune* best, double* best_seconds) {
    g_err.clear();
    if (n < 1 || !plcs || !meshes || !opts || !best || probe < 1) {
        g_err = "bad tuning arguments";
        return QM_EINVAL;
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return meshes[a].nt < meshes[b].nt; });
    const int p = std::min<int>(probe, n);
    std::vector<qm_plc> P(p);
    std::vector<qm_mesh> Mh(p);
    std::vector<qm_options> O(p);
    for (int k = 0; k < p; ++k) {
        const int i = order[p == 1 ? n - 1 : (int)((long)k * (n - 1) / (p - 1))];
        P[k] = plcs[i]; Mh[k] = meshes[i]; O[k] = opts[i];
    }
    std::vector<qm_result*> outs(p, nullptr);
    std::vector<int32_t> codes(p, 0);
    std::vector<std::string> msgs;
    auto timed = [&](const LsTune& t, int groups, double& sec) -> int {
        std::string err;
        const auto a = std::chrono::steady_clock::now();
        const int rc = lockstep_run(p, P.data(), Mh.data(), O.data(), nullptr, t, groups, outs.data(), codes.data(),
                                    msgs, err);
        sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
        for (auto*& r : outs) { qm_result_free(r); r = nullptr; }
        if (rc != QM_OK) g_err = "probe batch failed: " + err;
        return rc;
    };
    LsTune cur;
    int groups = 4;
    double cur_s = 0;
    int rc = timed(cur, groups, cur_s);
    if (rc != QM_OK) return rc;
    auto consider = [&](LsTune t, int g) -> int {
        double sec = 0;
        const int r = timed(t, g, sec);
        if (r != QM_OK) return r;
        if (sec < 0.97 * cur_s) { cur = t; groups = g; cur_s = sec; }
        return QM_OK;
    };
    for (int g : {1, 2, 8})
        if ((rc = consider(cur, g)) != QM_OK) return rc;
    for (int v : {256, 512, 2048}) {
        LsTune t = cur; t.hybrid_wgs = v;
        if (v != cur.hybrid_wgs && (rc = consider(t, groups)) != QM_OK) return rc;
    }
    for (int v : {2, 32}) {
        LsTune t = cur; t.classify_tiles = v;
        if (v != cur.classify_tiles && (rc = consider(t, groups)) != QM_OK) return rc;
    }
    for (int v : {8192, 262144}) {
        LsTune t = cur; t.select_one_wg = v;
        if (v != cur.select_one_wg && (rc = consider(t, groups)) != QM_OK) return rc;
    }
    {
        LsTune t = cur; t.rank_max = 1024;
        if ((rc = consider(t, groups)) != QM_OK) return rc;
    }
    tune_to(cur, groups, best);
    if (best_seconds) *best_seconds = cur_s;
    return QM_OK;
}

}  // extern "C"
