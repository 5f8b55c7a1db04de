// qm_lib.hip -- host driver of the round loop and the C-ABI (include/qm.h).
//
// One call = upload (or adopt device arrays) -> device setup -> rounds until
// no candidate is left -> compact and download.  Everything between setup
// and download runs on the GPU; the host only reads a few counters per round
// (class choice, overflow, selection passes, totals) to size launches and
// buffers.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>
#include <utility>
#include <thread>
#include <atomic>
#include <memory>
#include <mutex>
#include <condition_variable>

#include "qm.h"
#include "qm_insert.h"
#include "qm_round.h"
#include "qm_setup.h"

namespace {

thread_local std::string g_err;

struct QmError : std::runtime_error {
    int code;
    QmError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCK(x)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess)                                                                 \
            throw QmError(e_ == hipErrorOutOfMemory ? QM_ENOMEM : QM_EDEVICE,                 \
                          std::string(#x) + ": " + hipGetErrorString(e_));                   \
    } while (0)

inline int nblk(long n, int b = 256) { return (int)std::max(1L, (n + b - 1) / b); }

// Bump allocator over one device region: the no-alloc entry point carves
// every buffer of a call from the library's static scratch array.  `mark`
// separates what lives for the whole call (mesh arrays, counters) from what
// a round carves again (candidates, pools, tiles, sort scratch).
struct Arena {
    char* base = nullptr;
    size_t cap = 0, top = 0, mark = 0, high = 0;
    void* take(size_t bytes) {
        const size_t off = (top + 255) & ~(size_t)255;
        if (off + bytes > cap)
            throw QmError(QM_ECAPACITY, "the no-alloc scratch (" + std::to_string(cap >> 20) +
                                            " MiB) is too small for this refinement (" +
                                            std::to_string((off + bytes) >> 20) + " MiB needed so far)");
        top = off + bytes;
        high = std::max(high, top);
        return base + off;
    }
};

// device bytes a call holds (allocated and not yet freed) and their peak
struct Acct {
    size_t now = 0, peak = 0;
    void add(size_t b) { now += b; peak = std::max(peak, now); }
    void sub(size_t b) { now -= std::min(now, b); }
};

// growable device buffer (contents kept on growth when asked); with an
// arena it is carved from the arena and never freed
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t cap = 0;
    Arena* ar = nullptr;
    Acct* acct = nullptr;
    void ensure(size_t n, hipStream_t s, bool keep, int fill_byte = -1) {
        if (n <= cap) return;
        size_t nc = ar ? n : std::max(n, cap + cap / 2 + 1024);
        if (!keep && p && !ar) {        // contents not needed: free first, so both never coexist
            HIPCK(hipFreeAsync(p, s));
            if (acct) acct->sub(cap * sizeof(T));
            p = nullptr;
            cap = 0;
        }
        T* q = nullptr;
        if (ar) q = (T*)ar->take(nc * sizeof(T));
        else HIPCK(hipMallocAsync((void**)&q, nc * sizeof(T), s));
        if (acct && !ar) acct->add(nc * sizeof(T));
        if (fill_byte >= 0) HIPCK(hipMemsetAsync(q, fill_byte, nc * sizeof(T), s));
        if (keep && p && cap) HIPCK(hipMemcpyAsync(q, p, cap * sizeof(T), hipMemcpyDeviceToDevice, s));
        if (p && !ar) {
            HIPCK(hipFreeAsync(p, s));
            if (acct) acct->sub(cap * sizeof(T));
        }
        p = q;
        cap = nc;
    }
    void release(hipStream_t s) {
        if (p && !ar) {
            (void)hipFreeAsync(p, s);
            if (acct) acct->sub(cap * sizeof(T));
        }
        p = nullptr;
        cap = 0;
    }
    // exactly n elements (no growth slack), contents not kept
    void ensure_exact(size_t n, hipStream_t s) {
        if (n <= cap) return;
        release(s);
        if (ar) p = (T*)ar->take(n * sizeof(T));
        else {
            HIPCK(hipMallocAsync((void**)&p, n * sizeof(T), s));
            if (acct) acct->add(n * sizeof(T));
        }
        cap = n;
    }
};

// pinned host ints (hipHostMalloc), freed with the owner
struct PinnedInts {
    int* p = nullptr;
    explicit PinnedInts(size_t n) {
        if (hipHostMalloc((void**)&p, n * sizeof(int), hipHostMallocDefault) != hipSuccess || !p)
            throw std::runtime_error("pinned host allocation failed");
    }
    ~PinnedInts() { if (p) (void)hipHostFree(p); }
    PinnedInts(const PinnedInts&) = delete;
    PinnedInts& operator=(const PinnedInts&) = delete;
};

template <class T>
T read1(const T* dptr, hipStream_t s) {
    T v;
    HIPCK(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    return v;
}

}  // namespace

struct qm_result {
    std::vector<double> xyz;
    std::vector<int32_t> tets, sf, sff, ss, ssg;
    // QM_OUTPUT_DEVICE: the output arrays stay on the device (hipMalloc)
    bool on_device = false;
    double* d_xyz = nullptr;
    int32_t *d_tets = nullptr, *d_sf = nullptr, *d_sff = nullptr, *d_ss = nullptr, *d_ssg = nullptr;
    int32_t dnv = 0, dnt = 0, dnsf = 0, dnss = 0;
    ~qm_result() {
        for (void* p : {(void*)d_xyz, (void*)d_tets, (void*)d_sf, (void*)d_sff, (void*)d_ss, (void*)d_ssg})
            if (p) (void)hipFree(p);
    }
    std::vector<int32_t> rounds;   // QM_ROUND_FIELDS per round
    std::vector<int32_t> last;     // last round's candidates, 9 per candidate
    std::vector<double> round_ms;  // QM_PROFILE: QM_PROF_FAMILIES device ms per round
    qm_stats stats;
    // refinement state of the output (qm_result_state), host arrays aligned
    // with the output mesh
    std::vector<uint8_t> st_tfl, st_sfl, st_ssl;
    double st_hmin2 = 0.0;
    int32_t st_rounds = 0, st_next = 0;
};

namespace qm {

// round start: zero the round's counters (all of ctr[0..48) except the
// totals and the running dead-slot count, ctr[11..15))
__global__ void k_round_reset(int* ctr) {
    int i = threadIdx.x;
    if (i < 48 && (i < 11 || i >= 15)) ctr[i] = 0;
}

// ---- exclusive prefix sums (ints), SCAN_TILE elements per 256-lane
// workgroup: each lane sums 16 consecutive elements, the lanes' sums are
// scanned across the workgroup (wave shuffles, then the four wave totals)
constexpr int SCAN_TILE = 4096;
QMD int block_exclusive_256(int v, int* total) {
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int pre = 0;
    for (int i = 0; i < w; ++i) pre += wsum[i];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return pre + x - v;
}
__global__ __launch_bounds__(256) void k_scan_tile_sums(int n, const int* in, int* sums) {
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * 16;
    int v = 0;
    for (int j = 0; j < 16; ++j) v += base + j < n ? in[base + j] : 0;
    int total;
    block_exclusive_256(v, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}
__global__ __launch_bounds__(1024) void k_scan_sums(int m, int* sums) {   // in place, exclusive
    __shared__ int wsum[16];
    __shared__ int carry;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < m; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < m ? sums[i] : 0;
        int x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        int pre = carry;
        for (int k = 0; k < w; ++k) pre += wsum[k];
        if (i < m) sums[i] = pre + x - v;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = 0; k < 16; ++k) carry += wsum[k];
        __syncthreads();
    }
}
__global__ __launch_bounds__(256) void k_scan_tile(int n, const int* in, int* out, const int* offs) {
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * 16;
    int e[16], v = 0;
    for (int j = 0; j < 16; ++j) { e[j] = base + j < n ? in[base + j] : 0; v += e[j]; }
    int total;
    int run = block_exclusive_256(v, &total) + (offs ? offs[blockIdx.x] : 0);
    for (int j = 0; j < 16; ++j) {
        if (base + j < n) out[base + j] = run;
        run += e[j];
    }
}

// Priority order of a small round (n <= SORT_SMALL candidates), one
// workgroup: each candidate's position is its rank under the round's order
// (larger key first; equal keys by ascending tuple, then by index), the
// order the radix sort and the tie fix give together; the candidate is
// written straight to that position of the ordered arrays.
constexpr int SORT_SMALL = 256;
QMD void d_order_small(int n, const int* elem, const unsigned long long* key,
                                                           const int4* tup, const double4* p, const int* st,
                                                           const int* reason, Cands C, const int bid, const int gdim) {
    __shared__ unsigned long long K[SORT_SMALL];
    __shared__ int4 T[SORT_SMALL];
    const int i = threadIdx.x;
    if (i < n) { K[i] = key[i]; T[i] = tup[i]; }
    __syncthreads();
    if (i >= n) return;
    const unsigned long long ki = K[i];
    const int4 ti = T[i];
    int r = 0;
    for (int j = 0; j < n; ++j) {
        const unsigned long long kj = K[j];
        if (kj > ki) { ++r; continue; }
        if (kj != ki || j == i) continue;
        const int4 tj = T[j];
        r += tj.x != ti.x ? tj.x < ti.x : tj.y != ti.y ? tj.y < ti.y : tj.z != ti.z ? tj.z < ti.z
           : tj.w != ti.w ? tj.w < ti.w : j < i;
    }
    C.elem[r] = elem[i]; C.key[r] = ki; C.tup[r] = ti; C.p[r] = p[i];
    C.st[r] = st[i]; C.reason[r] = reason[i];
    C.seed[r] = -1; C.qw[r] = make_int2(-1, -1);
}
__global__ __launch_bounds__(SORT_SMALL) void k_order_small(int n, const int* elem, const unsigned long long* key,
                                                           const int4* tup, const double4* p, const int* st,
                                                           const int* reason, Cands C) {
    d_order_small(n, elem, key, tup, p, st, reason, C, blockIdx.x, gridDim.x);
}

// Priority order of a mid-size round (up to CAP candidates) in one
// workgroup of NT lanes: the same rank rule as k_order_small, keys staged in
// LDS, tuples read only for equal keys.
template <int NT, int CAP>
QMD void d_order_rank(int n, const int* elem, const unsigned long long* key, const int4* tup, const double4* p,
                      const int* st, const int* reason, Cands C) {
    __shared__ unsigned long long K[CAP];
    for (int i = threadIdx.x; i < n; i += NT) K[i] = key[i];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) {
        const unsigned long long ki = K[i];
        int r = 0, eq = 0;
        for (int j = 0; j < n; ++j) {
            const unsigned long long kj = K[j];
            r += kj > ki;
            eq += kj == ki;
        }
        if (eq > 1) {                                 // equal keys: ascending tuple, then index
            const int4 ti = tup[i];
            for (int j = 0; j < n; ++j) {
                if (K[j] != ki || j == i) continue;
                const int4 tj = tup[j];
                r += tj.x != ti.x ? tj.x < ti.x : tj.y != ti.y ? tj.y < ti.y : tj.z != ti.z ? tj.z < ti.z
                   : tj.w != ti.w ? tj.w < ti.w : j < i;
            }
        }
        C.elem[r] = elem[i]; C.key[r] = ki; C.tup[r] = tup[i]; C.p[r] = p[i];
        C.st[r] = st[i]; C.reason[r] = reason[i];
        C.seed[r] = -1; C.qw[r] = make_int2(-1, -1);
    }
}

__global__ void k_iota(int n, int* o) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = i;
}
__global__ void k_fill(int n, int* o, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = v;
}
// candidates to evaluate again: regions over the small LDS tiles (list a,
// count n[0]) and regions over the medium LDS tiles or the global-memory
// tiles (list c, n[4]); n[1] counts candidates whose results did not fit a
// pool, n[2] the regions over the global-memory tiles
QMD void d_overflow_list(Cands C, int* la, int* lc, int* n, const int bid, const int gdim) {
    int i = bid * blockDim.x + threadIdx.x;
    if (i >= C.n || C.st[i] != ST_PENDING) return;
    const int g = C.gst[i];
    if (g == ST_OVERFLOW) la[atomicAdd(&n[0], 1)] = i;
    else if (g == ST_POOLFULL) atomicAdd(&n[1], 1);
    else if (g == ST_OVERFLOW2 || g == ST_TOOBIG) lc[atomicAdd(&n[4], 1)] = i;
    if (g == ST_TOOBIG) atomicAdd(&n[2], 1);
}
__global__ void k_overflow_list(Cands C, int* la, int* lc, int* n) {
    d_overflow_list(C, la, lc, n, blockIdx.x, gridDim.x);
}
// a pass over again: zero the pool counters and the full flag
__global__ void k_round_reset_pools(int* ctr) {
    int i = threadIdx.x;
    if (i < 8) ctr[i] = 0;
}

// LDS tiles of the fast grow path (one 64-lane workgroup per candidate)
// (about 12 KB: 12 workgroups per CU, the register limit of this kernel)
constexpr int G_MAXRT = 192, G_HCAP = 512, G_RFHCAP = 128, G_MAXRF = 48, G_MAXBE = 64, G_QHCAP = 128,
              G_MAXQ = 64, G_MAXBF = 192;
#define QM_TILES_SMALL 64, 0, G_MAXRT, G_HCAP, G_RFHCAP, G_MAXRF, G_MAXBE, G_QHCAP, G_MAXQ, G_MAXBF, 0
// hybrid tier for the regions over the small tiles: hash tables in LDS
// (72 KB: two 256-lane workgroups per CU), lists and face records in a
// global slab (H_SLAB bytes per workgroup); up to 12288 tested tets
constexpr int H_LANES = 256, B_LANES = 256;   // workgroup widths of the hybrid and global tiers
constexpr int H_HCAP = 16384, H_RFHCAP = 1024, H_QHCAP = 512;
inline GrowTiles hybrid_tiles() {
    GrowTiles T{};
    T.maxrt = 3 * H_HCAP / 4; T.hcap = H_HCAP; T.rfhcap = H_RFHCAP; T.maxrf = H_RFHCAP / 2;
    T.maxbe = 4096; T.qhcap = H_QHCAP; T.maxq = H_QHCAP / 2; T.maxbf = 8192; T.maxcx = 8192; T.tier = 1;
    T.ehcap = 1;
    while (T.ehcap < 2 * (3 * T.maxbf + T.maxbe)) T.ehcap <<= 1;
    return T;
}
// global-slab tiles of the overflow path
constexpr int B_MAXRT = 16384, B_HCAP = 65536, B_RFHCAP = 8192, B_MAXRF = 4096, B_MAXBE = 4096,
              B_QHCAP = 8192, B_MAXQ = 4096, B_MAXBF = 32768;
// Largest scale of the global tiles.  Scales above 1 (4x per retry) are
// switched off: a 1M-point refinement faulted the GPU in the first round that
// used them and the cause is not yet shown; such a region is reported as
// QM_ECAPACITY instead.
constexpr int B_MAXSCALE = 1;
constexpr int MIS_BATCH = 4;       // selection passes launched per synchronisation
constexpr int SCAN_SMALL = 32768;  // up to this many candidates, one workgroup scans
constexpr int MIS_SMALL = 65536;   // up to this many claims and candidates, one workgroup selects
constexpr int MIS_SMALL_PASSES = 1 << 16;

struct Engine {
    hipStream_t s;
    Mesh M{};
    DBuf<double4> X;
    DBuf<int> TV, TA, TF, TS;
    DBuf<unsigned> TI;
    DBuf<int2> SV;
    DBuf<int> SSEG, STET, FAX;
    DBuf<unsigned> SFL;
    DBuf<unsigned long long> mark;
    DBuf<int> owner;
    // candidates
    DBuf<int> c_elem0, c_st0, c_reason0, order0, order1;
    DBuf<unsigned long long> c_key0, skey;
    DBuf<int4> c_tup0;
    DBuf<double4> c_p0;
    DBuf<int> c_elem, c_st, c_reason, c_seed, gst, greason, reg_off, reg_n, bf_off, bf_n, be_off, be_n,
        cl_off, cl_n, q_off, q_n, state, vk, vt, vs, sk, st_, ss_, kept, olist, glist, ulist0, ulist1;
    DBuf<unsigned char> mis_drop, mis_lose;   // selection: per-candidate pass flags (kept zero)
    DBuf<unsigned long long> c_key;
    DBuf<int4> c_tup;
    DBuf<double4> c_p;
    DBuf<int2> c_qw;
    // pools
    DBuf<int> p_cl, p_clc;
    DBuf<int4> p_be, p_bfr;
    DBuf<int2> p_q;
    DBuf<int> ctr;     // pool counters [0..5], candidates per class [8..10], totals [11..13],
                       // dead [14], stats [16..31], re-run list counts [32..34] and [36], tile code [35],
                       // passes of a one-workgroup selection [38],
                       // undecided per selection pass of a batch [40..40+MIS_BATCH)
    DBuf<char> tmp;    // sort and scan scratch
    DBuf<char> slab;   // overflow grow tiles
    DBuf<char> hslab;  // list tiles of the hybrid tier
    Cands C{};
    Pools PL{};
    BfPool BP{};
    unsigned pass = 1;
    int64_t dead = 0;
    // kernel-family timing with events on the call's stream (QM_PROFILE)
    bool prof = false;
    bool prof_grow = false;   // events around the small-tile and hybrid-tier grow launches only
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_cat, ev_round;
    int ev_used = 0, cur_round = 0;
    double prof_ms[QM_PROF_FAMILIES] = {0};
    int64_t prof_n[QM_PROF_FAMILIES] = {0};
    int64_t prof_over = 0, prof_full = 0;
    DBuf<unsigned long long> pctr;
    bool timed(int cat) const { return prof || (prof_grow && (cat == 3 || cat == 8)); }
    void pbegin(int cat = -1) {
        if (!timed(cat)) return;
        if (ev_used + 2 > (int)ev.size()) {
            for (int i = 0; i < 64; ++i) { hipEvent_t e; HIPCK(hipEventCreate(&e)); ev.push_back(e); }
            ev_cat.resize(ev.size());
            ev_round.resize(ev.size());
        }
        HIPCK(hipEventRecord(ev[ev_used], s));
    }
    void pend(int cat) {
        if (!timed(cat)) return;
        HIPCK(hipEventRecord(ev[ev_used + 1], s));
        ev_cat[ev_used] = cat;
        ev_round[ev_used] = cur_round;
        ev_used += 2;
        prof_n[cat]++;
    }
    // after a stream synchronisation: every recorded pair is complete
    void pflush(std::vector<double>* round_ms = nullptr) {
        for (int i = 0; i < ev_used; i += 2) {
            float ms = 0;
            HIPCK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            prof_ms[ev_cat[i]] += ms;
            if (round_ms) {
                size_t need = (size_t)(ev_round[i] + 1) * QM_PROF_FAMILIES;
                if (round_ms->size() < need) round_ms->resize(need, 0.0);
                (*round_ms)[(size_t)ev_round[i] * QM_PROF_FAMILIES + ev_cat[i]] += ms;
            }
        }
        ev_used = 0;
    }

    // no-alloc mode: every buffer is carved from `ar`; the mesh arrays are
    // sized once for the caller's output capacities
    Arena* ar = nullptr;
    size_t cap_v = 0, cap_t = 0, cap_s = 0;
    template <class F>
    void each_mesh_buf(F&& f) {
        f(X); f(TV); f(TA); f(TF); f(TS); f(TI); f(SV); f(SSEG); f(STET); f(FAX); f(SFL); f(mark); f(owner);
        f(ctr); f(pctr);
    }
    template <class F>
    void each_round_buf(F&& f) {
        for (auto* b : {&c_elem0, &c_st0, &c_reason0, &order0, &order1, &c_elem, &c_st, &c_reason, &c_seed,
                        &gst, &greason, &reg_off, &reg_n, &bf_off, &bf_n, &be_off, &be_n, &cl_off, &cl_n,
                        &q_off, &q_n, &state, &vk, &vt, &vs, &sk, &st_, &ss_, &kept, &olist, &glist, &ulist0, &ulist1, &p_cl,
                        &p_clc})
            f(*b);
        f(c_key0); f(skey); f(c_key); f(mis_drop); f(mis_lose); f(c_tup0); f(c_tup); f(c_p0); f(c_p); f(c_qw);
        f(p_be); f(p_bfr); f(p_q); f(tmp); f(slab); f(hslab);
    }
    void attach(Arena* a) {
        ar = a;
        each_mesh_buf([&](auto& b) { b.ar = a; });
        each_round_buf([&](auto& b) { b.ar = a; });
    }
    // no-alloc mode, start of a round (or of the output): the carvings of the
    // previous round are given back
    void arena_round() {
        if (!ar) return;
        ar->top = ar->mark;
        each_round_buf([&](auto& b) { b.p = nullptr; b.cap = 0; });
    }

    // device bytes of this call, and the budget the slab grids keep within
    // (0: none)
    Acct acct;
    size_t mem_cap = 0;
    explicit Engine(hipStream_t st) : s(st) {
        each_mesh_buf([&](auto& b) { b.acct = &acct; });
        each_round_buf([&](auto& b) { b.acct = &acct; });
        cblock.acct = &acct;
    }
    // Slab workgroups that fit the budget (at least one): the slab being
    // replaced (`held` bytes) is freed first, and the slabs together keep to
    // a quarter of the budget, leaving the rest to the mesh and the result
    // pools.
    int slab_grid(int grid, size_t block, size_t held) const {
        if (!mem_cap) return grid;
        const size_t others = acct.now - std::min(acct.now, held);
        const size_t slabs = slab.cap + hslab.cap - held;
        const size_t room = std::min(mem_cap > others ? mem_cap - others : 0,
                                     mem_cap / 4 > slabs ? mem_cap / 4 - slabs : 0);
        return (int)std::max<size_t>(1, std::min<size_t>((size_t)grid, room / block));
    }
    ~Engine() {
        DBuf<char>* bufs_c[] = {&tmp, &slab, &hslab, &cblock};
        for (auto* b : bufs_c) b->release(s);
        X.release(s); TV.release(s); TA.release(s); TF.release(s); TS.release(s); TI.release(s);
        SV.release(s); SSEG.release(s); STET.release(s); FAX.release(s); SFL.release(s);
        mark.release(s); owner.release(s);
        for (auto* b : {&c_elem0, &c_st0, &c_reason0, &order0, &order1, &c_elem, &c_st, &c_reason,
                        &c_seed, &gst, &greason, &reg_off, &reg_n, &bf_off, &bf_n, &be_off, &be_n, &cl_off,
                        &cl_n, &q_off, &q_n, &state, &vk, &vt, &vs, &sk, &st_, &ss_, &kept, &olist, &glist, &ulist0, &ulist1,
                        &p_cl, &p_clc, &ctr})
            b->release(s);
        c_key0.release(s); skey.release(s); c_key.release(s); mis_drop.release(s); mis_lose.release(s);
        c_tup0.release(s); c_tup.release(s); c_p0.release(s); c_p.release(s); c_qw.release(s);
        p_be.release(s); p_bfr.release(s); p_q.release(s); pctr.release(s);
        (void)hipStreamSynchronize(s);
        for (auto e : ev) (void)hipEventDestroy(e);
    }

    void bind() {
        M.X = X.p; M.TV = TV.p; M.TA = TA.p; M.TF = TF.p; M.TS = TS.p; M.TI = TI.p;
        M.SV = SV.p; M.SSEG = SSEG.p; M.SFL = SFL.p; M.STET = STET.p; M.FAX = FAX.p;
    }
    void ensure_mesh(int nv, int nt, int nss) {
        if (ar) {
            if ((size_t)nv > cap_v || (size_t)nt > cap_t || (size_t)std::max(nss, 1) > cap_s)
                throw QmError(QM_ECAPACITY, "the output arrays are too small for the refined mesh (vertices " +
                                                std::to_string(nv) + ", tet slots " + std::to_string(nt) +
                                                ", subsegments " + std::to_string(nss) + ")");
            nv = (int)cap_v; nt = (int)cap_t; nss = (int)cap_s;
        }
        X.ensure(nv, s, true);
        TV.ensure(4 * (size_t)nt, s, true);
        TA.ensure(4 * (size_t)nt, s, true);
        TF.ensure(4 * (size_t)nt, s, true, 0xFF);
        TS.ensure(6 * (size_t)nt, s, true, 0xFF);
        TI.ensure(nt, s, true, 0);
        mark.ensure(nt, s, true, 0);
        owner.ensure(nt, s, true, 0xFF);
        SV.ensure(std::max(nss, 1), s, true);
        SSEG.ensure(std::max(nss, 1), s, true);
        SFL.ensure(std::max(nss, 1), s, true, 0);
        STET.ensure(std::max(nss, 1), s, true);
        bind();
    }
    // Per-candidate arrays (contents not kept from round to round).  Without
    // an arena they are carved from one block, so a larger round costs one
    // allocation instead of one per array; the first-stage element list
    // c_elem0 (sized by the classification) stays a buffer of its own.
    DBuf<char> cblock;
    Arena cband;
    size_t cand_cap = 0;
    template <class F>
    void each_cand_buf(F&& f) {
        for (auto* b : {&c_st0, &c_reason0, &order0, &order1, &c_elem, &c_st, &c_reason, &c_seed,
                        &gst, &greason, &reg_off, &reg_n, &bf_off, &bf_n, &be_off, &be_n, &cl_off, &cl_n,
                        &q_off, &q_n, &state, &vk, &vt, &vs, &sk, &st_, &ss_, &kept, &olist, &glist, &ulist0, &ulist1})
            f(*b, 0);
        f(c_key0, 0); f(skey, 0); f(c_key, 0); f(mis_drop, 1); f(mis_lose, 1);
        f(c_tup0, 0); f(c_tup, 0); f(c_p0, 0); f(c_p, 0); f(c_qw, 0);
    }
    void ensure_cands(int n) {
        size_t m = std::max(n, 1);
        if (ar) {
            c_elem0.ensure(m, s, false);
            each_cand_buf([&](auto& b, int zero) { b.ensure(m, s, false, zero ? 0 : -1); });
        } else if (m > cand_cap) {
            const size_t cap = std::max(m, cand_cap + cand_cap / 2 + 1024);
            size_t bytes = 0;
            each_cand_buf([&](auto& b, int) { bytes += (cap * sizeof(*b.p) + 255) & ~(size_t)255; });
            each_cand_buf([&](auto& b, int) { b.p = nullptr; b.cap = 0; });
            cblock.release(s);
            cblock.ensure_exact(bytes, s);
            cband.base = cblock.p; cband.cap = bytes; cband.top = 0;
            each_cand_buf([&](auto& b, int zero) { b.ar = &cband; b.ensure(cap, s, false, zero ? 0 : -1); });
            cand_cap = cap;
        }
        C.n = n;
        C.elem = c_elem.p; C.key = c_key.p; C.tup = c_tup.p; C.p = c_p.p; C.st = c_st.p; C.reason = c_reason.p;
        C.seed = c_seed.p; C.qw = c_qw.p; C.gst = gst.p; C.greason = greason.p;
        C.reg_off = reg_off.p; C.reg_n = reg_n.p; C.bf_off = bf_off.p; C.bf_n = bf_n.p;
        C.be_off = be_off.p; C.be_n = be_n.p; C.cl_off = cl_off.p; C.cl_n = cl_n.p;
        C.q_off = q_off.p; C.q_n = q_n.p; C.state = state.p;
    }
    bool verbose = false;
    // pools: boundary-face records (bf entries), 2D boundary edges, claims
    // (each candidate's range starts with its region tets), queue entries
    void ensure_pools(size_t bf, size_t be, size_t cl, size_t q) {
        // pool offsets and counters are int32: refuse sizes they cannot index
        const size_t lim = (size_t)1 << 30;
        if (bf > lim || be > lim || cl > lim || q > lim)
            throw QmError(QM_ENOMEM, "a round's result pools exceed 2^30 entries");
        const size_t before = p_bfr.cap + p_be.cap + p_cl.cap + p_q.cap;
        p_bfr.ensure(BFR * bf, s, false);
        p_be.ensure(be, s, false); p_cl.ensure(cl, s, false); p_q.ensure(q, s, false);
        p_clc.ensure(cl, s, false);
        PL.be = p_be.p; PL.cl = p_cl.p; PL.clc = p_clc.p; PL.q = p_q.p;
        PL.cap_be = (int)p_be.cap; PL.cap_cl = (int)p_cl.cap; PL.cap_q = (int)p_q.cap; PL.ctr = ctr.p;
        BP.r = p_bfr.p; BP.cap = (int)(p_bfr.cap / BFR); BP.prof = prof ? pctr.p : nullptr;
        BP.tprof = prof ? pctr.p + 4 + GROW_PHASES : nullptr;
        if (verbose && p_bfr.cap + p_be.cap + p_cl.cap + p_q.cap != before)
            fprintf(stderr, "qm: pools grown: faces %zu (%.2f GB of records), edges %zu, claims %zu, queue %zu "
                    "entries\n", p_bfr.cap / BFR, p_bfr.cap * sizeof(int4) / 1e9, p_be.cap, p_cl.cap, p_q.cap);
    }
    // pool entries per candidate seen in the last round (region tets,
    // boundary faces, 2D boundary edges, claims, queue entries); the next
    // round reserves 1.5x that plus slack
    // pool entries per candidate (region tets, boundary faces, 2D boundary
    // edges, claims, queue entries) used by the last round of each class
    // (counters include ranges of re-run candidates); the next round of the
    // class reserves 1.25x that plus slack
    double pool_rate[3][5] = {{0, 48, 8, 56, 4}, {0, 48, 8, 56, 4}, {0, 48, 8, 56, 4}};
    size_t pool_need(int k, int ncand, int cls) const {
        return (size_t)(pool_rate[cls][k] * 1.25 * ncand) + 4096;
    }
    void pool_seen(const int* used, int ncand, int cls) {
        if (ncand <= 0) return;
        for (int k = 0; k < 5; ++k) pool_rate[cls][k] = (double)used[k] / ncand;
    }
    BfPool BPnoprof() const {   // region counters cover the first small-tile launch only
        BfPool b = BP;
        b.prof = nullptr;
        return b;
    }
    // Renumber the live tets in Morton order of their centroids (dead slots
    // dropped); the selection words are cleared, which every round expects
    // between rounds anyway.  Not used without allocation.
    int nt_ordered = 0;
    void reorder() {
        const int nt = M.nt;
        DBuf<unsigned long long> k0, k1;
        DBuf<int> v0, v1, perm;
        for (auto* b : {&v0, &v1, &perm}) b->acct = &acct;
        k0.acct = k1.acct = &acct;
        k0.ensure(nt, s, false); k1.ensure(nt, s, false); v0.ensure(nt, s, false); v1.ensure(nt, s, false);
        perm.ensure(nt, s, false);
        int* nlive_d = ctr.p + 50;
        HIPCK(hipMemsetAsync(nlive_d, 0, sizeof(int), s));
        k_order_keys<<<nblk(nt), 256, 0, s>>>(M, k0.p, v0.p, nlive_d);
        sort_asc(k0.p, k1.p, v0.p, v1.p, nt);
        k_order_perm<<<nblk(nt), 256, 0, s>>>(nt, v1.p, perm.p);
        const int nlive = read1(nlive_d, s);
        DBuf<int> nTV, nTA, nTF, nTS;
        DBuf<unsigned> nTI;
        for (auto* b : {&nTV, &nTA, &nTF, &nTS}) b->acct = &acct;
        nTI.acct = &acct;
        nTV.ensure(TV.cap, s, false); nTA.ensure(TA.cap, s, false); nTF.ensure(TF.cap, s, false);
        nTS.ensure(TS.cap, s, false); nTI.ensure(TI.cap, s, false);
        k_order_gather<<<nblk(nlive), 256, 0, s>>>(nlive, v1.p, perm.p, M, nTV.p, nTA.p, nTF.p, nTS.p, nTI.p);
        if (M.nss) k_order_stet<<<nblk(M.nss), 256, 0, s>>>(M.nss, perm.p, STET.p);
        auto swap_in = [](auto& a, auto& b) { std::swap(a.p, b.p); std::swap(a.cap, b.cap); };
        swap_in(TV, nTV); swap_in(TA, nTA); swap_in(TF, nTF); swap_in(TS, nTS); swap_in(TI, nTI);
        nTV.release(s); nTA.release(s); nTF.release(s); nTS.release(s); nTI.release(s);
        k0.release(s); k1.release(s); v0.release(s); v1.release(s); perm.release(s);
        HIPCK(hipMemsetAsync(mark.p, 0, mark.cap * sizeof(unsigned long long), s));
        HIPCK(hipMemsetAsync(owner.p, 0xFF, owner.cap * sizeof(int), s));
        HIPCK(hipMemsetAsync(ctr.p + 14, 0, sizeof(int), s));   // no dead slots left
        M.nt = nlive;
        dead = 0;
        nt_ordered = nlive;
        bind();
    }
    void* cub_tmp(size_t bytes) {
        tmp.ensure(bytes, s, false);
        return tmp.p;
    }
    // key-value radix sorts (rocPRIM; stable, so equal keys keep index order)
    template <class K, class V>
    void sort_desc(const K* kin, K* kout, const V* vin, V* vout, int n) {
        size_t bytes = 0;
        HIPCK(rocprim::radix_sort_pairs_desc(nullptr, bytes, kin, kout, vin, vout, (size_t)n, 0,
                                             (unsigned)(8 * sizeof(K)), s));
        void* t = cub_tmp(bytes);
        HIPCK(rocprim::radix_sort_pairs_desc(t, bytes, kin, kout, vin, vout, (size_t)n, 0,
                                             (unsigned)(8 * sizeof(K)), s));
    }
    template <class K, class V>
    void sort_asc(const K* kin, K* kout, const V* vin, V* vout, int n) {
        size_t bytes = 0;
        HIPCK(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)n, 0,
                                        (unsigned)(8 * sizeof(K)), s));
        void* t = cub_tmp(bytes);
        HIPCK(rocprim::radix_sort_pairs(t, bytes, kin, kout, vin, vout, (size_t)n, 0, (unsigned)(8 * sizeof(K)), s));
    }
    // exclusive prefix sum of n ints: tile sums, one workgroup scans them,
    // then each tile is scanned from its offset (one pass when n fits a tile)
    void exscan(const int* in, int* out, int n) {
        if (n <= 0) return;
        const int tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
        if (tiles == 1) {
            k_scan_tile<<<1, 256, 0, s>>>(n, in, out, nullptr);
            return;
        }
        int* sums = (int*)cub_tmp(sizeof(int) * (size_t)tiles);
        k_scan_tile_sums<<<tiles, 256, 0, s>>>(n, in, sums);
        k_scan_sums<<<1, 1024, 0, s>>>(tiles, sums);
        k_scan_tile<<<tiles, 256, 0, s>>>(n, in, out, sums);
    }
};

}  // namespace qm

using namespace qm;

// Device setup of one refinement, whose input is a CDT of the PLC (paper,
// Section 2): inputs staged (or used in place when they are device arrays),
// adjacency by face matching, subfaces and subsegments marked, facet
// projection axes, the h_min bound.  Input errors become QmError.  `e0`
// (optional) is recorded when the setup kernels start.
static void setup_mesh(Engine& E, const qm_plc* plc, const qm_mesh* in, const qm_options* opt, Arena* ar,
                       hipEvent_t e0, const qm_state* st = nullptr) {
    const hipStream_t s = E.s;
    const bool noalloc = ar != nullptr;
    const bool dev = (opt->flags & QM_INPUT_DEVICE) != 0;
    const int nv = in->nv, nt = in->nt, nsf = in->nsf, nss = in->nss, nftri = plc->nftri;
    int nfacet = 0;
    // staging of the input arrays on the device
    auto stage = [&](const void* p, size_t bytes, DBuf<char>& buf) -> const void* {
        if (dev || bytes == 0) return p;
        buf.ensure(bytes, s, false);
        HIPCK(hipMemcpyAsync(buf.p, p, bytes, hipMemcpyHostToDevice, s));
        return buf.p;
    };
    // staged copies (unused with device inputs), freed on the stream when setup ends
    struct Staged {
        DBuf<char> b[11];
        hipStream_t s;
        ~Staged() { for (auto& x : b) x.release(s); }
    } stg;
    stg.s = s;
    for (auto& b : stg.b) b.acct = &E.acct;
    DBuf<char>&b_xyz = stg.b[0], &b_tet = stg.b[1], &b_sf = stg.b[2], &b_sff = stg.b[3], &b_ss = stg.b[4],
             &b_ssg = stg.b[5], &b_ft = stg.b[6], &b_ftf = stg.b[7];
    const double* d_xyz = (const double*)stage(in->xyz, sizeof(double) * 3 * nv, b_xyz);
    const int* d_tet = (const int*)stage(in->tet, sizeof(int) * 4 * (size_t)nt, b_tet);
    const int* d_sf = (const int*)stage(in->sf, sizeof(int) * 3 * (size_t)nsf, b_sf);
    const int* d_sff = (const int*)stage(in->sf_facet, sizeof(int) * (size_t)nsf, b_sff);
    const int* d_ss = (const int*)stage(in->ss, sizeof(int) * 2 * (size_t)nss, b_ss);
    const int* d_ssg = (const int*)stage(in->ss_seg, sizeof(int) * (size_t)nss, b_ssg);
    const int* d_ft = (const int*)stage(plc->ftri, sizeof(int) * 3 * (size_t)nftri, b_ft);
    const int* d_ftf = (const int*)stage(plc->ftri_facet, sizeof(int) * (size_t)nftri, b_ftf);
    // a resumed refinement's flags (host arrays whatever the mesh's kind)
    auto stage_h = [&](const uint8_t* p, size_t bytes, DBuf<char>& buf) -> const unsigned char* {
        if (!st || bytes == 0) return nullptr;
        buf.ensure(bytes, s, false);
        HIPCK(hipMemcpyAsync(buf.p, p, bytes, hipMemcpyHostToDevice, s));
        return (const unsigned char*)buf.p;
    };
    const unsigned char* d_tfl = stage_h(st ? st->tet_flags : nullptr, (size_t)nt, stg.b[8]);
    const unsigned char* d_sfl = stage_h(st ? st->sf_flags : nullptr, (size_t)nsf, stg.b[9]);
    const unsigned char* d_ssl = stage_h(st ? st->ss_flags : nullptr, (size_t)nss, stg.b[10]);
    E.ctr.ensure(64, s, false, 0);
    // number of facets = 1 + max facet id over PLC triangles and subfaces
    if (nftri) k_count_ids<<<nblk(nftri), 256, 0, s>>>(nftri, d_ftf, E.ctr.p + 49);
    if (nsf) k_count_ids<<<nblk(nsf), 256, 0, s>>>(nsf, d_sff, E.ctr.p + 49);
    nfacet = read1(E.ctr.p + 49, s);
    E.ensure_mesh(nv, nt, std::max(nss, 1));
    E.FAX.ensure(std::max(nfacet, 1), s, false);
    E.bind();
    if (noalloc) ar->mark = ar->top;      // what follows is carved again every round
    E.M.nv = nv; E.M.nt = nt; E.M.nss = nss;
    E.M.err = E.ctr.p + 48;               // this call's error word of the exact paths
    E.nt_ordered = nt;
    if (opt->flags & QM_TEST_ERROR_WORD) HIPCK(hipMemsetAsync(E.M.err, 1, 1, s));
    int* err = E.ctr.p + 13;
    if (e0) HIPCK(hipEventRecord(e0, s));
    // ---- device setup
    k_setup_verts<<<nblk(nv), 256, 0, s>>>(nv, d_xyz, E.X.p, err);
    k_setup_tets<<<nblk(nt), 256, 0, s>>>(nt, nv, d_tet, d_tfl, E.M, err);
    {
        DBuf<unsigned long long> k0, k1;
        DBuf<int> v0, v1;
        k0.ar = k1.ar = ar; v0.ar = v1.ar = ar;
        k0.acct = k1.acct = &E.acct; v0.acct = v1.acct = &E.acct;
        size_t n4 = 4 * (size_t)nt, n6 = 6 * (size_t)nt;
        k0.ensure(n6, s, false); k1.ensure(n6, s, false); v0.ensure(n6, s, false); v1.ensure(n6, s, false);
        k_face_keys<<<nblk(n4), 256, 0, s>>>(nt, E.TV.p, k0.p, v0.p);
        E.sort_asc(k0.p, k1.p, v0.p, v1.p, (int)n4);
        k_face_match<<<nblk(n4), 256, 0, s>>>((int)n4, k1.p, v1.p, E.TA.p, err);
        if (nsf) k_mark_subfaces<<<nblk(nsf), 256, 0, s>>>(nsf, nv, nfacet, d_sf, d_sff, d_sfl, k1.p, v1.p, (int)n4,
                                                            E.TF.p, E.TI.p, err);
        k_edge_keys<<<nblk(n6), 256, 0, s>>>(nt, E.TV.p, k0.p, v0.p);
        E.sort_asc(k0.p, k1.p, v0.p, v1.p, (int)n6);
        if (nss) k_mark_subsegs<<<nblk(nss), 256, 0, s>>>(nss, nv, d_ss, d_ssg, d_ssl, k1.p, v1.p, (int)n6, E.M,
                                                           err);
        DBuf<int> first;
        first.ar = ar;
        first.acct = &E.acct;
        first.ensure(std::max(nfacet, 1), s, false);
        k_fill<<<nblk(nfacet), 256, 0, s>>>(nfacet, first.p, 0x7fffffff);   // "no triangle yet"
        if (nftri) k_facet_first<<<nblk(nftri), 256, 0, s>>>(nftri, d_ftf, nfacet, first.p, err);
        k_facet_axis<<<nblk(nfacet), 256, 0, s>>>(nfacet, first.p, d_ft, E.X.p, nv, E.FAX.p, err);
        unsigned long long* dmin = (unsigned long long*)(E.ctr.p + 40);
        HIPCK(hipMemsetAsync(dmin, 0x7F, sizeof(unsigned long long), s));
        k_min_edge<<<nblk(nt), 256, 0, s>>>(nt, E.M, dmin);
        HIPCK(hipStreamSynchronize(s));
        k0.release(s); k1.release(s); v0.release(s); v1.release(s); first.release(s);
        int e = read1(err, s);
        if (e & 1) throw QmError(QM_EINVAL, "ids out of range or coordinates off the 2^-53 lattice / outside [0,1]");
        if (e & 2) throw QmError(QM_ENONCONFORM, "a tet is not positively oriented");
        if (e & 4) throw QmError(QM_ENONCONFORM, "a face is shared by more than two tets");
        if (e & 8) throw QmError(QM_ENONCONFORM, "a subface is not a face of the mesh");
        if (e & 16) throw QmError(QM_ENONCONFORM, "a subsegment is not an edge of the mesh");
        unsigned long long bits = read1(dmin, s);
        double l2;
        std::memcpy(&l2, &bits, sizeof l2);
        E.M.hmin2 = st ? st->hmin2 : (opt->hmin_factor * opt->hmin_factor) * l2;   // fixed by the first call
        E.M.B2 = opt->B * opt->B;
    }
}

// Verdicts of the last round's candidates (9 values per candidate): the
// candidate arrays are only rewritten by a round that has candidates, so
// they still hold that round.
static void read_last_round(Engine& E, qm_result* R, int ncand) {
    const hipStream_t s = E.s;
    std::vector<int4> tup(ncand);
    std::vector<int> st0(ncand), gs(ncand), rs0(ncand), grs(ncand), stt(ncand), rn(ncand), bn(ncand);
    HIPCK(hipMemcpyAsync(tup.data(), E.c_tup.p, sizeof(int4) * ncand, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(st0.data(), E.c_st.p, sizeof(int) * ncand, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(gs.data(), E.gst.p, sizeof(int) * ncand, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(rs0.data(), E.c_reason.p, sizeof(int) * ncand, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(grs.data(), E.greason.p, sizeof(int) * ncand, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(stt.data(), E.state.p, sizeof(int) * ncand, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(rn.data(), E.reg_n.p, sizeof(int) * ncand, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(bn.data(), E.bf_n.p, sizeof(int) * ncand, hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    R->last.assign(9 * (size_t)ncand, 0);
    for (int i = 0; i < ncand; ++i) {
        int* o = R->last.data() + 9 * (size_t)i;
        int fs = st0[i] != ST_PENDING ? st0[i] : gs[i];
        o[0] = tup[i].x; o[1] = tup[i].y; o[2] = tup[i].z; o[3] = tup[i].w;
        o[4] = fs; o[5] = fs == ST_EXEMPT ? (st0[i] != ST_PENDING ? rs0[i] : grs[i]) : 0;
        o[6] = stt[i] == 1; o[7] = fs == ST_OK ? rn[i] : 0; o[8] = fs == ST_OK ? bn[i] : 0;
    }
}

// Output of one refinement: live tets and subfaces compacted in slot order,
// then written to the caller's device arrays (no-alloc form), to device
// arrays the result owns (QM_OUTPUT_DEVICE) or downloaded into the result.
// Returns the number of output tets.
static int emit_output(Engine& E, qm_result* R, const qm_options* opt, Arena* ar, qm_mesh_buf* dout) {
    const hipStream_t s = E.s;
    const bool noalloc = ar != nullptr;
    E.arena_round();
    int ntot = E.M.nt;
    DBuf<int> tf, ts, ff, fs;
    tf.ar = ts.ar = ff.ar = fs.ar = ar;
    tf.acct = ts.acct = ff.acct = fs.acct = &E.acct;
    tf.ensure(ntot, s, false); ts.ensure(ntot, s, false);
    ff.ensure(4 * (size_t)ntot, s, false); fs.ensure(4 * (size_t)ntot, s, false);
    k_out_flags<<<nblk(ntot), 256, 0, s>>>(E.M, tf.p, ff.p);
    E.exscan(tf.p, ts.p, ntot);
    E.exscan(ff.p, fs.p, 4 * ntot);
    int a = read1(ts.p + ntot - 1, s) + read1(tf.p + ntot - 1, s);
    int b = read1(fs.p + 4 * ntot - 1, s) + read1(ff.p + 4 * ntot - 1, s);
    if (!noalloc) {            // the refinement state, aligned with the output mesh (host arrays)
        const int nss = E.M.nss;
        const size_t nb = (size_t)a + (size_t)b + (size_t)nss;
        DBuf<char> ob;
        ob.acct = &E.acct;
        ob.ensure(std::max<size_t>(nb, 1), s, false);
        unsigned char* o = (unsigned char*)ob.p;
        k_out_state<<<nblk(std::max(ntot, nss)), 256, 0, s>>>(E.M, tf.p, ts.p, ff.p, fs.p, o, o + a, o + a + b);
        std::vector<uint8_t> h(nb);
        if (nb) HIPCK(hipMemcpyAsync(h.data(), o, nb, hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        ob.release(s);
        R->st_tfl.assign(h.begin(), h.begin() + a);
        R->st_sfl.assign(h.begin() + a, h.begin() + a + b);
        R->st_ssl.assign(h.begin() + a + b, h.end());
        R->st_hmin2 = E.M.hmin2;
    }
    if (noalloc) {
        dout->nv = E.M.nv; dout->nt = a; dout->nsf = b; dout->nss = E.M.nss;
        if (E.M.nv > dout->cap_v || a > dout->cap_t || b > dout->cap_sf || E.M.nss > dout->cap_ss)
            throw QmError(QM_ECAPACITY, "the output arrays are too small (vertices " + std::to_string(E.M.nv) +
                                            ", tets " + std::to_string(a) + ", subfaces " + std::to_string(b) +
                                            ", subsegments " + std::to_string(E.M.nss) + ")");
        k_out_tets<<<nblk(ntot), 256, 0, s>>>(E.M, tf.p, ts.p, dout->tet);
        if (b) k_out_sf<<<nblk(4L * ntot), 256, 0, s>>>(E.M, ff.p, fs.p, dout->sf, dout->sf_facet);
        k_out_xyz<<<nblk(E.M.nv), 256, 0, s>>>(E.M.nv, E.X.p, dout->xyz);
        if (E.M.nss) {
            HIPCK(hipMemcpyAsync(dout->ss, E.SV.p, sizeof(int) * 2 * (size_t)E.M.nss, hipMemcpyDeviceToDevice, s));
            HIPCK(hipMemcpyAsync(dout->ss_seg, E.SSEG.p, sizeof(int) * (size_t)E.M.nss, hipMemcpyDeviceToDevice, s));
        }
        HIPCK(hipStreamSynchronize(s));
    } else if (opt->flags & QM_OUTPUT_DEVICE) {   // the result stays on the device
        HIPCK(hipStreamSynchronize(s));
        auto dalloc = [&](auto** p, size_t n) {
            HIPCK(hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(**p)));
        };
        dalloc(&R->d_xyz, 3 * (size_t)E.M.nv); dalloc(&R->d_tets, 4 * (size_t)a);
        dalloc(&R->d_sf, 3 * (size_t)b); dalloc(&R->d_sff, (size_t)b);
        dalloc(&R->d_ss, 2 * (size_t)E.M.nss); dalloc(&R->d_ssg, (size_t)E.M.nss);
        k_out_tets<<<nblk(ntot), 256, 0, s>>>(E.M, tf.p, ts.p, R->d_tets);
        if (b) k_out_sf<<<nblk(4L * ntot), 256, 0, s>>>(E.M, ff.p, fs.p, R->d_sf, R->d_sff);
        k_out_xyz<<<nblk(E.M.nv), 256, 0, s>>>(E.M.nv, E.X.p, R->d_xyz);
        if (E.M.nss) {
            HIPCK(hipMemcpyAsync(R->d_ss, E.SV.p, sizeof(int) * 2 * (size_t)E.M.nss, hipMemcpyDeviceToDevice, s));
            HIPCK(hipMemcpyAsync(R->d_ssg, E.SSEG.p, sizeof(int) * (size_t)E.M.nss, hipMemcpyDeviceToDevice, s));
        }
        HIPCK(hipStreamSynchronize(s));
        R->on_device = true;
        R->dnv = E.M.nv; R->dnt = a; R->dnsf = b; R->dnss = E.M.nss;
    } else {
        DBuf<int> ot, osf, osff;
        DBuf<double> ox;
        ot.acct = osf.acct = osff.acct = &E.acct;
        ox.acct = &E.acct;
        ot.ensure(4 * (size_t)std::max(a, 1), s, false);
        osf.ensure(3 * (size_t)std::max(b, 1), s, false);
        osff.ensure(std::max(b, 1), s, false);
        ox.ensure(3 * (size_t)E.M.nv, s, false);
        k_out_tets<<<nblk(ntot), 256, 0, s>>>(E.M, tf.p, ts.p, ot.p);
        k_out_sf<<<nblk(4L * ntot), 256, 0, s>>>(E.M, ff.p, fs.p, osf.p, osff.p);
        k_out_xyz<<<nblk(E.M.nv), 256, 0, s>>>(E.M.nv, E.X.p, ox.p);
        R->xyz.resize(3 * (size_t)E.M.nv);
        R->tets.resize(4 * (size_t)a);
        R->sf.resize(3 * (size_t)b);
        R->sff.resize(b);
        R->ss.resize(2 * (size_t)E.M.nss);
        R->ssg.resize(E.M.nss);
        HIPCK(hipMemcpyAsync(R->xyz.data(), ox.p, sizeof(double) * R->xyz.size(), hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(R->tets.data(), ot.p, sizeof(int) * R->tets.size(), hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(R->sf.data(), osf.p, sizeof(int) * R->sf.size(), hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(R->sff.data(), osff.p, sizeof(int) * R->sff.size(), hipMemcpyDeviceToHost, s));
        if (E.M.nss) {
            HIPCK(hipMemcpyAsync(R->ss.data(), E.SV.p, sizeof(int) * R->ss.size(), hipMemcpyDeviceToHost, s));
            HIPCK(hipMemcpyAsync(R->ssg.data(), E.SSEG.p, sizeof(int) * R->ssg.size(), hipMemcpyDeviceToHost, s));
        }
        HIPCK(hipStreamSynchronize(s));
        ot.release(s); osf.release(s); osff.release(s); ox.release(s);
    }
    tf.release(s); ts.release(s); ff.release(s); fs.release(s);
    return a;
}

// One refinement.  Normal form: buffers from the stream-ordered allocator,
// result in *out (host arrays).  No-alloc form (ar != nullptr): every device
// buffer is carved from the arena, inputs are device arrays, the output mesh
// is written into the caller's device arrays `dout` and the statistics into
// *dstats; no qm_result, pinned buffer or event is created.
// A resumed refinement's state must describe its mesh (host check, before
// any device call).
static void check_state(const qm_mesh* in, const qm_state* rs) {
    if (rs->nt != in->nt || rs->nsf != in->nsf || rs->nss != in->nss)
        throw QmError(QM_EINVAL, "the state's counts differ from the mesh's");
    if ((in->nt && !rs->tet_flags) || (in->nsf && !rs->sf_flags) || (in->nss && !rs->ss_flags))
        throw QmError(QM_EINVAL, "state flag array missing");
    if (rs->next_class < 0 || rs->next_class > 2 || rs->rounds < 0 || !(rs->hmin2 >= 0.0) || !std::isfinite(rs->hmin2))
        throw QmError(QM_EINVAL, "state: next_class outside 0..2, negative rounds or bad hmin2");
    for (int i = 0; i < in->nt; ++i)
        if (rs->tet_flags[i] > 1) throw QmError(QM_EINVAL, "state: tet flag with bits other than bit0");
    for (int i = 0; i < in->nsf; ++i)
        if (rs->sf_flags[i] > 3) throw QmError(QM_EINVAL, "state: subface flag with bits other than 0-1");
    for (int i = 0; i < in->nss; ++i)
        if (rs->ss_flags[i] > 3) throw QmError(QM_EINVAL, "state: subsegment flag with bits other than 0-1");
}

// `stop` (served jobs, else null): when it is set, the refinement ends at the
// next round boundary with status 2 and its output and state on the host, a
// checkpoint to resume from.
static int run_refine(const qm_plc* plc, const qm_mesh* in, const qm_options* opt, hipStream_t s,
                      qm_result** out, Arena* ar = nullptr, qm_mesh_buf* dout = nullptr,
                      qm_stats* dstats = nullptr, size_t mem_cap = 0, const qm_state* rs = nullptr,
                      const std::atomic<bool>* stop = nullptr) {
    auto T0 = std::chrono::steady_clock::now();
    const bool noalloc = ar != nullptr;
    if (!plc || !in || !opt || (noalloc ? (!dout || !dstats) : !out)) throw QmError(QM_EINVAL, "null argument");
    if (!(opt->B > 0.0) || !(opt->hmin_factor >= 0.0) || opt->max_rounds < 0)
        throw QmError(QM_EINVAL, "B must be > 0, hmin_factor >= 0, max_rounds >= 0");
    if (in->nv < 8 || in->nt < 1 || in->nsf < 0 || in->nss < 0 || plc->nftri < 0 || plc->nseg < 0)
        throw QmError(QM_EINVAL, "bad counts");
    if (in->nv >= (1 << 21)) throw QmError(QM_EINVAL, "input vertex count must be below 2^21");
    if (rs) check_state(in, rs);
    const bool dev = (opt->flags & QM_INPUT_DEVICE) != 0;
    if (noalloc) {
        if (!dev) throw QmError(QM_EINVAL, "the no-alloc entry point takes device arrays (QM_INPUT_DEVICE)");
        if (opt->flags & (QM_PROFILE | QM_PROFILE_GROW))
            throw QmError(QM_EINVAL, "profiling flags are not available without allocation");
        if (dout->cap_v < in->nv || dout->cap_t < in->nt || dout->cap_ss < in->nss || dout->cap_sf < 0 ||
            !dout->xyz || !dout->tet || (dout->cap_sf > 0 && (!dout->sf || !dout->sf_facet)) ||
            (dout->cap_ss > 0 && (!dout->ss || !dout->ss_seg)))
            throw QmError(QM_EINVAL, "output arrays missing or smaller than the input mesh");
    }
    Engine E(s);
    E.mem_cap = mem_cap;
    if (noalloc) {
        E.attach(ar);
        E.cap_v = (size_t)dout->cap_v;
        E.cap_t = (size_t)dout->cap_t + (size_t)dout->cap_t / 8 + 256;   // slots of removed tets included
        E.cap_s = (size_t)std::max(dout->cap_ss, 1);
    }
    E.prof = (opt->flags & QM_PROFILE) != 0;
    E.prof_grow = !E.prof && (opt->flags & QM_PROFILE_GROW) != 0;
    if (E.prof) { E.pctr.ensure(4 + GROW_PHASES + 3 * TPROF_W, s, false, 0); }
    int64_t scan_tets = 0, scan_verts = 0;
    auto T1 = std::chrono::steady_clock::now();
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (!noalloc) {
        HIPCK(hipEventCreate(&e0)); HIPCK(hipEventCreate(&e1)); HIPCK(hipEventCreate(&e2));
    }
    setup_mesh(E, plc, in, opt, ar, e0, rs);

    auto T1s = std::chrono::steady_clock::now();
    if (!noalloc) HIPCK(hipEventRecord(e1, s));
    // ---- rounds
    std::unique_ptr<qm_result> R(noalloc ? nullptr : new qm_result());
    qm_stats ST;
    std::memset(&ST, 0, sizeof ST);
    int* cnt_d = E.ctr.p + 8;
    int* tot_d = E.ctr.p + 11;
    int* dead_d = E.ctr.p + 14;
    int* stats_d = E.ctr.p + 16;
    int* olist_n = E.ctr.p + 32;
    int* undec_d = E.ctr.p + 40;
    int* npass_d = E.ctr.p + 38;
    int* nu_d = E.ctr.p + 46;      // undecided-list lengths of the selection passes (two buffers)
    int round = 0, status = 0, last_ncand = 0;
    // host copies of the counters live in pinned memory: the per-round
    // read-backs are then direct copies, not staged through a bounce buffer
    std::unique_ptr<PinnedInts> pin(noalloc ? nullptr : new PinnedInts(48 + 46));
    int hloc[48 + 46];              // no-alloc form: pageable copies instead
    int* const hbase = noalloc ? hloc : pin->p;
    int* const hc = hbase;          // ctr[0..48), taken at each synchronisation
    auto sync_counters = [&]() {
        HIPCK(hipMemcpyAsync(hc, E.ctr.p, 48 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        if (E.prof) E.pflush(&R->round_ms);
        else if (E.prof_grow) E.pflush();
    };
    // the dead-slot count after a round's insertion is read at the next
    // synchronisation; it completes that round's record (tets after)
    auto patch_last_record = [&]() {
        if (!R || R->rounds.empty()) return;
        E.dead = hc[14];
        R->rounds[R->rounds.size() - QM_ROUND_FIELDS + 16] = E.M.nt - (int)E.dead;
    };
    // global-memory tiles: scale 1 first; a region over them (cavities can
    // grow with the number of vertices a point sees, e.g. next to a dense
    // cluster) makes the round retry those candidates at 4x the scale
    int tile_scale = 1;
    auto big_tiles = [&](int k) {
        GrowTiles T{};
        T.maxrt = B_MAXRT * k; T.hcap = B_HCAP * k; T.rfhcap = B_RFHCAP * k; T.maxrf = B_MAXRF * k;
        T.maxbe = B_MAXBE * k; T.qhcap = B_QHCAP * k; T.maxq = B_MAXQ * k; T.maxbf = B_MAXBF * k;
        T.maxcx = B_MAXBF * k; T.tier = 2;
        T.ehcap = 1;
        while (T.ehcap < 2 * (3 * T.maxbf + T.maxbe)) T.ehcap <<= 1;
        return T;
    };
    const bool verbose = (opt->flags & QM_VERBOSE) != 0;
    const int min_tier = (opt->flags & QM_TEST_TIER2) ? 2 : (opt->flags & QM_TEST_TIER1) ? 1 : 0;
    const bool early_stop = (opt->flags & QM_EARLY_STOP) != 0;
    // three-sub-phase rounds: the class is forced in turn (SS, SF, TET); a
    // sub-phase without candidates is skipped and is not a round
    const bool subphases = (opt->flags & QM_SUBPHASE_ROUNDS) != 0;
    int sub = rs ? rs->next_class : CLS_SS, empty_subphases = 0;
    const unsigned long long key_mask = (opt->flags & QM_TEST_KEY_COLLIDE) ? 0xE000000000000000ull : ~0ull;
    E.verbose = verbose;
    auto last_note = std::chrono::steady_clock::now();
    // progress inside a long round (verbose): at most one line per 10 s
    auto note = [&](const char* phase, int round_, int cls_, int n_) {
        if (!verbose || std::chrono::steady_clock::now() - last_note < std::chrono::seconds(10)) return;
        last_note = std::chrono::steady_clock::now();
        fprintf(stderr, "qm: round %d class %d %s (%d)\n", round_, cls_, phase, n_);
    };
    for (;; ++round) {
        if (round >= opt->max_rounds) { status = 1; break; }
        if (stop && stop->load(std::memory_order_relaxed)) { status = 2; break; }
        E.cur_round = round;
        E.arena_round();
        // slots appended since the last renumbering are in priority order,
        // scattered in space: renumber once they are a tenth of the mesh
        if (!noalloc && E.M.nt - E.nt_ordered > std::max(E.M.nt / 10, 65536)) {
            E.reorder();
            if (verbose) fprintf(stderr, "qm: round %d: tets renumbered in Morton order (%d live)\n", round, E.M.nt);
        }
        // step 1: classify, in the paper's order (a class is skipped on the
        // device when an earlier one has candidates); one synchronisation
        // candidates go straight to the first candidate array, sized for the
        // largest class (so the later sizing never moves it)
        E.c_elem0.ensure(std::max((size_t)E.M.nss, 4 * (size_t)E.M.nt), s, false);
        k_round_reset<<<1, 64, 0, s>>>(E.ctr.p);
        E.pbegin();
        // (a sub-phase classifies its class alone: the earlier classes' counts
        // stay zero, so its kernel does not skip)
        if (E.M.nss && (!subphases || sub == CLS_SS))
            k_classify_ss<<<nblk(E.M.nss), 256, 0, s>>>(E.M, E.c_elem0.p, cnt_d);
        if (!subphases || sub == CLS_SF) k_classify_sf<<<nblk(E.M.nt), 256, 0, s>>>(E.M, E.c_elem0.p, cnt_d);
        if (!subphases || sub == CLS_TET) k_classify_tet<<<nblk(E.M.nt), 256, 0, s>>>(E.M, E.c_elem0.p, cnt_d);
        E.pend(0);
        sync_counters();
        patch_last_record();
        int cls = CLS_NONE, ncand = 0;
        for (int c = CLS_SS; c <= CLS_TET && cls == CLS_NONE; ++c)
            if (hc[8 + c] > 0) { cls = c; ncand = hc[8 + c]; }
        if (hc[8 + CLS_SS] == 0 && hc[8 + CLS_SF] == 0) { scan_tets += E.M.nt; scan_verts += E.M.nv; }
        if (subphases) {
            if (cls == CLS_NONE) {
                if (++empty_subphases == 3) break;      // a whole round without work
                sub = (sub + 1) % 3;
                --round;
                continue;
            }
            empty_subphases = 0;
            sub = (sub + 1) % 3;
        }
        if (cls == CLS_NONE) break;
        E.ensure_cands(ncand);
        // step 2: splitting points and priorities, then priority order
        E.pbegin();
        k_split<<<nblk(ncand), 256, 0, s>>>(E.M, cls, ncand, E.c_elem0.p, E.c_key0.p, E.c_tup0.p, E.c_p0.p,
                                          E.c_st0.p, E.c_reason0.p, key_mask);
        if (ncand <= SORT_SMALL) {
            k_order_small<<<1, SORT_SMALL, 0, s>>>(ncand, E.c_elem0.p, E.c_key0.p, E.c_tup0.p, E.c_p0.p,
                                                   E.c_st0.p, E.c_reason0.p, E.C);
        } else {
            k_iota<<<nblk(ncand), 256, 0, s>>>(ncand, E.order0.p);
            E.sort_desc(E.c_key0.p, E.skey.p, E.order0.p, E.order1.p, ncand);
            k_fix_ties<<<nblk(ncand), 256, 0, s>>>(ncand, E.skey.p, E.order1.p, E.c_tup0.p);
            k_permute<<<nblk(ncand), 256, 0, s>>>(ncand, E.order1.p, E.c_elem0.p, E.c_key0.p, E.c_tup0.p,
                                                E.c_p0.p, E.c_st0.p, E.c_reason0.p, E.C);
        }
        E.pend(1);
        // step 3: locate
        if (cls != CLS_SS) { E.pbegin(); k_locate<<<nblk(ncand, 64), 64, 0, s>>>(E.M, cls, E.C); E.pend(2); }
        // steps 4-5: grow and validate.  Pools are sized from the previous
        // round's use per candidate; candidates whose results did not fit are
        // evaluated again after the pools grow, and regions over the LDS tiles
        // are evaluated again with global-memory tiles.
        E.ensure_pools(E.pool_need(1, ncand, cls), E.pool_need(2, ncand, cls), E.pool_need(3, ncand, cls),
                       E.pool_need(4, ncand, cls));
        // A pass evaluates every candidate once: small LDS tiles, then the
        // regions over them with medium LDS tiles, then global-memory tiles.
        // When a result pool was full the pass is repeated whole with fresh
        // pools sized for everything it reserved (no pool is ever copied).
        int ncl_final = 0;
        for (int pass = 0;; ++pass) {
            if (pass > 0) k_round_reset_pools<<<1, 64, 0, s>>>(E.ctr.p);
            // early-stop mode: this pass's marks compare above every earlier one
            E.PL.es_mark = early_stop ? E.mark.p : nullptr;
            E.PL.es_pass = early_stop ? E.pass++ : 0u;
            E.pbegin(3);
            k_grow_lds<QM_TILES_SMALL><<<std::min(ncand, 16384), 64, 0, s>>>(E.M, cls, E.C, E.PL,
                                                                             pass == 0 ? E.BP : E.BPnoprof(),
                                                                             nullptr, 0, nullptr, min_tier);
            E.pend(3);
            int* const cw = hbase + 48;  // ctr[0..46) after a grow pass
            for (int attempt = 0;; ++attempt) {
                if (attempt > 0 || pass > 0) {
                    HIPCK(hipMemsetAsync(olist_n, 0, 3 * sizeof(int), s));
                    HIPCK(hipMemsetAsync(olist_n + 4, 0, sizeof(int), s));
                }
                k_overflow_list<<<nblk(ncand), 256, 0, s>>>(E.C, E.olist.p, E.glist.p, olist_n);
                HIPCK(hipMemcpyAsync(cw, E.ctr.p, 46 * sizeof(int), hipMemcpyDeviceToHost, s));
                HIPCK(hipStreamSynchronize(s));
                const int nover = cw[32], nbig = cw[36];
                if (cw[34]) {
                    if (tile_scale >= B_MAXSCALE)
                        throw QmError(QM_ECAPACITY, "a region exceeds the largest supported size (round " +
                                                        std::to_string(round) + ", class " + std::to_string(cls) +
                                                        ", " + std::to_string(cw[34]) + " regions, tile code " +
                                                        std::to_string(cw[35]) + ", reached " +
                                                        std::to_string(cw[44]) + " region tets, " +
                                                        std::to_string(cw[45]) + " tested)");
                    tile_scale *= 4;
                    if (verbose)
                        fprintf(stderr, "qm: round %d class %d: %d regions over the global tiles (code %d), "
                                "tile scale %d\n", round, cls, cw[34], cw[35], tile_scale);
                    HIPCK(hipMemsetAsync(E.ctr.p + 35, 0, sizeof(int), s));
                }
                note("grown; regions over the tiles", round, cls, nover + nbig);
                if (E.prof) E.prof_over += nover + nbig;
                if (nover + nbig == 0) break;
                if (attempt >= 64) throw QmError(QM_EINTERNAL, "regions kept outgrowing the tiles");
                const BfPool BPr = E.BPnoprof();
                if (nover > 0) {             // hybrid tier (a shared-counter loop: any grid)
                    E.pbegin(8);
                    const GrowTiles HT = hybrid_tiles();
                    const size_t block = lists_slab_bytes(HT);
                    // the workgroups that stay resident (two per CU): they take the
                    // candidates from a shared counter, so more would only add slab
                    const int grid = E.slab_grid(std::min(nover, noalloc ? 4 : 512), block, E.hslab.cap);
                    E.hslab.ensure_exact(block * grid, s);
                    int* const next = E.ctr.p + 56;      // the shared candidate counter
                    HIPCK(hipMemsetAsync(next, 0, sizeof(int), s));
                    k_grow_hybrid<H_LANES, H_HCAP, H_RFHCAP, H_QHCAP><<<grid, H_LANES, 0, s>>>(
                        E.M, cls, E.C, E.PL, BPr, E.olist.p, nover, HT, E.hslab.p, block, next);
                    E.pend(8);
                }
                if (nbig > 0) {              // global-memory tiles
                    const GrowTiles BT = big_tiles(tile_scale);
                    const size_t slab_block = grow_slab_bytes(BT);
                    // up to 1024 workgroups (three resident per CU) and 8 GiB of tiles
                    int grid = (int)std::min<size_t>({(size_t)nbig, 1024,
                                                      std::max<size_t>(1, (8ull << 30) / slab_block)});
                    if (noalloc) grid = std::min(grid, 2);
                    grid = E.slab_grid(grid, slab_block, E.slab.cap);
                    E.pbegin(9);
                    E.slab.ensure_exact(slab_block * grid, s);
                    k_grow_global<B_LANES><<<grid, B_LANES, 0, s>>>(E.M, cls, E.C, E.PL, BPr, E.glist.p, nbig, BT, E.slab.p,
                                                      slab_block);
                    E.pend(9);
                }
            }
            if (!cw[5]) { E.pool_seen(cw, ncand, cls); ncl_final = cw[3]; break; }
            // a pool was full: the counters hold everything this pass reserved
            if (E.prof) E.prof_full += cw[33];
            if (pass >= 8) throw QmError(QM_ENOMEM, "result pools kept overflowing");
            auto need = [](int used, size_t cap) { return std::max(cap, (size_t)used + (size_t)used / 8 + 4096); };
            E.ensure_pools(need(cw[1], E.p_bfr.cap / BFR), need(cw[2], E.p_be.cap), need(cw[3], E.p_cl.cap),
                           need(cw[4], E.p_q.cap));
            note("result pools grown; evaluating the round again", round, cls, pass + 1);
        }
        const int ncl = std::min(ncl_final, E.PL.cap_cl);
        // verdicts: flags of rejected / exempted candidates, round statistics,
        // selection state
        E.pbegin();
        k_verdicts<<<nblk(ncand), 256, 0, s>>>(E.M, cls, E.C, E.PL, stats_d);
        E.pend(4);
        // step 6: maximal set of disjoint claim sets, greedy by priority, in
        // batches of passes; step 7 ids and slots are scanned with each batch
        // and taken once the selection is complete (one synchronisation)
        auto scans = [&](bool cap) {
            E.pbegin();
            if (!cap && ncand <= SCAN_SMALL) {
                k_scan_small<<<1, 1024, 0, s>>>(E.C, cls, ncand, E.sk.p, E.st_.p, E.ss_.p, tot_d);
                E.pend(6);
                return;
            }
            k_scan_vals<<<nblk(ncand), 256, 0, s>>>(E.C, cls, E.vk.p, E.vt.p, E.vs.p);
            E.exscan(E.vk.p, E.sk.p, ncand);
            if (cap) {
                k_cap_kept<<<nblk(ncand), 256, 0, s>>>(E.C, E.sk.p, opt->max_kept);
                k_scan_vals<<<nblk(ncand), 256, 0, s>>>(E.C, cls, E.vk.p, E.vt.p, E.vs.p);
                E.exscan(E.vk.p, E.sk.p, ncand);
            }
            E.exscan(E.vt.p, E.st_.p, ncand);
            E.exscan(E.vs.p, E.ss_.p, ncand);
            k_totals<<<1, 1, 0, s>>>(ncand, E.sk.p, E.vk.p, E.st_.p, E.vt.p, E.ss_.p, E.vs.p, tot_d);
            E.pend(6);
        };
        int passes = 0;
        const bool small_sel = ncl > 0 && ncl <= MIS_SMALL && ncand <= MIS_SMALL;
        if (small_sel) {
            E.pbegin();
            k_mis_small<<<1, 1024, 0, s>>>(ncl, E.p_cl.p, E.p_clc.p, ncand, E.state.p, E.mark.p, E.owner.p,
                                           E.mis_drop.p, E.mis_lose.p, E.pass, MIS_SMALL_PASSES, npass_d);
            E.pend(5);
        }
        for (int batch = 0;; ++batch) {
            if (ncl > 0 && !small_sel) {
                if (batch > 0) HIPCK(hipMemsetAsync(undec_d, 0, MIS_BATCH * sizeof(int), s));
                E.pbegin();
                for (int b = 0; b < MIS_BATCH; ++b) {
                    const unsigned ps = E.pass++;
                    const int p = batch * MIS_BATCH + b;     // pass of this round
                    int* const u_out = (p & 1) ? E.ulist1.p : E.ulist0.p;
                    int* const nu_out = nu_d + (p & 1);
                    if (p == 0) {            // every accepted candidate: one thread per claim
                        k_mis_mark<<<nblk(ncl), 256, 0, s>>>(ncl, E.p_cl.p, E.p_clc.p, E.state.p, E.mark.p, ps,
                                                             nullptr);
                        k_mis_check<<<nblk(ncl), 256, 0, s>>>(ncl, E.p_cl.p, E.p_clc.p, E.state.p, E.mark.p,
                                                              E.owner.p, ps, E.mis_drop.p, E.mis_lose.p, nullptr);
                        k_mis_decide<<<nblk(ncand), 256, 0, s>>>(ncand, E.state.p, E.mis_drop.p, E.mis_lose.p,
                                                                 undec_d + b, nullptr, u_out, nu_out);
                        k_mis_commit<<<nblk(ncl), 256, 0, s>>>(ncl, E.p_cl.p, E.p_clc.p, E.state.p, E.owner.p,
                                                               nullptr);
                    } else {                 // the undecided ones only: one wave per candidate
                        const int* const u_in = (p & 1) ? E.ulist0.p : E.ulist1.p;
                        const int* const nu_in = nu_d + ((p - 1) & 1);
                        k_mis_mark_list<<<MIS_LIST_GRID, 256, 0, s>>>(u_in, nu_in, E.C, E.p_cl.p, E.mark.p, ps,
                                                                      nu_out);
                        k_mis_check_list<<<MIS_LIST_GRID, 256, 0, s>>>(u_in, nu_in, E.C, E.p_cl.p, E.mark.p,
                                                                       E.owner.p, ps, E.mis_drop.p, E.mis_lose.p);
                        k_mis_decide_list<<<MIS_LIST_GRID / 4, 256, 0, s>>>(u_in, nu_in, E.state.p, E.mis_drop.p,
                                                                            E.mis_lose.p, undec_d + b, u_out,
                                                                            nu_out);
                        k_mis_commit_list<<<MIS_LIST_GRID, 256, 0, s>>>(u_in, nu_in, E.C, E.p_cl.p, E.state.p,
                                                                        E.owner.p);
                    }
                }
                E.pend(5);
            }
            scans(false);
            sync_counters();
            if (small_sel) {
                if (hc[38] < 0) throw QmError(QM_EINTERNAL, "selection did not finish");
                passes = hc[38];
                E.pass += (unsigned)passes;      // marks of later passes must compare higher
                break;
            }
            if (ncl > 0)
                for (int b = 0; b < MIS_BATCH; ++b) {
                    ++passes;
                    if (hc[40 + b] == 0) break;
                }
            if (ncl == 0 || hc[40 + MIS_BATCH - 1] == 0) break;
            note("selection batch", round, cls, batch + 1);
        }
        if (opt->max_kept > 0) {        // a cap applies to the complete selection
            scans(true);
            sync_counters();
        }
        const int nkept = hc[11], newt = hc[12], newss = hc[13];
        const int* st = hc + 16;
        if (st[13]) throw QmError(QM_EINTERNAL, "candidate left unresolved");
        if (nkept > 0) {
            E.ensure_mesh(E.M.nv + nkept, E.M.nt + newt, E.M.nss + newss);
            k_kept_list<<<nblk(ncand), 256, 0, s>>>(E.C, E.sk.p, E.kept.p);
            int grid = std::min(nkept, 16384);
            E.pbegin();
            k_insert<<<grid, 64, 0, s>>>(E.M, cls, E.C, E.PL, E.BP, E.kept.p, nkept, E.sk.p, E.st_.p, E.ss_.p,
                                         E.M.nv, E.M.nt, E.M.nss, dead_d);
            E.pend(7);
            E.M.nv += nkept; E.M.nt += newt; E.M.nss += newss;
        }
        if (ncl > 0) k_mis_release<<<nblk(ncl), 256, 0, s>>>(ncl, E.p_cl.p, E.p_clc.p, E.owner.p);
        int rec[QM_ROUND_FIELDS] = {cls, st[0], st[1], st[2], st[3], nkept};
        for (int r = 1; r < EX_NREASON; ++r) rec[5 + r] = st[3 + r];
        rec[15] = E.M.nv;
        rec[16] = E.M.nt - (int)E.dead;   // completed at the next synchronisation
        if (R) R->rounds.insert(R->rounds.end(), rec, rec + QM_ROUND_FIELDS);
        ST.inserted[cls] += nkept;
        if (verbose && std::chrono::steady_clock::now() - last_note > std::chrono::seconds(5)) {
            last_note = std::chrono::steady_clock::now();
            fprintf(stderr, "qm: round %d class %d candidates %d inserted %d vertices %d\n", round, cls, ncand,
                    nkept, E.M.nv);
        }
        last_ncand = ncand;
        ST.candidates += ncand;
        ST.mis_passes += passes;
        ST.deferred += st[14];
    }
    if (!noalloc) HIPCK(hipEventRecord(e2, s));
    sync_counters();
    auto T2s = std::chrono::steady_clock::now();
    patch_last_record();
    // verdicts of the last round's candidates: the candidate arrays are only
    // rewritten by a round that has candidates, so they still hold that round
    if (last_ncand > 0 && !noalloc) read_last_round(E, R.get(), last_ncand);


    const int gerr = read1(E.M.err, s);
    if (gerr) throw QmError(QM_EINTERNAL, "exact predicate precondition failed (code " + std::to_string(gerr) + ")");
    // ---- output: live tets and subfaces compacted in slot order
    qm_options opt_out = *opt;
    if (status == 2) opt_out.flags &= ~QM_OUTPUT_DEVICE;   // a checkpoint is kept on the host
    ST.nt_out = emit_output(E, R.get(), &opt_out, ar, dout);
    float ms_setup = 0, ms_ref = 0;
    if (noalloc) {            // host clock: the call's stream was synchronised at both points
        ms_setup = (float)std::chrono::duration<double, std::milli>(T1s - T0).count();
        ms_ref = (float)std::chrono::duration<double, std::milli>(T2s - T1s).count();
    } else {
        HIPCK(hipEventElapsedTime(&ms_setup, e0, e1));
        HIPCK(hipEventElapsedTime(&ms_ref, e1, e2));
        (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); (void)hipEventDestroy(e2);
    }
    if (E.prof_grow) {             // the stream is synchronised: every pair is complete
        E.pflush();
        for (int f : {3, 8}) { ST.prof_ms[f] = E.prof_ms[f]; ST.prof_launches[f] = E.prof_n[f]; }
    }
    if (E.prof) {
        for (int i = 0; i < QM_PROF_FAMILIES; ++i) { ST.prof_ms[i] = E.prof_ms[i]; ST.prof_launches[i] = E.prof_n[i]; }
        unsigned long long pc[4 + GROW_PHASES + 3 * TPROF_W];
        HIPCK(hipMemcpy(pc, E.pctr.p, sizeof pc, hipMemcpyDeviceToHost));
        for (int i = 0; i < GROW_PHASES; ++i) ST.prof_grow_cycles[i] = (int64_t)pc[4 + i];
        for (int i = 0; i < 3 * TPROF_W; ++i) ST.prof_tier[i / TPROF_W][i % TPROF_W] = (int64_t)pc[4 + GROW_PHASES + i];
        ST.prof_tested = (int64_t)pc[0]; ST.prof_region = (int64_t)pc[1];
        ST.prof_bfaces = (int64_t)pc[2]; ST.prof_claims = (int64_t)pc[3];
        ST.prof_scan_tets = scan_tets; ST.prof_scan_verts = scan_verts;
        ST.prof_overflow = E.prof_over;
        ST.prof_poolfull = E.prof_full;
    }
    ST.rounds = round;
    ST.status = status;
    ST.device_bytes_peak = (int64_t)E.acct.peak;
    ST.nv_out = E.M.nv;
    ST.seconds_setup = ms_setup * 1e-3;
    ST.seconds_refine = ms_ref * 1e-3;
    ST.seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - T0).count();
    (void)T1;
    if (noalloc) *dstats = ST;
    else {
        R->stats = ST;
        R->st_rounds = (rs ? rs->rounds : 0) + round;
        R->st_next = subphases ? sub : 0;
        *out = R.release();
    }
    return status == 1 ? QM_EROUNDS : QM_OK;
}

// One refinement with errors turned into return codes; mem_cap > 0 bounds
// the slab tiles of the larger grow tiers to what fits beside the call's
// other buffers in that many bytes (the served form passes each job's
// admitted estimate).
static int refine_within(const qm_plc* plc, const qm_mesh* in, const qm_options* opt, hipStream_t s,
                         qm_result** out, size_t mem_cap, const qm_state* rs = nullptr,
                         const std::atomic<bool>* stop = nullptr) {
    g_err.clear();
    try {
        return run_refine(plc, in, opt, s, out, nullptr, nullptr, nullptr, mem_cap, rs, stop);
    } catch (const QmError& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return QM_EINTERNAL;
    } catch (...) {
        g_err = "unknown failure";
        return QM_EINTERNAL;
    }
}

extern "C" {

int qm_refine(const qm_plc* plc, const qm_mesh* in, const qm_options* opt, void* hip_stream, qm_result** out) {
    return refine_within(plc, in, opt, (hipStream_t)hip_stream, out, 0);
}

int qm_refine_resume(const qm_plc* plc, const qm_mesh* in, const qm_state* st, const qm_options* opt,
                     void* hip_stream, qm_result** out) {
    if (!st) { g_err = "null state"; return QM_EINVAL; }
    return refine_within(plc, in, opt, (hipStream_t)hip_stream, out, 0, st);
}

int qm_result_state(const qm_result* r, qm_state* o) {
    if (!r || !o) { g_err = "null argument"; return QM_EINVAL; }
    o->hmin2 = r->st_hmin2;
    o->rounds = r->st_rounds;
    o->next_class = r->st_next;
    o->nt = (int32_t)r->st_tfl.size(); o->nsf = (int32_t)r->st_sfl.size(); o->nss = (int32_t)r->st_ssl.size();
    o->tet_flags = r->st_tfl.data(); o->sf_flags = r->st_sfl.data(); o->ss_flags = r->st_ssl.data();
    return QM_OK;
}

}  // extern "C"

// ---- scratch of the no-alloc entry point: one array per device (each
// device that runs the entry point holds its own copy until the process
// ends).  Host code never names it as an address: its device address is
// taken once per device with hipGetSymbolAddress and kept below.
static __device__ __align__(256) char scratch[QM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_rc[kMaxDevices];
std::mutex g_scratch_mu[kMaxDevices];   // calls on one device take turns
}  // namespace

extern "C" {

int qm_refine_noalloc(const qm_plc* plc, const qm_mesh* in, const qm_options* opt, void* hip_stream,
                      qm_mesh_buf* out, qm_stats* stats) {
    g_err.clear();
    try {
        int dev = -1;
        HIPCK(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevices) throw QmError(QM_EDEVICE, "device index out of range");
        std::call_once(g_scratch_once[dev], [dev] {   // the current device is `dev`
            g_scratch_rc[dev] = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
        });
        if (g_scratch_rc[dev] != hipSuccess || !g_scratch_ptr[dev])
            throw QmError(QM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(g_scratch_rc[dev]));
        std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
        Arena A;
        A.base = static_cast<char*>(g_scratch_ptr[dev]);
        A.cap = QM_NOALLOC_SCRATCH_BYTES;
        return run_refine(plc, in, opt, (hipStream_t)hip_stream, nullptr, &A, out, stats);
    } catch (const QmError& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return QM_EINTERNAL;
    } catch (...) {
        g_err = "unknown failure";
        return QM_EINTERNAL;
    }
}

// ---- tests only: the device predicates and constructions on given points
__global__ void k_test_geometry(int op, int n, const double* in, double param, double* out, int* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int w = op == 0 || op == 4 || op == 5 || op == 12 || op == 13 ? 12 : op == 1 ? 15 : op == 10 ? 6 : 9;
    const double* q = in + (size_t)w * i;
    double p[4] = {0, 0, 0, 0};
    double* o = out + 4 * (size_t)i;
    switch (op) {
        case 0: o[0] = orient3d(q, q + 3, q + 6, q + 9, err); break;
        case 1: o[0] = insphere(q, q + 3, q + 6, q + 9, q + 12, err); break;
        case 2: o[0] = orient2d((int)param, q, q + 3, q + 6, err); break;
        case 3: o[0] = segdot(q, q + 3, q + 6, err); break;
        case 4: o[0] = facedot(q, q + 3, q + 6, q + 9, err); break;
        case 5: o[0] = orient3d_any(q, q + 3, q + 6, q + 9, err); break;
        case 10: midpoint(q, q + 3, p); break;
        case 11: tri_cc(q, q + 3, q + 6, p); break;
        case 12: tet_cc(q, q + 3, q + 6, q + 9, p, p[3]); break;
        case 13: o[0] = is_bad(q, q + 3, q + 6, q + 9, param * param) ? 1.0 : 0.0; break;
        default: atomicOr(err, 1 << 30); return;
    }
    if (op >= 10 && op <= 12)
        for (int k = 0; k < 4; ++k) o[k] = p[k];
}

// Instances of a batch run concurrently: worker threads, each with its own
// stream on the caller's device, take the instances in index order.
int qm_refine_batch(int32_t n, const qm_plc* plcs, const qm_mesh* meshes, const qm_options* opts,
                    int32_t nstreams, qm_result** outs, int32_t* codes) {
    g_err.clear();
    if (n < 0 || (n > 0 && (!plcs || !meshes || !opts || !outs || !codes)) || nstreams < 1) {
        g_err = "bad batch arguments";
        return QM_EINVAL;
    }
    for (int i = 0; i < n; ++i) { outs[i] = nullptr; codes[i] = QM_EINTERNAL; }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { g_err = "no HIP device"; return QM_EDEVICE; }
    std::atomic<int> next{0};
    std::vector<std::string> msgs(n);
    auto work = [&]() {
        if (hipSetDevice(dev) != hipSuccess) return;
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
        for (int i = next++; i < n; i = next++) {
            codes[i] = qm_refine(&plcs[i], &meshes[i], &opts[i], st, &outs[i]);
            if (codes[i] != QM_OK && codes[i] != QM_EROUNDS) msgs[i] = qm_last_error();
        }
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    };
    std::vector<std::thread> th;
    const int nw = std::min<int>(nstreams, std::max(n, 1));
    for (int w = 0; w < nw; ++w) th.emplace_back(work);
    for (auto& t : th) t.join();
    for (int i = 0; i < n; ++i)
        if (codes[i] != QM_OK && codes[i] != QM_EROUNDS) {
            g_err = "instance " + std::to_string(i) + ": " + (msgs[i].empty() ? "not run" : msgs[i]);
            return codes[i];
        }
    return QM_OK;
}

int qm_result_view(const qm_result* r, qm_mesh* v, qm_stats* st) {
    if (!r) { g_err = "null result"; return QM_EINVAL; }
    if (v && r->on_device) {
        v->nv = r->dnv; v->xyz = r->d_xyz; v->nt = r->dnt; v->tet = r->d_tets;
        v->nsf = r->dnsf; v->sf = r->d_sf; v->sf_facet = r->d_sff;
        v->nss = r->dnss; v->ss = r->d_ss; v->ss_seg = r->d_ssg;
    } else if (v) {
        v->nv = (int32_t)(r->xyz.size() / 3); v->xyz = r->xyz.data();
        v->nt = (int32_t)(r->tets.size() / 4); v->tet = r->tets.data();
        v->nsf = (int32_t)r->sff.size(); v->sf = r->sf.data(); v->sf_facet = r->sff.data();
        v->nss = (int32_t)r->ssg.size(); v->ss = r->ss.data(); v->ss_seg = r->ssg.data();
    }
    if (st) *st = r->stats;
    return QM_OK;
}

int qm_result_rounds(const qm_result* r, int32_t* buf, int32_t cap) {
    if (!r) { g_err = "null result"; return QM_EINVAL; }
    int n = (int)(r->rounds.size() / QM_ROUND_FIELDS);
    if (buf) std::memcpy(buf, r->rounds.data(), sizeof(int32_t) * QM_ROUND_FIELDS * (size_t)std::min(n, (int)cap));
    return n;
}

int qm_result_last_round(const qm_result* r, int32_t* buf, int32_t cap) {
    if (!r) { g_err = "null result"; return QM_EINVAL; }
    int n = (int)(r->last.size() / 9);
    if (buf) std::memcpy(buf, r->last.data(), sizeof(int32_t) * 9 * (size_t)std::min(n, (int)cap));
    return n;
}

int qm_result_round_profile(const qm_result* r, double* buf, int32_t cap) {
    if (!r) { g_err = "null result"; return QM_EINVAL; }
    int n = (int)(r->round_ms.size() / QM_PROF_FAMILIES);
    if (buf) std::memcpy(buf, r->round_ms.data(), sizeof(double) * QM_PROF_FAMILIES * (size_t)std::min(n, (int)cap));
    return n;
}

void qm_result_free(qm_result* r) { delete r; }

int qm_test_geometry(int32_t op, int32_t n, const double* in, double param, double* out) {
    g_err.clear();
    try {
        if (n < 0 || (n > 0 && (!in || !out)) || !((op >= 0 && op <= 5) || (op >= 10 && op <= 13)))
            throw QmError(QM_EINVAL, "bad arguments");
        if (n == 0) return QM_OK;
        const int w = op == 0 || op == 4 || op == 5 || op == 12 || op == 13 ? 12 : op == 1 ? 15 : op == 10 ? 6 : 9;
        double *din = nullptr, *dout = nullptr;
        int* derr = nullptr;
        HIPCK(hipMalloc((void**)&din, sizeof(double) * w * (size_t)n));
        HIPCK(hipMalloc((void**)&dout, sizeof(double) * 4 * (size_t)n));
        HIPCK(hipMalloc((void**)&derr, sizeof(int)));
        HIPCK(hipMemset(derr, 0, sizeof(int)));
        HIPCK(hipMemcpy(din, in, sizeof(double) * w * (size_t)n, hipMemcpyHostToDevice));
        k_test_geometry<<<nblk(n), 256>>>(op, n, din, param, dout, derr);
        HIPCK(hipGetLastError());
        int e = 0;
        HIPCK(hipMemcpy(out, dout, sizeof(double) * 4 * (size_t)n, hipMemcpyDeviceToHost));
        HIPCK(hipMemcpy(&e, derr, sizeof(int), hipMemcpyDeviceToHost));
        (void)hipFree(din); (void)hipFree(dout); (void)hipFree(derr);
        if (e) throw QmError(QM_EINVAL, "a point is off the lattice or outside the cube (error word " +
                                            std::to_string(e) + ")");
        return QM_OK;
    } catch (const QmError& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return QM_EINTERNAL;
    }
}

const char* qm_last_error(void) { return g_err.c_str(); }

const char* qm_version(void) { return "qm 0.1 (gfx950)"; }

}  // extern "C"

#include "qm_lockstep.h"
#include "qm_server.h"
