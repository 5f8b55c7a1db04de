/*
 * qm.h -- C-ABI of libqm: round-based constrained Delaunay refinement on one
 * AMD MI355X (gfx950).
 *
 * Problem (paper, Section 1): given a piecewise linear complex G = (P, E, F),
 * a constrained Delaunay tetrahedralisation (CDT) T conforming to G and a
 * bound B, add Steiner points so that the result is again a CDT conforming to
 * G whose tetrahedra mostly have radius-edge ratio at most B.  Method (paper,
 * Section 2): subsegments, then subfaces, then bad tetrahedra are split in
 * rounds; each round computes splitting points, grows their Delaunay regions,
 * keeps a set of points with disjoint regions (priority blasting) and inserts
 * them concurrently.
 *
 * All entry points return 0 on success or a negative QM_E* code; the message
 * of the last failure on the calling thread is qm_last_error().  No C++
 * exception crosses this boundary.
 *
 * Coordinates: FP64, row-major [n][3], every value a multiple of 2^-53 inside
 * the closed unit cube [0,1]^3 (the coordinate lattice; the library rounds
 * every splitting point onto it, which keeps all predicates exact).  Ids are
 * int32, 0-based.
 */
#ifndef QM_H
#define QM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QM_OK 0
#define QM_EINVAL (-1)        /* bad ids, off-lattice or out-of-cube coordinates, B <= 0 */
#define QM_ENONCONFORM (-2)   /* a subface or subsegment is not a face or edge of the mesh,
                                 a tet is not positively oriented, or faces do not match */
#define QM_ENOMEM (-3)        /* device or host allocation failed */
#define QM_EROUNDS (-4)       /* round guard reached (the result is still returned) */
#define QM_EDEVICE (-5)       /* HIP runtime error */
#define QM_EINTERNAL (-6)     /* a kernel found an impossible state (bug) */
#define QM_ECAPACITY (-7)     /* a cavity exceeded the largest supported region size */
#define QM_EAGAIN (-8)        /* server: over the memory budget now, or the job is not done yet */

/* The PLC G = (P, E, F): polygons are given as triangles carrying a polygon
   (facet) id.  Borrowed for the duration of the call. */
typedef struct qm_plc {
    int32_t nv;              /* |P|; P are the first nv vertices of the mesh */
    int32_t nseg;            /* |E| */
    const int32_t* seg;      /* [nseg][2] */
    int32_t nftri;           /* triangles of the polygons of F */
    const int32_t* ftri;     /* [nftri][3] */
    const int32_t* ftri_facet;   /* [nftri] polygon id, 0-based, dense */
} qm_plc;

/* A mesh: vertices, tetrahedra, subfaces and subsegments (paper, Section 1
   definitions).  As input it is the CDT T; borrowed, never written. */
typedef struct qm_mesh {
    int32_t nv;
    const double* xyz;       /* [nv][3] */
    int32_t nt;
    const int32_t* tet;      /* [nt][4], each positively oriented:
                                det[b-a; c-a; d-a] > 0 */
    int32_t nsf;
    const int32_t* sf;       /* [nsf][3] subfaces (faces of T lying on polygons) */
    const int32_t* sf_facet; /* [nsf] polygon id of each subface */
    int32_t nss;
    const int32_t* ss;       /* [nss][2] subsegments (edges of T lying on segments) */
    const int32_t* ss_seg;   /* [nss] segment id of each subsegment */
} qm_mesh;

#define QM_INPUT_DEVICE 1u   /* mesh/PLC arrays are device pointers (same device) */
#define QM_PROFILE 2u        /* time each kernel family with HIP events on the call's
                                stream and count the region work (qm_stats.prof_*) */
#define QM_VERBOSE 4u        /* progress line on stderr every few seconds of rounds */
#define QM_PROFILE_GROW 8u   /* time only the grow launches with small LDS tiles and those of
                                the hybrid tier (families 3 and 8 of qm_stats.prof_ms and
                                prof_launches; the rest stay 0) with HIP events on the call's
                                stream; the kernels run as unprofiled. Ignored with QM_PROFILE */
#define QM_EARLY_STOP 256u   /* a non-parity mode: early-stop blasting as the paper runs it
                                (Section 2): while growing, a candidate marks each tet it takes
                                with its priority and stops, for this round, on meeting a
                                higher priority's mark.  The kept points still have disjoint
                                claim sets and full validation, so the output is a CDT of the
                                same kind, but which points win depends on timing: the result
                                is not reproducible and not the oracle's. */
#define QM_SUBPHASE_ROUNDS 1024u   /* the other class-order reading: each round runs three sub-phases in the
                                     paper's order (Section 2: subsegments, then subfaces, then bad
                                     tets), each the usual round restricted to its class (that
                                     class classified alone, so a later class no longer waits for
                                     the earlier ones to run out); a sub-phase without candidates
                                     is skipped and not counted as a round, and the refinement
                                     ends after three empty sub-phases in a row.  Encroachment of
                                     constraints by a later class's points is rejected and queued
                                     as usual.  Reproducible, a CDT of the same kind; it equals
                                     the oracle refined with the same reading, not the paper-order
                                     refinement (the insertion order differs) */
#define QM_OUTPUT_DEVICE 512u   /* the result's output arrays stay on the device (same device):
                                   qm_result_view returns device pointers, valid until
                                   qm_result_free; records and statistics stay on the host */
#define QM_TEST_ERROR_WORD 16u  /* tests only: raise this call's device error word at set-up, so
                                   the call ends with QM_EINTERNAL (the word is per call: other
                                   calls, concurrent or later, are not affected) */
#define QM_TEST_TIER1 32u     /* tests only: every region is grown with the medium tiles (or larger) */
#define QM_TEST_TIER2 64u     /* tests only: every region is grown with the global-memory tiles */
#define QM_TEST_KEY_COLLIDE 128u  /* tests only: priority keys keep their top 3 bits (the rest 0),
                                     so many are equal and the tie rule (ascending tuple) orders them */

typedef struct qm_options {
    double B;                /* radius-edge bound (> 0) */
    double hmin_factor;      /* h_min = hmin_factor * shortest input edge (0.5 typical) */
    int32_t max_rounds;      /* round guard; QM_EROUNDS when reached */
    int32_t max_kept;        /* > 0: insert at most this many points per round */
    uint32_t flags;          /* QM_INPUT_DEVICE | QM_PROFILE | QM_VERBOSE | QM_PROFILE_GROW |
                                QM_TEST_ERROR_WORD | QM_TEST_TIER1 | QM_TEST_TIER2 |
                                QM_TEST_KEY_COLLIDE */
} qm_options;

/* per-round record (17 int32): class (0 subsegment, 1 subface, 2 tet),
   candidates, accepted, rejected, exempted, inserted, exempted by reason
   (non-finite point, walk cap, encroached exempt element, h_min, region
   subface without region tets, invisible boundary face, invisible 2D
   boundary edge, unclosed cavity boundary, a new face that would not be
   locally Delaunay), vertices after, tets after */
#define QM_ROUND_FIELDS 17
#define QM_PROF_FAMILIES 10

typedef struct qm_stats {
    int32_t rounds;
    int32_t status;          /* 0 converged, 1 round guard reached */
    int64_t inserted[3];     /* Steiner points by class */
    int64_t candidates;      /* candidate evaluations over all rounds */
    int64_t mis_passes;      /* marking passes of the disjoint-set selection */
    int64_t deferred;        /* QM_EARLY_STOP: evaluations stopped early by a higher priority */
    int64_t device_bytes_peak;   /* most device memory the call held at once (its own buffers) */
    int64_t nv_out, nt_out;  /* output sizes */
    double seconds_setup;    /* device-side setup from the input arrays */
    double seconds_refine;   /* round loop (device resident) */
    double seconds_total;    /* whole call incl. transfers */
    /* QM_PROFILE only: device milliseconds and launches per kernel family
       0 classify, 1 split+order, 2 locate, 3 grow+validate with the small
       LDS tiles, 4 flags+stats, 5 selection, 6 scans, 7 insert, 8 grow+
       validate of the regions over the small tiles (hybrid tier: LDS hash
       tables, lists in global memory), 9 the same for the regions over the
       hybrid tier (global-memory tiles) */
    double prof_ms[QM_PROF_FAMILIES];
    int64_t prof_launches[QM_PROF_FAMILIES];
    /* QM_PROFILE only: region work of the grow kernel with LDS tiles (family
       3): tets tested, region tets, boundary faces, claimed tets (accepted
       candidates) */
    int64_t prof_tested, prof_region, prof_bfaces, prof_claims;
    /* QM_PROFILE only: tets and vertices scanned by the tet classification */
    int64_t prof_scan_tets, prof_scan_verts;
    /* QM_PROFILE only: candidates evaluated again with global-memory tiles
       (region over the LDS tiles), and again after a result pool grew */
    int64_t prof_overflow, prof_poolfull;
    /* QM_PROFILE only: shader-clock cycles of the small-tile grow kernel's
       phases summed over its workgroups: 0 set-up and seeds, 1 facet region,
       2 tet region, 3 encroachment, 4 insertion radius and facet-region tets,
       5 boundary faces, 6 2D boundary edges and closure, 7 claims and
       results (phases a candidate leaves early are not counted) */
    int64_t prof_grow_cycles[8];
    /* QM_PROFILE only: region evaluations by grow tier (0 small LDS tiles,
       1 medium LDS tiles, 2 global-memory tiles), 28 counters each:
       evaluations, evaluations that outgrew the tier's tiles, then over the
       others: tets tested, region tets, boundary faces, and the largest
       region, tested count and boundary-face count; then how often each
       tile overflowed (region list, tested-tet hash, facet region, queue,
       boundary faces, 2D boundary edges, claims, edge table), then accepted
       evaluations and their region tets, boundary faces and claims, then
       shader-clock cycles of the 8 phases (as prof_grow_cycles) */
    int64_t prof_tier[3][28];
} qm_stats;

typedef struct qm_result qm_result;

/* Refine one instance.  `hip_stream` is a hipStream_t (NULL: default stream).
   On success *out owns the output until qm_result_free. */
int qm_refine(const qm_plc* plc, const qm_mesh* in, const qm_options* opt, void* hip_stream,
              qm_result** out);

/* Refine n independent instances (each as qm_refine: the round loop of
   paper, Section 2, on its own mesh).  plcs, meshes and opts are arrays of n;
   the instances run concurrently on `nstreams` HIP streams of the calling
   thread's current device (default priority), each taken in index order by a
   worker thread.  outs[i] receives instance i's result (free each with
   qm_result_free) and codes[i] its return code.  Returns 0 when every
   instance returned 0 or QM_EROUNDS, else the code of the first instance that
   failed (qm_last_error names it).  Inputs are borrowed for the call. */
int qm_refine_batch(int32_t n, const qm_plc* plcs, const qm_mesh* meshes, const qm_options* opts,
                    int32_t nstreams, qm_result** outs, int32_t* codes);

/* Launch-shape knobs of the lockstep form.  None of them changes a result. */
typedef struct {
    int32_t groups;          /* lockstep groups (1..64): with more than one, the instances are dealt,
                                largest input first, to that many groups, each run by a host thread of
                                its own on a stream of its own (default priority) */
    int32_t classify_tiles;  /* 256-element tiles per classification workgroup (1..64) */
    int32_t rank_max;        /* rounds of up to this many candidates are ordered by one workgroup
                                (256..4096); larger ones by a radix sort */
    int32_t select_one_wg;   /* selections of up to this many claims and candidates run in one
                                workgroup (0..2^20); larger ones in passes over many workgroups */
    int32_t hybrid_wgs;      /* hybrid-tier workgroups of a launch, over all instances (16..4096) */
    int32_t global_wgs;      /* global-tier workgroups of a launch, over all instances (4..1024) */
} qm_lockstep_tune;

/* Refine n independent instances in lockstep: every instance runs the round
   loop of paper, Section 2, on its own mesh, and each phase of a round
   (classification, splitting points, location, region growth and
   validation, verdicts, selection, insertion) is one launch over the work of
   all instances of a group in that phase, each instance picking its own
   class.  Each result is bit-identical to qm_refine on the same instance.
   Arguments as qm_refine_batch; `tune` NULL means one group on `hip_stream`
   (a hipStream_t, NULL: default stream) with classify_tiles 8, rank_max
   4096, select_one_wg 65536, hybrid_wgs 1024, global_wgs 256; with
   tune->groups > 1 the groups run on streams of the library.  QM_EINVAL for
   knobs out of range.  Options may not ask for profiling (QM_PROFILE,
   QM_PROFILE_GROW), a non-parity mode (QM_EARLY_STOP, QM_SUBPHASE_ROUNDS) or
   max_kept > 0: such an instance ends with QM_EINVAL and the others go on.
   Every instance's mesh stays on the device until it finishes. */
int qm_refine_lockstep(int32_t n, const qm_plc* plcs, const qm_mesh* meshes, const qm_options* opts,
                       void* hip_stream, const qm_lockstep_tune* tune, qm_result** outs, int32_t* codes);

/* Choose the knobs of qm_refine_lockstep for a batch: a probe batch of
   `probe` instances, evenly spaced in input size, is refined with the
   knobs in turn (groups 1, 2, 4, 8; hybrid_wgs 256..2048; classify_tiles 2,
   8, 32; select_one_wg 8192, 65536, 262144; rank_max 1024, 4096; one pass of
   coordinate descent from groups 4 and the defaults, a change kept when it
   gains 3%); the fastest knobs go to *best and their probe time to
   *best_seconds (may be NULL).  Costs about a dozen refinements of the probe
   batch; the probe results are freed. */
int qm_lockstep_autotune(int32_t n, const qm_plc* plcs, const qm_mesh* meshes, const qm_options* opts,
                         int32_t probe, qm_lockstep_tune* best, double* best_seconds);

/* View of a result: the output mesh (Steiner vertices appended after the
   input vertices, numbered by round and priority) and the statistics.  The
   arrays are host memory, or device memory when the refinement ran with
   QM_OUTPUT_DEVICE.  Pointers stay valid until qm_result_free. */
int qm_result_view(const qm_result* r, qm_mesh* view, qm_stats* stats);

/* Copy at most `cap` rounds of per-round records (QM_ROUND_FIELDS each) into
   buf; returns the number of rounds available. */
int qm_result_rounds(const qm_result* r, int32_t* buf, int32_t cap);

/* Verdicts of the last round's candidates in priority order, 9 int32 each:
   sorted vertex ids (4, -1 padded), status (0 accepted, 1 rejected,
   2 exempted), exemption reason, inserted flag, region tets and boundary
   faces (accepted candidates).  Copies at most `cap`; returns the count.
   For inspecting one round of a run (max_rounds) against a reference. */
int qm_result_last_round(const qm_result* r, int32_t* buf, int32_t cap);

/* QM_PROFILE only: device milliseconds of each kernel family (as in
   qm_stats.prof_ms, QM_PROF_FAMILIES doubles) for each round; one more entry
   than rounds run holds the last classification (the one that found no work
   or was cut by the round guard).  Copies at most `cap` entries; returns the
   number recorded (0 without QM_PROFILE). */
int qm_result_round_profile(const qm_result* r, double* buf, int32_t cap);

void qm_result_free(qm_result* r);

/* ---- Checkpoint and resume ----------------------------------------------
   The round rule (paper, Section 2) carries, from one round to the next,
   the mesh and a few flags per element: a subsegment or subface queued by a
   rejected point (it is split in a later round although no vertex encroaches
   it) or exempted (its point was filtered away for good), and a bad tet
   exempted the same way.  h_min is fixed by the first input mesh's shortest
   edge.  A refinement stopped by max_rounds therefore resumes exactly from
   its output mesh and this state. */
typedef struct qm_state {
    double hmin2;              /* h_min^2 of the refinement (from its first call) */
    int32_t rounds;            /* rounds run so far, over every call */
    int32_t next_class;        /* QM_SUBPHASE_ROUNDS: the sub-phase run next (0 SS, 1 SF,
                                  2 TET); 0 otherwise */
    int32_t nt, nsf, nss;      /* lengths of the flag arrays: the mesh's counts */
    const uint8_t* tet_flags;  /* [nt] bit0 exempt; aligned with the mesh's tets */
    const uint8_t* sf_flags;   /* [nsf] bit0 queued, bit1 exempt; aligned with its subfaces */
    const uint8_t* ss_flags;   /* [nss] bit0 queued, bit1 exempt; aligned with its subsegments */
} qm_state;

/* The state after a refinement, aligned with qm_result_view's mesh arrays
   (host arrays, also for QM_OUTPUT_DEVICE results; valid until
   qm_result_free).  QM_EINVAL for a null argument. */
int qm_result_state(const qm_result* r, qm_state* out);

/* Continue a refinement: `in` is the mesh a call returned and `st` its
   state (qm_result_state; its arrays are host memory, the mesh's follow
   QM_INPUT_DEVICE as in qm_refine).  opt->hmin_factor is not used (st->hmin2
   is); opt->max_rounds bounds this call's rounds.  In the deterministic modes
   (the paper-order rounds and QM_SUBPHASE_ROUNDS) the output mesh and the
   round records of the calls together equal one uninterrupted qm_refine with
   the same options; with QM_EARLY_STOP the result is a valid refinement of
   the same kind.  QM_EINVAL when the state's counts differ from the mesh's,
   a flag has bits outside those listed, next_class is out of range or hmin2
   is negative or not finite; otherwise as qm_refine. */
int qm_refine_resume(const qm_plc* plc, const qm_mesh* in, const qm_state* st, const qm_options* opt,
                     void* hip_stream, qm_result** out);

/* ---- Without allocation ------------------------------------------------ */

/* Bytes of the static device scratch array used by qm_refine_noalloc (per
   device; held from the first call on that device until the process ends). */
#define QM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* Output arrays of qm_refine_noalloc: device pointers on the current device,
   owned by the caller, with their capacities in elements (rows).  The
   library writes the output mesh into them and its sizes into nv..nss; on
   QM_ECAPACITY the sizes reached are still written when known. */
typedef struct qm_mesh_buf {
    int32_t cap_v, cap_t, cap_sf, cap_ss;
    double* xyz;             /* [cap_v][3] */
    int32_t* tet;            /* [cap_t][4] */
    int32_t* sf;             /* [cap_sf][3] */
    int32_t* sf_facet;       /* [cap_sf] */
    int32_t* ss;             /* [cap_ss][2] */
    int32_t* ss_seg;         /* [cap_ss] */
    int32_t nv, nt, nsf, nss;
} qm_mesh_buf;

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   refinement as qm_refine, bit for bit, with no hipMalloc, hipFree, pinned
   host allocation, event or qm_result.  Every working buffer is carved from
   the library's static device array of QM_NOALLOC_SCRATCH_BYTES, so the
   meshes it can refine are small (about 10^5 output tets; more rounds with
   many candidates need more).  Inputs are device arrays (opt->flags must
   include QM_INPUT_DEVICE; profiling flags are refused).  The output goes to
   `out` (cap_v >= in->nv, cap_t >= in->nt, cap_ss >= in->nss required; tet
   slots of removed tets count against cap_t + cap_t/8 + 256) and the
   statistics to *stats; per-round records are not kept.  Returns
   QM_ECAPACITY when the scratch array or an output array is too small.
   Calls on one device share its scratch array; this library makes them take
   turns (a mutex per device), so calls that overlap in time are serialised,
   never mixed.  The array keeps the last call's contents, and every call
   clears what it needs. */
int qm_refine_noalloc(const qm_plc* plc, const qm_mesh* in, const qm_options* opt, void* hip_stream,
                      qm_mesh_buf* out, qm_stats* stats);

/* ---- Served form: refinement jobs (each one qm_refine, the round loop of
   paper, Section 2) arriving over time on one device -------------------- */

typedef struct qm_server qm_server;

typedef struct qm_server_stats {
    size_t budget;           /* device-memory budget given at creation (bytes) */
    size_t resident;         /* estimates of the admitted, unfinished jobs (bytes) */
    int32_t queued;          /* admitted jobs not started */
    int32_t running;         /* jobs being refined */
    int64_t admitted, refused, completed;   /* since creation; refused = QM_EAGAIN */
    int64_t evictions;       /* jobs taken off the device by qm_server_evict, since creation */
    int32_t parked;          /* evicted jobs not yet readmitted */
} qm_server_stats;

/* Device bytes the library budgets for refining this instance: 16 KB per
   input tet for B < 1.6, 8 KB otherwise, plus 320 MiB.  An upper estimate
   from measured peaks (qm_stats.device_bytes_peak), not a bound: a served
   job runs with its estimate as its budget, so the slab tiles of the larger
   grow tiers shrink to a quarter of it, but its mesh and result pools take what
   the refinement needs.  0 for bad arguments. */
size_t qm_estimate_bytes(const qm_plc* plc, const qm_mesh* in, const qm_options* opt);

/* Create a server on the calling thread's current device with `nworkers`
   (1..64) worker threads, each owning a HIP stream (non-blocking, default
   priority) on which it runs one job at a time.  With nworkers = 0 the
   server is stepped: admitted jobs form four lockstep batches (as
   qm_refine_lockstep; a new job joins the batch with the fewest resident
   input tets), each on a stream and a host thread of the server, stay
   resident on the device between rounds and advance only through
   qm_server_step; their
   options may not ask for profiling, a non-parity mode or max_kept > 0
   (such a job ends with QM_EINVAL).  `hbm_budget_bytes` bounds
   the summed estimates of admitted, unfinished jobs.  *out is freed with
   qm_server_destroy. */
int qm_server_create(size_t hbm_budget_bytes, int32_t nworkers, qm_server** out);

/* Submit one job (host arrays only; QM_INPUT_DEVICE is rejected).  The
   server copies the arrays, so they are borrowed for the call only.
   `est_bytes` is the job's device-memory estimate (0: qm_estimate_bytes).
   Returns 0 and a ticket when admitted; QM_EAGAIN when the estimate does not
   fit in the budget minus the resident estimates (nothing is kept: retry
   after jobs finish); QM_ENOMEM when it exceeds the whole budget.  Input
   errors of the job itself are reported by qm_server_poll. */
int qm_server_submit(qm_server* srv, const qm_plc* plc, const qm_mesh* in, const qm_options* opt,
                     size_t est_bytes, uint64_t* ticket);

/* Collect a job.  wait_ms: 0 returns at once, > 0 waits at most that long,
   < 0 waits until the job is done.  Returns QM_EAGAIN while it is not done;
   0 when done, with *out the result (or NULL if the job failed; free it with
   qm_result_free), *code the job's qm_refine return code (its message is
   then this thread's qm_last_error) and, if `seconds` is not NULL,
   seconds[0] the time queued and seconds[1] the time from submission to
   completion.  A ticket is collected once; unknown tickets give QM_EINVAL. */
int qm_server_poll(qm_server* srv, uint64_t ticket, int32_t wait_ms, qm_result** out, int32_t* code,
                   double* seconds);

/* Stepped server only (continuous batching): jobs admitted since the last
   step are set up on the device and join a batch, then every resident job
   runs one round of the paper's round loop (Section 2), each phase of the
   round one launch over all resident jobs of a batch, the batches at the
   same time; returns when the round is complete.  Jobs that finish (no work left, or their round guard) hand
   their result to qm_server_poll.  *nresident receives the number of jobs
   still resident.  Calls take turns.  QM_EINVAL on a server with workers. */
int qm_server_step(qm_server* srv, int32_t* nresident);

/* Take a job off the device (a server's HBM budget is then free for other
   jobs): a queued job leaves the queue; a running one ends at its next round
   boundary (the worker form waits for it; the stepped form evicts between
   steps), and its output mesh and refinement state (qm_result_state) become
   a host checkpoint.  Its estimate leaves the budget.  QM_OK when the job is
   evicted; QM_EAGAIN when it finished first (its result is ready to poll);
   QM_EINVAL for an unknown, collected, finished or already evicted ticket.
   qm_server_poll on an evicted job returns QM_EAGAIN at once. */
int qm_server_evict(qm_server* srv, uint64_t ticket);

/* Admit an evicted job again against the budget (QM_EAGAIN while it does
   not fit; it stays evicted).  It resumes from its checkpoint
   (qm_refine_resume) with the rounds left of its round limit.  The result it
   finally gives holds the round records and summed statistics of every
   segment, and its mesh and records equal the uninterrupted refinement's.
   QM_EINVAL when the ticket is not an evicted job. */
int qm_server_readmit(qm_server* srv, uint64_t ticket);

/* Counters of the server (a consistent snapshot). */
int qm_server_info(qm_server* srv, qm_server_stats* info);

/* Drop the jobs not yet started, wait for the running ones, free every
   uncollected result and the server.  No other call on `srv` may run
   concurrently with it or follow it. */
void qm_server_destroy(qm_server* srv);

/* Tests only: evaluate the device's exact predicates or FP64 constructions
   on n point tuples (host arrays; the call copies them to the device and
   back).  op and the tuple layout of `in` (points as x, y, z doubles):
     0 orient3d(a,b,c,d)  1 insphere(a,b,c,d,e)  2 orient2d dropping axis
     `param` (a,b,c)  3 segment encroachment (a,b,v)  4 equatorial-ball
     encroachment (a,b,c,v)  5 orient3d for any finite points (a,b,c,d):
     out[4i] is the sign (-1, 0, +1);
     10 midpoint(a,b)  11 triangle circumcentre(a,b,c)  12 tet circumcentre
     (a,b,c,d), out[4i..4i+3] = point and squared radius;  13 radius-edge
     ratio above B = `param` (a,b,c,d): out[4i] = 1 or 0.
   Ops 0-4 require lattice points of the cube (Section 1's exact
   predicates; QM_EINVAL otherwise).  out holds 4 doubles per tuple. */
int qm_test_geometry(int32_t op, int32_t n, const double* in, double param, double* out);

/* Message of the last failure on this thread ("" if none). */
const char* qm_last_error(void);

/* Library version string. */
const char* qm_version(void);

#ifdef __cplusplus
}
#endif

#endif
