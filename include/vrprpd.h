/*
 * vrprpd.h — C-ABI of the MI355X (gfx950) VRP-RPD evaluation library.
 *
 * Problem (Section 3): a depot (node 0), customers 1..n, m vehicles that each
 * carry at most k identical resources.  Every customer needs a drop (a vehicle
 * deploys a resource), p_c time units of autonomous processing, and a pickup
 * (some vehicle, possibly another one, retrieves the resource).  Travel times
 * d[i][j] are integers.  The objective is the makespan: the time the last
 * vehicle is back at the depot (Eq. 21-23).
 *
 * Conventions shared by every entry point
 *  - Return value: VRPRPD_OK (0) or a negative error code.  The message of the
 *    last error on the calling thread is available from vrprpd_last_error().
 *  - Infeasibility is data, not an error: each evaluated candidate gets status
 *    bits (VRPRPD_ST_*), status 0 meaning feasible.
 *  - Buffers named "device" are caller-owned device memory (for instance torch
 *    tensors).  "host" buffers are read before the call returns.  The library
 *    keeps no pointer to a caller buffer after a call returns.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).  Every
 *    compute call is asynchronous on it; a fault inside a kernel surfaces at the
 *    caller's next synchronisation.  Calls that allocate (the *_create
 *    functions) synchronise the device.
 *  - All times are int32.  vrprpd_set_create refuses (VRPRPD_ERANGE) an
 *    instance on which some schedule could exceed INT32_MAX - 1:
 *    (2n + 1) * max d + sum p must stay below 2^31 - 1.
 *  - A candidate is a list of per-vehicle operation sequences.  An operation is
 *    the uint16 code (c << 1) | isPickup, c in [1, n].  The ops of a candidate
 *    are stored vehicle after vehicle; rt_end[v] is the cumulative end of
 *    vehicle v's sequence (so rt_end[m-1] is the candidate's op count).
 *    This is the tour representation of Section 4.3 (a list of (customer, op)
 *    per vehicle).
 *  - Handles are not thread-safe: one host thread at a time per handle.
 */
#ifndef VRPRPD_H
#define VRPRPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define VRPRPD_OK 0
#define VRPRPD_EINVAL (-1) /* bad argument (null pointer, size out of range) */
#define VRPRPD_ERANGE (-2) /* an instance whose times could overflow int32 */
#define VRPRPD_ENOMEM (-3) /* device allocation failed */
#define VRPRPD_EHIP (-4)   /* a HIP API call or kernel launch failed */

/* ---- per-candidate status bits --------------------------------------------- */
#define VRPRPD_ST_BAD_COVER 1u  /* Eq. (1) violated: missing/duplicate op, bad customer id or route ends */
#define VRPRPD_ST_LOAD 2u       /* Eq. (13)-(18): a vehicle's load leaves [0, k] */
#define VRPRPD_ST_RES 4u        /* the fleet needs more than R resources */
#define VRPRPD_ST_DEADLOCK 8u   /* pickups wait on each other in a cycle: no schedule exists */
#define VRPRPD_ST_BAD_KEY 16u   /* a random key outside [0, 1) or NaN */
#define VRPRPD_ST_BAD_TUPLE 32u /* an insertion tuple that does not fit its base solution */

/* ---- load models ------------------------------------------------------------
 * VRPRPD_MIN_PRELOAD: each vehicle leaves the depot with the least load its
 *   sequence needs (L_v = max over prefixes of drops - pickups); its load must
 *   stay within [0, k] and the preloads together within R.
 * VRPRPD_FULL_START: the MILP as printed (Eq. 13, q_0 = k): every vehicle
 *   leaves with k resources; the fleet needs m*k <= R. */
#define VRPRPD_MIN_PRELOAD 0
#define VRPRPD_FULL_START 1

/* ---- eval flags ------------------------------------------------------------- */
#define VRPRPD_ALLOW_PARTIAL 1 /* customers may be absent (neither op present) */

typedef struct vrprpd_set vrprpd_set;
typedef struct vrprpd_mlp vrprpd_mlp;

typedef struct {
    int32_t n;          /* customers, 1 <= n <= 10000 (per-candidate state lives in LDS) */
    int32_t m;          /* vehicles, 1 <= m <= 64 */
    int32_t k;          /* vehicle capacity, k >= 1 */
    int32_t R;          /* resources available to the fleet, R >= 0 */
    int32_t load_model; /* VRPRPD_MIN_PRELOAD or VRPRPD_FULL_START */
    const int32_t* dist; /* host, (n+1)*(n+1) row-major travel times >= 0, d[i][i] = 0 */
    const int32_t* proc; /* host, n+1 processing times >= 0, proc[0] = 0 */
} vrprpd_instance_desc;

const char* vrprpd_last_error(void);

/* Instance set: copies num_inst instances to the current device, packing the
 * travel times as uint16 when every entry fits (else int32).  Synchronous.
 * Errors: EINVAL (sizes, negative entries, nonzero diagonal or proc[0]),
 * ERANGE (see above), ENOMEM, EHIP.  *out is NULL on error. */
int vrprpd_set_create(vrprpd_set** out, int32_t num_inst, const vrprpd_instance_desc* desc);
int vrprpd_set_destroy(vrprpd_set* set);
/* Largest n and m over the set, and whether travel times are packed to 16 bits. */
int vrprpd_set_info(const vrprpd_set* set, int32_t* num_inst, int32_t* n_max, int32_t* m_max,
                    int32_t* dist16);

/*
 * vrprpd_eval — exact makespan of B candidates (Section 3, Eq. 1-23).
 *
 * For each candidate b:
 *   1. cover (Eq. 1): every op code names a customer in [1, n(inst)]; each
 *      customer has at most one drop and one pickup, a drop iff a pickup, and
 *      (without VRPRPD_ALLOW_PARTIAL) both; route ends are non-decreasing and
 *      at most 2n.  Else status = BAD_COVER, makespan = INT32_MAX.
 *   2. load (Eq. 13-18) under the instance's load model -> LOAD, RES bits.
 *   3. timing (Eq. 7-12): the earliest-start schedule of the given sequences.
 *      Vehicles start at time 0 at the depot; a drop happens on arrival; a
 *      pickup departs at max(arrival, drop time + p_c) whichever vehicle made
 *      the drop (Eq. 9).  If the pickups' waits form a cycle: DEADLOCK and
 *      makespan = INT32_MAX.
 *   4. makespan (Eq. 21-22): the latest return time; an empty route adds 0.
 *
 * Arguments (all device pointers unless said otherwise):
 *   set       instance set
 *   B         number of candidates, B >= 0
 *   inst      [B] int32 instance index per candidate, or NULL: all use instance 0;
 *             an index outside [0, num_inst) gives status BAD_COVER
 *   op_off    [B] int64 offset of candidate b's first op in ops, or NULL: b * 2 * n(0)
 *   ops       op codes (uint16)
 *   rt_off    [B] int64 offset of candidate b's route ends in rt_end, or NULL: b * m(0)
 *   rt_end    m(inst) cumulative route ends per candidate (uint16)
 *   flags     0 or VRPRPD_ALLOW_PARTIAL
 *   makespan  [B] int32 out
 *   status    [B] uint32 out
 * op_off/rt_off NULL with inst non-NULL requires every instance to share n, m.
 * The launch shape (kernel form, candidates per wave, ops per sweep step) is
 * the one vrprpd_autotune_eval kept or vrprpd_eval_set_shape pinned for this
 * (n, m), else a default (see vrprpd_autotune_eval); every shape gives the
 * same results bit for bit.
 * Errors: EINVAL (NULL set or buffers with B > 0, B < 0, bad flags, or a
 * shape whose LDS does not fit: n above about 6,700 for the staged form and
 * 10,200 for the live-leg form with 16-lane groups), EHIP.
 */
int vrprpd_eval(const vrprpd_set* set, int64_t B, const int32_t* inst, const int64_t* op_off,
                const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end, int32_t flags,
                int32_t* makespan, uint32_t* status, void* stream);

/* Autotuner of vrprpd_eval's launch shape: form x candidates per 64-lane
 * wave (one wave per block; with 16-lane groups 2, 3 or 4, with 32-lane
 * groups 1 or 2, with 64 lanes 1 -- fewer candidates per wave leave LDS room
 * for more resident waves) x ops per lane per sweep step (2 or 4).  The two
 * forms compute the same thing: "staged" gathers every travel time of a
 * candidate into LDS before its timing sweep, "live legs" keeps only the op
 * codes in LDS (packed 12 bits each below n = 2048: 7.0 instead of 12.3 KB per
 * candidate at n = 1000, so more candidates stay resident)
 * and reads each travel time from the matrix as the sweep takes the op.
 * Without tuning, vrprpd_eval uses live legs when the staged layout of a
 * candidate exceeds 8 KB (about n > 650 with 16-bit travel times).  Runs
 * every shape on the caller's batch `reps` times, checks that each gives the
 * default shape's makespans and statuses bit for bit (EHIP otherwise), and
 * keeps the fastest in the set for later vrprpd_eval launches of the same
 * (n, m) -- n, m of the instance, or n_max, m_max when inst != NULL.
 * Arguments as vrprpd_eval; outputs the chosen candidates per wave and step
 * and, if ms_out != NULL, the mean milliseconds of twelve shapes at index
 * 6 * form (0 staged, 1 live legs) + 2 * i + (step == 4), option i of
 * candidates per wave in the order listed, -1 where an option does not exist
 * or its LDS does not fit.  Synchronous; not concurrent with other calls on
 * the same set. */
int vrprpd_autotune_eval(vrprpd_set* set, int64_t B, const int32_t* inst, const int64_t* op_off,
                         const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end, int32_t flags,
                         int32_t* makespan, uint32_t* status, int32_t reps, int32_t* ng_out, int32_t* step_out,
                         float* ms_out, void* stream);

/* Pins vrprpd_eval's launch shape for launches of (n, m) -- n, m of the
 * instance, or n_max, m_max when vrprpd_eval gets an instance array -- as
 * vrprpd_autotune_eval would keep it: ng candidates per wave (0: the
 * default for this form; else one of the options listed above), step 2 or 4
 * ops per lane per sweep step, live 0 (staged) or 1 (live legs).  Lets a
 * caller reuse a shape tuned in an earlier process or compare the forms.
 * Not concurrent with other calls on the same set.  Errors: EINVAL (NULL
 * set, n or m < 1, an option that does not exist or whose LDS does not fit). */
int vrprpd_eval_set_shape(vrprpd_set* set, int32_t n, int32_t m, int32_t ng, int32_t step, int32_t live);

/* Rate of random reads of one instance's travel-time matrix (measurement
 * for vrprpd_eval's secondary bound: staging a candidate of 2n ops makes
 * 2n + m such reads, one per leg, at entries spread over the whole matrix).
 * blocks x 256 threads each make per_thread reads (a multiple of 16, 16 in
 * flight) at hash-chosen entries of instance `inst`; sink [blocks] int32
 * device out (block sums).  One warm-up launch, then one timed launch
 * between HIP events on the stream; *ms_out (host) receives its
 * milliseconds.  Synchronous.  Errors: EINVAL, EHIP. */
int vrprpd_gather_rate(const vrprpd_set* set, int32_t inst, int32_t blocks, int32_t per_thread, int32_t* sink,
                       float* ms_out, void* stream);

/* One way to put a removed customer back into a partial solution
 * (Section 4.2.3, repair operators): its drop into route vD before index pD
 * (pD = len(vD) appends), its pickup into route vP before index pP, where pP
 * counts positions after the drop was inserted (so on one vehicle
 * pD + 1 <= pP <= len + 1, and pP = pD + 1 means the vehicle waits at c). */
typedef struct {
    uint16_t c;
    uint8_t vD;
    uint8_t vP;
    uint16_t pD;
    uint16_t pP;
} vrprpd_tuple;

/*
 * vrprpd_insert_scan — exact makespan of insertion candidates (Section 4.2.3).
 *
 * The repair operators price inserting a removed customer's drop and pickup
 * at every (vehicle, position) pair, including different vehicles for the two
 * ops, by the resulting makespan, and keep the best options (greedy: the
 * cheapest; regret-k: the k cheapest).  Here every tuple is evaluated exactly
 * (cover, load and the full timing of vrprpd_eval under ALLOW_PARTIAL) on its
 * segment's base solution with the tuple applied, and each segment reports
 * its three smallest keys (makespan << 32 | tuple index) over tuples with
 * status 0.
 *
 * A tuple is BAD_TUPLE (makespan INT32_MAX) when c is outside [1, n], c
 * already has an op in the base, a vehicle index is >= m, or a position is
 * outside the ranges above.  A base that breaks cover rules (even allowing
 * absent customers) makes every valid tuple on it BAD_COVER.
 *
 * Arguments (device pointers unless said otherwise):
 *   num_bases     >= 1 base (partial) solutions
 *   base_inst     [num_bases] instance index, or NULL: all instance 0
 *   base_op_off   [num_bases] offset of each base's ops in base_ops, or NULL: b * 2n(0)
 *   base_ops      op codes of the bases
 *   base_rt_off   [num_bases] offset of each base's route ends, or NULL: b * m(0)
 *   base_rt_end   cumulative route ends of the bases
 *   num_seg       S >= 0 segments; segment s covers tuples [seg_off[s], seg_off[s+1])
 *   seg_off       [S+1] int64, non-decreasing, seg_off[0] = 0
 *   seg_base      [S] base index of each segment, or NULL: all base 0
 *   tuples        [seg_off[S]] tuples
 *   mk_out        [seg_off[S]] int32 makespans, or NULL
 *   st_out        [seg_off[S]] uint32 status bits, or NULL
 *   seg_top3      [S][3] int64 out, ascending; INT64_MAX where fewer than 3 feasible tuples
 *   blocks_per_seg  (host) workgroups sharing each segment's tuples, 0 or 1
 *                 for one; more spreads long segments over the GPU (each
 *                 workgroup stages the base once)
 * Errors: EINVAL, EHIP.  seg_base / base_inst values out of range make the
 * segment's tuples BAD_TUPLE.
 */
int vrprpd_insert_scan(const vrprpd_set* set, int32_t num_bases, const int32_t* base_inst,
                       const int64_t* base_op_off, const uint16_t* base_ops, const int64_t* base_rt_off,
                       const uint16_t* base_rt_end, int32_t num_seg, const int64_t* seg_off,
                       const int32_t* seg_base, const vrprpd_tuple* tuples, int32_t* mk_out,
                       uint32_t* st_out, int64_t* seg_top3, int32_t blocks_per_seg, void* stream);

/*
 * brkga_decode_eval — multi-pass decoder (Section 4.4.2, Algorithm 2) and the
 * penalised fitness of the schedule (Section 4.4.2, infeasibility handling).
 *
 * Chromosome b holds 2n priority keys pi_o and (optionally) 2n vehicle hints
 * alpha_o for the ops o = 2(c-1) + isPickup (Section 4.4.1).  The decoder
 * visits the ops by ascending priority (equal keys: lower op index first) in
 * passes; an op is scheduled at its turn when feasible:
 *   drop:   some vehicle can hand out a resource (FULL_START: load > 0;
 *           MIN_PRELOAD: load > 0, or it may take one more from the depot
 *           within k and the fleet total R);
 *   pickup: its drop is scheduled and some vehicle has room (load < k); the
 *           vehicle waits for drop time + p_c (Eq. 9).
 * SelectVehicle picks the feasible vehicle with the earliest completion time
 * of the op (arrival for a drop, max(arrival, ready) for a pickup); ties go to
 * the first vehicle counting cyclically from floor(m * alpha_o) (fp32
 * product), or from vehicle 0 without hints.  With flags =
 * VRPRPD_DECODE_HINT_FIRST the hint vehicle floor(m * alpha_o) takes the op
 * whenever it can (Section 4.4.1: the hint is the vehicle, overridden only to
 * keep the schedule feasible; Section 4.4.4: the encoded ALNS solution then
 * decodes close to itself), and SelectVehicle decides only when it cannot.
 * Passes repeat until every op is scheduled or a pass schedules nothing (at
 * most 2n passes).
 * makespan = latest return of a used vehicle; unscheduled = 2n - #scheduled;
 * fitness = makespan + 10^6 * unscheduled (lambda of the paper).
 * Keys must lie in [0, 1) (-0.0 counts as 0.0): otherwise status BAD_KEY,
 * fitness INT64_MAX, makespan INT32_MAX, unscheduled 2n.  Under FULL_START
 * with m*k > R the status carries RES (the fleet as loaded needs more than R).
 *
 * Arguments (device pointers):
 *   B            chromosomes; inst [B] instance index or NULL (all instance 0)
 *   prio, hint   [B][key_stride] fp32 keys (hint may be NULL); key_stride >= 2n
 *   flags        (host) 0, or VRPRPD_DECODE_HINT_FIRST
 *   fitness      [B] int64 out; makespan, unscheduled [B] int32 out; status [B] out
 *   ops_out      [B][2 n_max] uint16 out, the decoded sequences route after
 *                route (only the first rt_end_out[m-1] entries are written), or NULL
 *   rt_end_out   [B][m_max] uint16 out, cumulative route ends, or NULL
 * Limits: 2n <= 8192.  Errors: EINVAL, EHIP.
 */
#define VRPRPD_DECODE_HINT_FIRST 1
int brkga_decode_eval(const vrprpd_set* set, int64_t B, const int32_t* inst, const float* prio,
                      const float* hint, int64_t key_stride, int32_t flags, int64_t* fitness, int32_t* makespan,
                      int32_t* unscheduled, uint32_t* status, uint16_t* ops_out, uint16_t* rt_end_out,
                      void* stream);

/*
 * brkga_decode_eval_noalloc — brkga_decode_eval for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * brkga_decode_eval, bit for bit; it calls no hipMalloc / hipMallocAsync /
 * hipFree.  Its workspace (op orders, key flags and, with ops_out, schedule
 * logs) is a fixed device array inside the library of
 * brkga_decode_noalloc_max_bytes() = 32 MiB, one per GPU, held from the
 * library's load until the process ends; its address is looked up on the
 * first call on each device.  A batch whose workspace would exceed it is
 * rejected with EINVAL (message in vrprpd_last_error()); the workspace of B
 * chromosomes is about 2 * 2^ceil(log2(2n)) * B bytes, three times that with
 * ops_out (at n = 1000: up to 8,190 chromosomes, 2,730 with ops_out).
 * Every call on one GPU uses the same array and leaves its contents behind
 * (each call writes what it reads before reading it): calls that overlap on
 * one GPU (two streams, two host threads) race and must be serialised by the
 * caller.
 */
int brkga_decode_eval_noalloc(const vrprpd_set* set, int64_t B, const int32_t* inst, const float* prio,
                              const float* hint, int64_t key_stride, int32_t flags, int64_t* fitness,
                              int32_t* makespan, int32_t* unscheduled, uint32_t* status, uint16_t* ops_out,
                              uint16_t* rt_end_out, void* stream);
/* Size in bytes of brkga_decode_eval_noalloc's fixed workspace. */
int64_t brkga_decode_noalloc_max_bytes(void);

/*
 * brkga_evolve — one BRKGA generation (Section 4.4.3): rank by (fitness,
 * index); children [0, n_elite) copy the ranked elites; [n_elite,
 * n_elite + n_mutant) get fresh U(0,1) genes; the rest take each gene from a
 * uniformly chosen elite parent with probability rho_e, else from a
 * uniformly chosen non-elite parent.  Genes are the `genes` priorities and,
 * when hint != NULL, as many hints.  Draws: Philox4x32-10 keyed by seed,
 * counter (gene / 4, child, generation, stream tag); uniform fp32 =
 * (w >> 8) * 2^-24, Bernoulli = (w >> 8) < floor(rho_e * 2^24).
 *   prio/hint      [Np][key_stride] in; prio_out/hint_out same shape, out (no aliasing)
 *   fitness        [Np] int64 in
 *   rank_out       [Np] int32 out: index of the individual of each rank
 * Errors: EINVAL (sizes: n_elite + n_mutant <= Np, and n_elite >= 1 and a
 * non-elite individual when crossover children exist), EHIP.
 */
int brkga_evolve(int32_t Np, int32_t genes, int64_t key_stride, const float* prio, const float* hint,
                 const int64_t* fitness, int32_t n_elite, int32_t n_mutant, double rho_e, uint64_t seed,
                 uint32_t generation, float* prio_out, float* hint_out, int32_t* rank_out, void* stream);

/*
 * brkga_warm_start — initial population seeded from one solution (Section
 * 4.4.4).  Encoding: the op at 1-based position r of a route of L_v ops gets
 * priority (r-1)/L_v (fp64 quotient rounded to fp32) and hint (v + 1/2)/m;
 * ops absent from the solution get 0.  Slots [0, n_warm) cycle through
 * n_variants variants (slot s takes variant s mod n_variants; variant 0 is
 * the encoding, variant t > 0 adds U(-0.03, 0.03) to every gene in fp64 and
 * clamps into [0, 1)); slots [n_warm, Np) are fresh U(0,1) individuals.
 * Draws: Philox4x32-10, counter (gene / 4, variant or slot, 0, tag).
 *   ops, rt_end   the solution of instance `inst` (device)
 *   prio_out, hint_out   [Np][key_stride] fp32 out
 */
int brkga_warm_start(const vrprpd_set* set, int32_t inst, const uint16_t* ops, const uint16_t* rt_end,
                     int32_t Np, int32_t n_warm, int32_t n_variants, uint64_t seed, int64_t key_stride,
                     float* prio_out, float* hint_out, void* stream);

/*
 * brkga_warm_start_multi — the warm start from several solutions (Section
 * 4.4.4: the ALNS incumbent plus construction seeds, see vrprpd_construct).
 * Source s (device ops + s op_stride, rt_end + s rt_stride) is encoded as
 * above and contributes n_var[s] variants (host array; variant 0 the
 * encoding itself, variant t > 0 perturbed with draws at counter (gene / 4,
 * t, s, 'WARM')); slots [0, n_warm) cycle through all variants in source
 * order, the other slots are fresh U(0,1) individuals as above.  With one
 * source this equals brkga_warm_start.  1 <= n_src <= 16; n_var[s] >= 0 (all
 * zero: every slot fresh).  Allocates a stream-ordered workspace of
 * 8 n_src n bytes.  Errors: EINVAL, EHIP.
 */
int brkga_warm_start_multi(const vrprpd_set* set, int32_t inst, int32_t n_src, const uint16_t* ops,
                           int64_t op_stride, const uint16_t* rt_end, int64_t rt_stride, const int32_t* n_var,
                           int32_t Np, int32_t n_warm, uint64_t seed, int64_t key_stride, float* prio_out,
                           float* hint_out, void* stream);

/* ---- construction heuristics ------------------------------------------------
 * vrprpd_construct — one solution per instance from a construction heuristic,
 * one block per instance (B instances: inst[b], device, or b when NULL).
 * VRPRPD_CONS_SWEEP is the initial solution of Section 4.2 ("Initial Solution
 * Construction"), its first three phases; the fourth (refinement) is
 * alns_refine.  NN, LB and SPT are the construction seeds of the BRKGA warm
 * start (Section 4.4.4).  The paper names the phases and their aims; the
 * library's readings, which a CPU implementation of the same readings
 * reproduces exactly (integer arithmetic throughout):
 *  - pseudo-angle: the depot is the origin, the customer r farthest from it
 *    (lowest index on ties) gives angle 0; with a_c = d(0,c), b = d(0,r) and
 *    X_c = a_c^2 + b^2 - d(r,c)^2 (the law of cosines: the coordinate along
 *    the axis times 2b), the second reference r2 maximises 4 a^2 b^2 - X^2
 *    (farthest from the axis, lowest index on ties) and fixes the positive
 *    side: sign(y_c) = sign(2 b^2 (a_c^2 + a_r2^2 - d(r2,c)^2) - X_c X_r2).
 *    Customers are ordered by (half-plane, cosine) with the cosine taken as
 *    trunc(2^30 X_c / (2 a_c b)) clamped to [-2^30, 2^30], ties by index, all
 *    on distances shifted right until the largest is below 2^14;
 *  - sectors: m' = m under FULL_START, max(1, min(m, R)) under MIN_PRELOAD;
 *    the order is cut into m' runs, the first n mod m' one longer;
 *  - balancing (workload w_c = 2 d(0,c) + p_c): while 10 (W_max - W_min) >=
 *    W_max (heaviest / lightest sector, lowest index on ties), the customer
 *    of the heaviest sector with 0 < w_c < W_max - W_min closest to half the
 *    gap (ties by index) moves to the lightest; stops when none qualifies
 *    or after n m' moves;
 *  - routes: each vehicle serves its sector alone with at most cap_v
 *    resources out (k under FULL_START; under MIN_PRELOAD R split over the
 *    m' vehicles, the first R mod m' one more, capped at k), each step the op
 *    of earliest completion (a drop at arrival, a pickup at max(arrival,
 *    drop time + p_c)), ties by op index 2(c-1) + isPickup;
 *  - LB: whole customers, heaviest w_c first, each to the vehicle of least
 *    assigned workload (ties by index), then routes as above;
 *  - NN, SPT: one dispatch loop over all vehicles with the decoder's load
 *    rules (Algorithm 2); NN: the vehicle free earliest among those with a
 *    feasible op (ties by index) takes its nearest op (least d, ties by op);
 *    SPT: drops only in ascending (p_c, c) order, the (vehicle, op) pair of
 *    earliest completion among that drop and every pending pickup (ties by
 *    op, then vehicle).
 * Every op is placed unless no resource may move at all (R = 0 under
 * MIN_PRELOAD): then the routes stay empty.
 *   ops      [B][op_stride] out, op_stride >= 2 n_max; rt_end [B][rt_stride]
 *            out, rt_stride >= m_max (route ends of the instance's m vehicles)
 * A row whose instance index is out of range gets all-empty routes.
 * Allocates a stream-ordered workspace (about 40 n_max bytes per instance).
 * Errors: EINVAL, EHIP.
 */
/*
 * vrprpd_solution_stats — the coordination measures of Section 5.2 per
 * solution: cross[b] = customers whose drop and pickup are on different
 * vehicles; interleaved[b] = customers for which the drop vehicle does
 * another operation between the drop and the pickup (same vehicle: an
 * operation between the two in its route; another vehicle: the drop
 * vehicle's next operation, if its time -- arrival for a drop, departure for
 * a pickup, in the earliest-start schedule -- is before the pickup's time).
 * Both -1 when the cover is incomplete (every customer needs exactly one drop
 * and one pickup), the route ends are invalid, the instance index is out of
 * range, or the waits form a cycle.  Arguments as vrprpd_eval (inst, op_off,
 * rt_off NULL-able the same way); cross, interleaved [B] int32 out.
 * Allocates a stream-ordered workspace (about 24 n_max bytes for each of at
 * most 2048 blocks).  Errors: EINVAL, EHIP.
 */
int vrprpd_solution_stats(const vrprpd_set* set, int64_t B, const int32_t* inst, const int64_t* op_off,
                          const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end, int32_t* cross,
                          int32_t* interleaved, void* stream);

#define VRPRPD_CONS_SWEEP 0
#define VRPRPD_CONS_NN 1
#define VRPRPD_CONS_LB 2
#define VRPRPD_CONS_SPT 3
int vrprpd_construct(const vrprpd_set* set, int32_t B, const int32_t* inst, int32_t heuristic, int64_t op_stride,
                     uint16_t* ops, int64_t rt_stride, uint16_t* rt_end, void* stream);

/*
 * brkga_state — many instances' BRKGA populations evolved together (the
 * batched form): each generation decodes and evaluates every individual of
 * every population in one brkga_decode_eval launch, then ranks, keeps each
 * population's best and evolves every population in one launch each, all
 * captured once as a HIP graph per population buffer and replayed
 * (use_graph = 1) or launched directly (0, same results).  Population p (of
 * instance inst_ids[p]) is Np individuals of 2 n_p priorities and hints at
 * key_stride = 2 n_max, seeded pop_seed = seed + 0x9E3779B97F4A7C15 * p
 * (mod 2^64); generation g of population p equals brkga_evolve with that
 * seed and generation g.  The set's largest instance must be among
 * inst_ids.  prio0 / hint0 (device [n_inst * Np][2 n_max]) give the initial
 * populations, or NULL for U(0,1) genes (Philox, counter (gene / 4,
 * individual, 0, 'RAND'), key pop_seed).  decode_flags: the decoder's flags
 * (0 or VRPRPD_DECODE_HINT_FIRST, see brkga_decode_eval).
 */
typedef struct brkga_state brkga_state;
int brkga_state_create(brkga_state** out, const vrprpd_set* set, int32_t n_inst, const int32_t* inst_ids,
                       int32_t Np, int32_t n_elite, int32_t n_mutant, double rho_e, uint64_t seed,
                       int32_t decode_flags, const float* prio0, const float* hint0, void* stream);
int brkga_state_step(brkga_state* st, int32_t generations, int32_t use_graph, void* stream);
/* Generations done (host), best fitness per population so far (host
 * [n_inst], synchronises), the best chromosomes (device [n_inst][2 n_max])
 * and the current populations (device); any pointer may be NULL. */
int brkga_state_get(const brkga_state* st, int64_t* generations, int64_t* best_fitness, float* best_prio,
                    float* best_hint, float* prio, float* hint, void* stream);
int brkga_state_destroy(brkga_state* st);
/* Checkpoint of a BRKGA state: the populations to be decoded next, every
 * population's best chromosome and fitness so far and the generation counter.
 * buf (host, caller-owned) receives it; with buf = NULL only *bytes (host) is
 * set to the size it needs.  Waits for the stream, then copies (synchronous).
 * EINVAL if capacity is below that size. */
int brkga_state_save(const brkga_state* st, void* buf, int64_t capacity, int64_t* bytes, void* stream);
/* Restores a checkpoint into a state created on the same set and instances
 * with the same Np, elite and mutant counts, rho_e and seed (EINVAL
 * otherwise, or when bytes is not the checkpoint's size): generations run
 * after the load equal those the saved state would have run.  Synchronous. */
int brkga_state_load(brkga_state* st, const void* buf, int64_t bytes, void* stream);

/* ---- ALNS (Section 4.2) ----------------------------------------------------
 * alns_params: the hyper-parameters of Table 2 (Section 4.2.7) plus this
 * library's repair budget.  Defaults: T0 = 0.30, alpha = 0.9998, reheat =
 * 0.50, gate = 0.01, stag_limit = 2000, tau = 100, r = 0.1, sigma = (33, 9,
 * 13), w_min = 0.1, q_min = q_max = 0 (the rule of Section 4.2.2:
 * q_max = max(4, floor(0.05 n)), q_min = max(4, floor(q_max / 2))),
 * tuple_budget = 0 (every slot pair), import_interval = 1000,
 * op_mask = 0x0F3F (all six destroy and four repair operators),
 * ls_repos_interval = 200, ls_reloc_interval = 500, ls_budget = 16384.
 *
 * Periodic local search (Section 4.2.6), after the acceptance step of every
 * ls_repos_interval-th (pickup repositioning) and ls_reloc_interval-th
 * (cross-agent relocation) iteration, repositioning first; 0 turns one off.
 * Up to three passes each, on the chain's current solution, no acceptance
 * test: a pass takes the best strictly improving move.  Repositioning: every
 * pickup on a vehicle returning within 5% of the makespan (20 f_v >= 19 z)
 * may move to any pickup slot of any vehicle (after its drop on the drop's
 * vehicle); relocation: every customer with an op on the bottleneck vehicle
 * (latest return, lowest index on ties) may move both ops to one other
 * vehicle.  At most the first 256 candidates (route order) are tried per
 * pass.  Slots are ranked by detour as in the repair, T = max(1,
 * ls_budget / candidates) tuples per candidate (relocation: K_D =
 * max(1, floor(sqrt T)) drop slots x K_P = max(1, T / K_D) pickup slots);
 * ties between moves go to the earlier candidate (route order), then the
 * earlier tuple.  A new best resets the stagnation counter.  ls_budget must
 * be >= 1 when either interval is on.
 *
 * One iteration of a chain (Algorithm 1): roulette-select a destroy and a
 * repair operator by weight; draw q in [q_min, q_max]; destroy (random,
 * worst, Shaw, cluster, route, critical path); repair (greedy, regret-2,
 * regret-3, regret-m) with every candidate priced by the exact evaluator;
 * accept by simulated annealing; cool; reheat after stag_limit iterations
 * without a new best once T < gate * T_init; every tau iterations update the
 * weights.  The operators' readings of the paper (candidate slots ranked by
 * detour, the K_D / K_P budget split, regret over per-drop-vehicle options,
 * the rank weights 2^60 / r^6 of worst removal, the integer Shaw relatedness,
 * exp by a fixed Taylor evaluation, ...) are stated in the library's design
 * notes and followed exactly, so a CPU implementation of the same readings
 * reproduces every chain's trajectory.
 * Random draws: Philox4x32-10 keyed by seed, counter (a / 4, iteration,
 * chain_base + chain, 'ALNS'): a = 0 destroy roulette, 1 repair roulette,
 * 2 q, 8 annealing, 16.. destroy operator.  chain_base (default 0) shifts
 * the chains' ids in the draws: a state over one instance with chain_base =
 * k * chains_per_inst follows, chain for chain, the trajectories of the
 * k-th instance's chains in a state over several instances. */
typedef struct {
    double T0, alpha, reheat, gate;
    int32_t stag_limit, tau;
    double r;
    int32_t sigma1, sigma2, sigma3;
    double w_min;
    int32_t q_min, q_max;
    int32_t tuple_budget;
    int32_t import_interval;
    uint32_t op_mask;
    int32_t ls_repos_interval;
    int32_t ls_reloc_interval;
    int32_t ls_budget;
    int32_t chain_base;
} alns_params;

typedef struct alns_state alns_state;

/* chains_per_inst chains for each of n_inst instances (inst_ids, host), all
 * starting from that instance's initial solution: init_ops (device) holds
 * instance i's 2n ops at [i * 2 n_max), init_rt (device) its route ends at
 * [i * m_max), where n_max, m_max are the largest n, m among inst_ids.  The
 * initial solutions must be feasible (status 0).  Chain c = i *
 * chains_per_inst + j.  Synchronous; allocates device memory.
 * Errors: EINVAL, ENOMEM, EHIP. */
int alns_state_create(alns_state** out, const vrprpd_set* set, int32_t n_inst, const int32_t* inst_ids,
                      int32_t chains_per_inst, const alns_params* params, uint64_t seed,
                      const uint16_t* init_ops, const uint16_t* init_rt, void* stream);
/* Runs `iterations` more iterations of every chain (asynchronous on stream).
 * By default the launches of one iteration are captured once into a HIP
 * graph (on a stream of the state's own) and the graph is replayed per
 * iteration; the iteration number lives in device memory.  The capture is
 * redone after alns_set_trace, alns_set_learned or alns_record. */
int alns_step(alns_state* st, int32_t iterations, void* stream);
/*
 * alns_autotune — the launch shape of the insertion scans in the state's
 * repair rounds: tuples per workgroup 8, 16, 32 or 64 (fewer tuples per
 * workgroup spread each waiting customer's tuples over more workgroups).
 * Each shape runs one warm-up iteration (graph capture) and `iterations`
 * timed iterations from a checkpoint of the state (alns_state_save); the
 * state after the runs must be byte-identical for every shape (EHIP
 * otherwise: the shape never changes the search).  The fastest shape is kept
 * for this state and recorded in the set for later states with the same
 * (n_max, m_max, tuple_budget); the state is restored to its checkpoint, so
 * it continues as if the call had not been made.  tpb_out (host, nullable)
 * receives the chosen tuples per workgroup, ms_out (host, nullable, 4
 * floats) the milliseconds per iteration of the four shapes.  Synchronous;
 * not while recording (EINVAL).  Errors: EINVAL, EHIP.
 */
int alns_autotune(alns_state* s, int32_t iterations, int32_t* tpb_out, float* ms_out, void* stream);

/* enable = 0: launch every kernel of every iteration instead (same results). */
int alns_set_graph(alns_state* st, int32_t enable);
/* Records (candidate makespan, current z, best z, destroy | repair << 8 |
 * outcome << 16 | removed << 24) of every chain for the next `capacity`
 * iterations into trace [chains][capacity][4] int64 (device), or stops
 * recording (trace = NULL). */
int alns_set_trace(alns_state* st, int64_t* trace, int64_t capacity);
/* Best makespan (host out) and, if ops / rt_end are non-NULL, the best
 * solution (device out, 2 n_max ops and m_max route ends) of one chain, or of
 * the best chain when chain = -1.  Synchronises the stream. */
int alns_get_best(const alns_state* st, int32_t chain, int32_t* mk, uint16_t* ops, uint16_t* rt_end, void* stream);
/* Host copies of the iteration count, the number of exact evaluations done
 * so far (insertion tuples priced and removal gains), and every chain's
 * current and best makespan, temperature and operator weights ([chains][6],
 * [chains][4]); any pointer may be NULL.  Synchronises the device. */
int alns_get_state(const alns_state* st, int64_t* iterations, int64_t* evals, int32_t* z, int32_t* zb, double* T,
                   double* wD, double* wR);
int alns_state_destroy(alns_state* st);
/* Checkpoint of every chain's state in Algorithm 1 (Section 4.2): current
 * and best solutions and makespans, temperature and its initial value,
 * operator weights, the scores and attempts of the running weight period,
 * the stagnation counter, plus the evaluation count and the iteration
 * counter (the random draws are keyed by the iteration, so nothing else is
 * needed to continue).  buf (host, caller-owned) receives it; with buf = NULL
 * only *bytes (host) is set to the size it needs.  Waits for the stream, then
 * copies (synchronous).  Not included: the learned proposal's settings,
 * traces and records, which stay as the loading state has them.  EINVAL if
 * capacity is below that size. */
int alns_state_save(const alns_state* st, void* buf, int64_t capacity, int64_t* bytes, void* stream);
/* Restores a checkpoint into a state created on the same set with the same
 * instances, chains per instance, parameters and seed (EINVAL otherwise, or
 * when bytes is not the checkpoint's size).  k iterations, a save, a load
 * into a fresh state and k' more iterations give the same chains, bit for
 * bit, as k + k' iterations without the checkpoint.  Synchronous. */
int alns_state_load(alns_state* st, const void* buf, int64_t bytes, void* stream);
/* The last phase of the initial construction (Section 4.2, "Initial Solution
 * Construction": relocation and pickup reassignment until nothing improves),
 * before the first iteration: rounds of the periodic local searches
 * (repositioning, then relocation, up to three passes each, with the
 * state's ls_budget) on every chain's current solution; a chain stops after
 * a round that improved nothing, at most max_rounds rounds run.  Each chain's
 * best becomes the refined solution and its temperature T0 times the refined
 * makespan (the refined solution is the initial one).  rounds_out (host,
 * nullable): rounds run.  Synchronous (reads the stop flags back after each
 * round).  Errors: EINVAL (after alns_step, or ls_budget < 1), EHIP. */
int alns_refine(alns_state* st, int32_t max_rounds, int32_t* rounds_out, void* stream);

/* ---- ALNS with a learned destroy proposal ----------------------------------
 * (Section 7.4 names learned destroy operators as future work; this is the
 * library's form.)  Each iteration every chain builds K candidate removal
 * sets with the roulette-selected destroy operator, candidate j drawing its
 * random words at counters 16 + 4096 j + i (candidate 0 is the plain
 * operator's set).  The network (vrprpd_mlp_*) scores each customer of the
 * current solution S from 64 features; a set's score is the sum over its
 * customers, the predicted (z' - z) / z; the chain takes the lowest score
 * (ties to the lower index) -- or, with probability eps (Philox counter 3),
 * candidate 0.  Repair, acceptance and scoring are unchanged: the exact
 * evaluator prices every insertion and judges every makespan.
 *
 * Features of customer c in S (fp32, each one correctly rounded division of
 * two integers, stored as bfloat16 [C][n_max][64], row c - 1): with z the
 * makespan, dbar = max(1, floor(sum_i d[0][i] / n)), for c's drop D and
 * pickup P: vehicle v, 0-based position i, route length L, start time t,
 * arrival a, neighbours prev / next (depot 0 at the route ends), route finish
 * f, walk = drops - pickups up to the op, g = z - z(S without c):
 *  0 1, 1 d(0,c)/dbar, 2 p_c/dbar, 3 tD/z, 4 tP/z, 5 (tP-tD-p_c)/z,
 *  6 (tP-aP)/z, 7 [vD=vP], 8 iD/LD, 9 iP/LP, 10 fD/z, 11 fP/z, 12 [fD=z],
 *  13 [fP=z], 14 (d(prevD,c)+d(c,nextD)-d(prevD,nextD))/dbar, 15 the same
 *  for P, 16 d(prevD,c)/dbar, 17 d(c,nextD)/dbar, 18 d(prevP,c)/dbar,
 *  19 d(c,nextP)/dbar, 20 g/z, 21 walkD/k, 22 walkP/k, 23 LD m/(2n),
 *  24 LP m/(2n), 25 (iP-iD)/LD if vD=vP else 0, 26 nearest other node/dbar,
 *  27 (sum of the 4 nearest other nodes)/(4 dbar) (fewer others: all of
 *  them), 28 (z-fD)/z, 29 (z-fP)/z, 30 [g>0], 31 p_c/(tP-tD) (1 if tP=tD);
 *  32..63 = 0..31 times [fD=z or fP=z].
 *
 * mlp: not owned; NULL turns the proposal off (K = 1).  Its max_rows must be
 * >= chains x n_max.  EINVAL unless 1 <= K <= 64 and 0 <= eps <= 1. */
int alns_set_learned(alns_state* st, vrprpd_mlp* mlp, int32_t K, double eps, void* stream);
/* Starts recording one (features of the removed customers, (z' - z) / z)
 * set per chain per iteration, up to `capacity` sets (0: stop and free),
 * from the next iteration on; z' is the repaired candidate's makespan (a
 * failed repair records an empty set).  Synchronises the stream. */
int alns_record(alns_state* st, int64_t capacity, void* stream);
/* Sets recorded so far and the most customers a set can hold (q_max). */
int alns_record_info(const alns_state* st, int64_t* sets, int32_t* q_max);
/* A training batch of num_sets recorded sets drawn uniformly with
 * replacement (Philox, seed): x (device bf16 [num_sets * q_max][64]) gets
 * their rows back to back, seg_off (device int64 [num_sets + 1]) the row
 * offsets, target (device fp32 [num_sets]) the makespan changes. */
int alns_record_batch(const alns_state* st, int32_t num_sets, uint64_t seed, uint16_t* x, int64_t* seg_off,
                      float* target, void* stream);
/* Device copies of the last iteration's features ([C][n_max][64] bf16),
 * candidate sets ([C][K][q_max] and counts [C][K]) and choices ([C]); any
 * pointer may be NULL. */
int alns_get_learned(const alns_state* st, uint16_t* feat, int32_t* cand_rem, int32_t* cand_cnt, int32_t* chosen,
                     void* stream);

/* ---- Learned destroy proposal: the scorer network --------------------------
 * The paper names learned destroy operators as future work (Section 7.4) and
 * fixes no model.  This library's: per-customer features (VRPRPD_MLP_IN =
 * 64) -> 256 -> 256 -> 256 -> 1, ReLU after each hidden layer.  A removal
 * set's score is the sum of its customers' scores; training fits it to the
 * makespan change the set produced by mean squared error over sets.
 * Precision: bfloat16 GEMM operands (features, weights, hidden activations
 * and masked upstream gradients, rounded to nearest even) with fp32
 * accumulation on the matrix cores; biases, head, loss, gradients and the
 * master weights in fp32.
 * Flat parameter layout (fp32, VRPRPD_MLP_NUM_PARAMS values): W1[256][64],
 * b1[256], W2[256][256], b2[256], W3[256][256], b3[256], w4[256], b4[1]
 * (weights [out][in]).
 * The handle owns its parameters, momentum and all activations and
 * workspaces for up to max_rows rows (about 3.1 KB per row plus 150 KB per
 * 1024 rows); calls on one handle are ordered by the caller's stream and
 * must not overlap. */
#define VRPRPD_MLP_IN 64
#define VRPRPD_MLP_HIDDEN 256
#define VRPRPD_MLP_NUM_PARAMS 148481
/* params: host fp32 flat vector, or NULL for Glorot-uniform hidden weights
 * (Philox draws from seed), zero biases and a zero head (w4, b4).  Synchronous.  EINVAL unless 1 <=
 * max_rows <= 2^26; ENOMEM; EHIP. */
int vrprpd_mlp_create(vrprpd_mlp** out, int64_t max_rows, const float* params, uint64_t seed);
int vrprpd_mlp_destroy(vrprpd_mlp* mlp);
/* Device copies of the parameters and/or of the last backward's gradient
 * (either pointer may be NULL). */
int vrprpd_mlp_get_params(const vrprpd_mlp* mlp, float* params, float* grad, void* stream);
/* Replaces the parameters (device fp32 flat) and clears the momentum. */
int vrprpd_mlp_set_params(vrprpd_mlp* mlp, const float* params, void* stream);
/* Scores rows: x is device bf16 [rows][64] (16-byte aligned, kept by
 * reference until the next forward: backward reads it); y (device fp32
 * [rows]) may be NULL.  Hidden activations stay in the handle.  EINVAL if
 * rows > max_rows. */
int vrprpd_mlp_forward(vrprpd_mlp* mlp, int64_t rows, const uint16_t* x, float* y, void* stream);
/* Set scores of the last forward: set_score[s] = sum of the scores of rows
 * [seg_off[s], seg_off[s+1]) (device int64 offsets, non-decreasing, within
 * the rows). */
int vrprpd_mlp_set_scores(vrprpd_mlp* mlp, int32_t num_sets, const int64_t* seg_off, float* set_score, void* stream);
/* Loss of the last forward against target[s] (device fp32): stores each
 * set's squared error in sq_err (device, nullable; the loss is their mean)
 * and keeps dL/dscore per row for vrprpd_mlp_backward (zero for rows in no
 * set). */
int vrprpd_mlp_loss(vrprpd_mlp* mlp, int32_t num_sets, const int64_t* seg_off, const float* target, float* sq_err,
                    void* stream);
/* Gradient of the loss through the last forward, from dy (device fp32
 * [rows], dL/d(row score)) or, when dy is NULL, from vrprpd_mlp_loss.  The
 * result (flat, fp32) stays in the handle for vrprpd_mlp_sgd_step. */
int vrprpd_mlp_backward(vrprpd_mlp* mlp, const float* dy, void* stream);
/* Heavy-ball step: v = momentum v + grad; p = p - lr v (fp32), then the
 * bfloat16 copy is refreshed.  EINVAL unless lr >= 0, 0 <= momentum < 1. */
int vrprpd_mlp_sgd_step(vrprpd_mlp* mlp, float lr, float momentum, void* stream);
/* Device copy of a kept tensor of the last forward/backward, bf16
 * [rows][256]: layer 0..2 = hidden activations h1..h3, 3..4 = the two
 * masked-gradient buffers (after a backward: 3 holds dz1, 4 holds dz2). */
int vrprpd_mlp_hidden(const vrprpd_mlp* mlp, int32_t layer, uint16_t* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif
