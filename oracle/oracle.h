/*
 * CPU oracle for VRP-RPD makespan evaluation — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded C that states what the GPU path must compute.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or helper with the HIP
 * library; the two are compared on the same seeded inputs.
 *
 * Problem statement and timing model: Section 3 (problem formulation) and the
 * MILP of Section 3.1, Eq. (1)-(23).  Decoder: Section 4.4.2, Algorithm 2.
 * Genetic operators: Section 4.4.3.  ALNS: Section 4.2, Algorithm 1.
 */
#ifndef VRPRPD_ORACLE_H
#define VRPRPD_ORACLE_H
#include <stdint.h>

#define ORC_BAD_COVER 1u
#define ORC_LOAD 2u
#define ORC_RES 4u
#define ORC_DEADLOCK 8u
#define ORC_BAD_KEY 16u
#define ORC_BAD_TUPLE 32u

#define ORC_MIN_PRELOAD 0
#define ORC_FULL_START 1

typedef struct {
    int32_t n, m, k, R, load_model;
    const int32_t* d; /* (n+1)*(n+1) row-major travel times */
    const int32_t* p; /* n+1 processing times, p[0] = 0 */
} orc_inst;

/* Sweep evaluator (definition).  ops: L codes (c<<1 | isPickup) grouped by
 * vehicle; rt_end: m cumulative route ends.  op_time (nullable, L entries)
 * receives each op's time: the drop time for D, the pickup (departure) time
 * for P.  Returns status bits; *makespan = INT32_MAX when BAD_COVER or
 * DEADLOCK. */
uint32_t orc_eval(const orc_inst* I, int allow_partial, const uint16_t* ops,
                  const uint16_t* rt_end, int32_t* makespan, int64_t* op_time);

/* Independent second evaluator of the timing part only: builds the operation
 * graph explicitly and runs Kahn's topological order with a longest-path
 * pass.  Returns 0 or ORC_DEADLOCK (a cycle); cover must already hold. */
uint32_t orc_eval_dag(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end,
                      int32_t* makespan, int64_t* op_time);

void orc_eval_batch(const orc_inst* I, int allow_partial, int64_t B, const int64_t* op_off,
                    const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end,
                    int32_t* makespan, uint32_t* status);

typedef struct { uint16_t c; uint8_t vD, vP; uint16_t pD, pP; } orc_tuple;

/* Insertion scan over one base (partial) solution: each tuple's exact
 * makespan and status, and per segment the three smallest keys
 * (makespan << 32 | tuple index) among feasible tuples (INT64_MAX if fewer). */
void orc_insert_scan(const orc_inst* I, const uint16_t* base_ops, const uint16_t* base_rt,
                     int64_t T, const orc_tuple* tuples, int32_t S, const int64_t* seg_off,
                     int32_t* mk_out, uint32_t* st_out, int64_t* seg_top3);

/* Multi-pass decoder (Algorithm 2).  prio/hint: 2n keys each, op o = 2(c-1)+isP;
 * hint may be NULL.  Writes fitness, makespan, unscheduled count; ops_out (2n)
 * and rt_end_out (m) if non-NULL.  Returns status (0 or ORC_BAD_KEY). */
uint32_t orc_decode(const orc_inst* I, const float* prio, const float* hint,
                    int64_t* fitness, int32_t* makespan, int32_t* unscheduled,
                    uint16_t* ops_out, uint16_t* rt_end_out);
/* The same with flags: ORC_DECODE_HINT_FIRST gives the op to the hint
 * vehicle whenever it can take it (SelectVehicle decides otherwise). */
#define ORC_DECODE_HINT_FIRST 1
uint32_t orc_decode_ex(const orc_inst* I, const float* prio, const float* hint,
                       int64_t* fitness, int32_t* makespan, int32_t* unscheduled,
                       uint16_t* ops_out, uint16_t* rt_end_out, int32_t flags);

/* Philox4x32-10 (Salmon et al., SC'11). */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* One BRKGA generation (Section 4.4.3). */
void orc_brkga_evolve(int32_t Np, int32_t genes, const float* prio, const float* hint,
                      const int64_t* fitness, int32_t n_elite, int32_t n_mutant,
                      uint32_t rho_thr24, uint64_t seed, uint32_t generation,
                      float* prio_out, float* hint_out, int32_t* rank_out);

/* ALNS parameters (Table 2 defaults in oracle/__init__.py). */
typedef struct {
    double T0, alpha, reheat, gate;
    int32_t stag_limit, tau;
    double r;
    int32_t sigma1, sigma2, sigma3;
    double w_min;
    int32_t q_min, q_max;      /* 0: from n (Section 4.2.2) */
    int32_t tuple_budget;      /* tuples per iteration; 0: every slot pair */
    int32_t import_interval;   /* 0: never */
    uint32_t op_mask;          /* destroy ops bits 0-5, repair ops bits 8-11 */
    int32_t ls_repos_interval; /* pickup repositioning every this many iterations; 0: never */
    int32_t ls_reloc_interval; /* cross-agent relocation every this many iterations; 0: never */
    int32_t ls_budget;         /* tuples per local-search pass (> 0) */
} orc_alns_params;

/* The scalars Algorithm 1 keeps per chain: current and best makespan,
 * temperature and its initial value, operator weights (6 destroy, 4 repair),
 * scores and attempts of the current period, and the stagnation counter. */
typedef struct {
    int32_t z, zb;
    double T, T_init;
    double wD[6], wR[4];
    int64_t sD[6], sR[4];
    int32_t aD[6], aR[4];
    int32_t stag;
} orc_alns_chain;

/* Algorithm 1 after the repair of iteration it (0-based): attempts,
 * acceptance with the uniform u for the annealing test, scores, cooling,
 * stagnation and reheat, weights every tau iterations.  Returns 0 rejected,
 * 1 improving, 2 new best, 3 accepted by annealing. */
int32_t orc_alns_update(const orc_alns_params* P, orc_alns_chain* c, int32_t di, int32_t ri, int32_t repaired,
                        int32_t zn, double u, int64_t it);
/* Insertion candidates of customer c against a partial solution (ranked). */
int32_t orc_alns_enumerate(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end, int32_t c, int32_t KD,
                           int32_t KP, orc_tuple* out);
/* One repair of a partial solution; returns 1, or 0 if a customer could not
 * be inserted. */
int32_t orc_alns_repair(const orc_inst* I, int32_t op, const uint16_t* ops, const uint16_t* rt_end, const int32_t* rem,
                        int32_t nrem, int32_t KD, int32_t KP, uint16_t* out_ops, uint16_t* out_rt, int32_t* z,
                        int32_t* order);
void orc_alns_budget_split(int32_t budget, int32_t nrem, int32_t* KD, int32_t* KP);
double orc_det_exp(double x);
void orc_alns_qrange(int n, int* q_min, int* q_max);
int32_t orc_alns_run(const orc_inst* I, const orc_alns_params* P, int32_t chains, int64_t iterations,
                     uint64_t seed, const uint16_t* init_ops, const uint16_t* init_rt, uint16_t* best_ops,
                     uint16_t* best_rt, int32_t* best_mk, int64_t* trace);
/* The same with the chains numbered chain0, chain0 + 1, ... in the draws. */
int32_t orc_alns_run_from(const orc_inst* I, const orc_alns_params* P, int32_t chains, int64_t iterations,
                          uint64_t seed, const uint16_t* init_ops, const uint16_t* init_rt, uint16_t* best_ops,
                          uint16_t* best_rt, int32_t* best_mk, int64_t* trace, uint32_t chain0);
/* The same, also writing each chain's final current makespan (cur_mk
 * [chains], nullable) and its final temperature and operator weights (fstate
 * [chains][1 + 6 + 4] = T, w_D, w_R; nullable). */
int32_t orc_alns_run_ex(const orc_inst* I, const orc_alns_params* P, int32_t chains, int64_t iterations,
                        uint64_t seed, const uint16_t* init_ops, const uint16_t* init_rt, uint16_t* best_ops,
                        uint16_t* best_rt, int32_t* best_mk, int64_t* trace, uint32_t chain0, int32_t* cur_mk,
                        double* fstate);
/* One destroy operator on a complete feasible solution, as iteration `it` of
 * chain `chain` applies it, candidate `cand` of a learned proposal (draw
 * counters 16 + 4096 cand + i).  Returns the number of removed customers
 * written to rem, or -1 if the solution is infeasible. */
int32_t orc_alns_destroy(const orc_inst* I, int32_t op, const uint16_t* ops, const uint16_t* rt_end, int32_t q,
                         int32_t q_min, uint64_t seed, uint32_t it, uint32_t chain, int32_t cand, int32_t* rem);
/* Periodic local search (Section 4.2.6) on a complete feasible solution: kind
 * 0 pickup repositioning, 1 cross-agent relocation, up to `passes` passes of
 * `budget` tuples.  Returns the number of improving passes (-1: infeasible). */
int32_t orc_alns_local_search(const orc_inst* I, int32_t kind, int32_t budget, int32_t passes, const uint16_t* ops,
                              const uint16_t* rt_end, uint16_t* out_ops, uint16_t* out_rt, int32_t* z);

/* Warm-start population from one solution (Section 4.4.4). */
void orc_brkga_warm_start(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end,
                          int32_t Np, int32_t n_warm, int32_t n_variants, uint64_t seed,
                          float* prio_out, float* hint_out);
/* The same from n_src solutions (source s at ops + s op_stride, rt_end +
 * s rt_stride) with n_var[s] variants each. */
void orc_brkga_warm_start_multi(const orc_inst* I, int32_t n_src, const uint16_t* ops, int64_t op_stride,
                                const uint16_t* rt_end, int64_t rt_stride, const int32_t* n_var, int32_t Np,
                                int32_t n_warm, uint64_t seed, float* prio_out, float* hint_out);

/* Construction heuristics (initial solution of Section 4.2, phases 1-3;
 * warm-start seeds of Section 4.4.4): heuristic 0 sweep + balance + nearest
 * neighbour per vehicle, 1 nearest neighbour, 2 load balanced, 3 shortest
 * processing time.  Writes ops (2n) and rt_end (m), the placement order to
 * seq_v / seq_o (nullable); returns the number of ops placed. */
int32_t orc_construct(const orc_inst* I, int32_t heuristic, uint16_t* ops, uint16_t* rt_end, int32_t* seq_v,
                      int32_t* seq_o);
int32_t orc_cons_vehicles(const orc_inst* I);
void orc_cons_angle_order(const orc_inst* I, int32_t* order);
int32_t orc_cons_sectors(const orc_inst* I, int32_t* sector0, int32_t* sector);

/* Coordination statistics of a solution (Section 5.2): customers served
 * cross-vehicle and customers interleaved.  Returns 0, or -1 when the cover
 * is incomplete or the schedule deadlocks. */
int32_t orc_solution_stats(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end, int32_t* cross,
                           int32_t* interleaved);
#endif
