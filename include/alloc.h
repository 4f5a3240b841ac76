/*
 * alloc.h -- C ABI of the MI355X energy-efficiency resource allocator for
 * PD-NOMA heterogeneous cloud RANs.
 *
 * The operation is the suboptimal solver of "Cross-Layer Energy Efficient
 * Resource Allocation in PD-NOMA based H-CRANs: Implementation via GPU":
 * maximise E = R/P (Sec. II-A; R the weighted sum rate of elastic users, P the
 * fibre, circuit and amplifier power) subject to at most l users per RRH and
 * subcarrier (C1/C2), the RRH power budget (C3/C12), the spectral mask (C4),
 * one RRH per user (C5/C6), the streaming users' minimum rate derived from
 * their M/G/1 delay target (C7 -> C9/C13, Sec. II-B) and SIC decodability
 * (C8/C14).  It runs the Dinkelbach iteration (Sec. III-IV) around Jacobi
 * sweeps of the SCALE-approximated Lagrangian dual (Sec. IV-A, Alg. 1):
 * SIC-ordered SINRs, SCALE refit, closed-form elastic/streaming powers,
 * selection of users and RRHs from the per-triple Lagrangian maximum, and
 * subgradient steps on the multipliers xi' (C12), zeta' (C13), zeta~' (C14).
 *
 * Conventions
 *  - Index sets: m in [0,M) RRHs (0 = HPN), n in [0,N) subcarriers,
 *    k in [0,K) users.  Three-index arrays are [M][N][K], k fastest.
 *  - All pointers are owned by the caller; the library never frees them.
 *    A context owns its device workspace and releases it in
 *    alloc_ctx_destroy.
 *  - Arithmetic is IEEE double precision on the device; gains are read as
 *    the given float32 values.
 *  - Return codes: 0 success; negative = error, outputs untouched:
 *      ALLOC_EINVAL  bad sizes, l < 1 or l > K, non-positive or non-finite
 *                    gain, budget or noise, streaming user with arrival
 *                    rate or delay target <= 0, NULL required pointer;
 *      ALLOC_ETOOBIG the problem exceeds a kernel limit (see below);
 *      ALLOC_ENOMEM  device allocation failed;
 *      ALLOC_EDEVICE a HIP runtime call failed;
 *      ALLOC_EFILE   (network files only) a file could not be read or written.
 *    Non-fatal conditions are reported in alloc_result.status_flags.
 *  - Limits: M <= 32, l <= 4, K <= 1024, M*K <= 4608 (one subcarrier's gain
 *    slab and its state must fit one workgroup's LDS).
 *  - Threading: one context per stream; calls on one context must not
 *    overlap.
 */
#ifndef ALLOC_H
#define ALLOC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ALLOC_API __attribute__((visibility("default")))

#define ALLOC_OK 0
#define ALLOC_EINVAL (-22)
#define ALLOC_ENOMEM (-12)
#define ALLOC_EDEVICE (-5)
#define ALLOC_ETOOBIG (-27)
#define ALLOC_EFILE (-2) /* a file could not be read or written, or has the wrong contents */

/* alloc_params.flags */
#define ALLOC_GAIN_ON_DEVICE 1u /* problem.gain is a device pointer */
#define ALLOC_OUT_ON_DEVICE 2u  /* array outputs of alloc_result are device pointers */
#define ALLOC_WARM_ON_DEVICE 4u /* alloc_warm arrays are device pointers */

/* alloc_result.status_flags */
#define ALLOC_NOT_CONVERGED 1u  /* Dinkelbach stopped at max_dinkelbach */
#define ALLOC_QOS_INFEASIBLE 2u /* C13: a streaming user ends below (1-1e-6) of its minimum rate */
#define ALLOC_NEAR_TIE 4u       /* with tie_rel > 0: some discrete decision was within tie_rel
                                   of going the other way (see alloc_params.tie_rel) */
#define ALLOC_NONFINITE 8u      /* a non-finite rate or power appeared */
#define ALLOC_SIC_INFEASIBLE 16u /* C14: a co-scheduled pair ends with SIC margin above 1e-9 */
#define ALLOC_BUDGET_INFEASIBLE 64u /* C12: an RRH ends above (1+1e-6) of its power budget */
#define ALLOC_GROUP_TIMEOUT 32u /* batched solver: the workgroups sharing this drop did not
                                   meet within 20 s (never expected: the persistent grid
                                   stays resident); the result is not valid */

typedef struct alloc_ctx alloc_ctx;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL = the
 * null stream).  Returns 0 and sets *out, or a negative code.
 * alloc_ctx_destroy while batches (alloc_batch) or networks (alloc_mlp) made
 * on the context are alive only closes it: those keep working, direct calls
 * on the context return ALLOC_EINVAL, and it is freed when the last of them
 * is destroyed. */
ALLOC_API int alloc_ctx_create(int device, void* hip_stream, alloc_ctx** out);
ALLOC_API void alloc_ctx_destroy(alloc_ctx* ctx);

/* One drop (Table I symbols). */
typedef struct {
  int32_t M, N, K, l;
  const float* gain;          /* [M][N][K] Gamma = |h|^2 (host or device, see flags) */
  const uint8_t* user_type;   /* [K] host: 0 elastic, 1 streaming */
  const double* arrival_bps;  /* [K] host: lambda_k * zbar (bits/s), streaming users */
  const double* delay_s;      /* [K] host: delay target T_k (s), streaming users */
  const double* pmax_w;       /* [M] host: RRH budget p_m^max (W) */
  const double* eta;          /* [M] host: amplifier factor eta_m */
  const double* pmask_w;      /* [M] host: spectral mask per RRH, NULL -> pmax/N */
  const double* weight;       /* [M][K] host: priority weight w_{m,k}, NULL -> 1 */
  double noise_w;             /* noise power per subcarrier sigma (W) */
  double bw_hz;               /* subcarrier bandwidth B_n (Hz) */
  double packet_bits;         /* packet size zbar (bits) */
  double p_fiber_hpn, p_fiber_lpn, p_circuit_hpn, p_circuit_lpn; /* static power (W) */
} alloc_problem;

/* Solver schedule.  alloc_params_default fills the defaults shown. */
typedef struct {
  int32_t max_dinkelbach;        /* 20: cap on Dinkelbach steps */
  int32_t sweeps_per_dinkelbach; /* 200: dual sweeps per step (cap, or exact count) */
  int32_t refit_period;          /* 1: SCALE refit every this many sweeps (<=0 never) */
  int32_t fixed_count;           /* 1: run exactly sweeps_per_dinkelbach sweeps */
  int32_t stall_sweeps;          /* 30: with fixed_count = 0, the dual loop also ends
                                    after this many sweeps without a better state (a
                                    violation of C12-C14 lower by more than 1e-6
                                    relative counts as better; <= 0: never) */
  double tol_dinkelbach;         /* 1e-6: stop when the returned state meets C12 and C13
                                    and |R - E P| <= tol * R; also the relative gain of
                                    R - E P that counts as progress of the dual loop */
  double tol_dual;               /* 1e-7: dual loop stops when max|dp|/pmask and every
                                    projected multiplier subgradient are below tol and
                                    no association changed (fixed_count = 0) */
  double step0;                  /* 0.1: subgradient step step0/sqrt(1+v) */
  double qos_down;               /* 0.2: the relative C13 violation (Psi - r_hat)/Psi of
                                    the zeta' step is clipped to [-qos_down, 1] */
  uint32_t flags;                /* ALLOC_GAIN_ON_DEVICE | ALLOC_OUT_ON_DEVICE */
  int32_t max_groups;            /* 0: cap on the workgroups of the solve grid
                                    (0 = one per compute unit, <= N, and one per
                                    two subcarriers when two subcarriers' triples
                                    fit one round of a workgroup's threads) */
  int32_t tile;                  /* 0: cap on the subcarriers a workgroup processes
                                    together (0 = as many as its LDS holds); its
                                    subcarriers are split into the fewest tiles
                                    within the cap, of equal size */
  int32_t lds_kb;                /* 0: batched solver only: requested LDS per workgroup
                                    in KiB (0 = a whole compute unit's); smaller shares
                                    let several workgroups share a compute unit.  Raised
                                    to what the batch's largest drop needs for a
                                    one-subcarrier tile. */
  int32_t block;                 /* 0: batched solver only: threads per workgroup,
                                    256, 512 or 1024 (0 = 512) */
  int32_t wave;                  /* 0: batched solver only, drops solved by one
                                    workgroup: 1..16 = each 64-lane wave runs its own
                                    subcarriers, this many at a time, with no
                                    workgroup barrier inside a pass (a drop whose
                                    wave tiles do not fit the LDS share keeps
                                    workgroup tiles); 0 = workgroup tiles.  With
                                    lds_kb = 0 the share is what the wave tiles need. */
  int32_t group_triples;         /* 0: batched solver only: a drop of more than this many
                                    (RRH, subcarrier, user) triples is solved by about
                                    triples/group_triples workgroups together (at most
                                    one per subcarrier and the resident number); 0 = a
                                    drop above 1.5 times the average triples per
                                    resident workgroup, by about triples/average */
  double tie_rel;                /* 0: when positive, count the discrete decisions of the
                                    solve whose relative margin is at most tie_rel (a
                                    different summation order could have taken them the
                                    other way): the SIC decoding order of two users of an
                                    (m,n), and where a candidate would enter it (relative
                                    difference of their normalised gains),
                                    a candidate among the first l of its RRH's selection
                                    order and the next one (relative difference of the
                                    per-triple Lagrangian maxima H), and a user's best and
                                    second-best RRH (relative difference of the sums of H);
                                    the count is alloc_result.near_ties and a positive count
                                    sets ALLOC_NEAR_TIE.  0: not counted (no cost) */
  int32_t warm_max_dinkelbach;   /* 0: the network's solves (alloc_solve_mlp,
                                    alloc_solve_batch_mlp) only: when positive and below
                                    max_dinkelbach, the warm-started attempt runs at most
                                    this many Dinkelbach steps, and one that has not met
                                    the stopping test within them falls back to the cold
                                    solve too (which runs max_dinkelbach); 0: the warm
                                    attempt runs max_dinkelbach steps */
} alloc_params;

ALLOC_API void alloc_params_default(alloc_params* p);

/* Optional warm start: any pointer may be NULL (double; host, or device with
 * ALLOC_WARM_ON_DEVICE).  With p0 the initial allocation is built from it and
 * is Dinkelbach's p^0 (Sec. III), feasible or not: the first step evaluates
 * it without dual sweeps, E^1 = R(p^0)/P(p^0), and the sweeps start from it
 * (R - E P is strictly decreasing in E with its root at the optimum, Lemma 1
 * and Theorem 1, so the iteration converges from above the optimum too, and
 * the solve stops at |R - E P| <= tol R).  Users go to the RRH of largest total p0
 * (a user with no positive p0 keeps the cold-start RRH, the one of largest
 * sum over n of log2(1 + Gamma pmask/sigma)); each (m,n) takes the l users of
 * largest positive p0 among its users, at power min(p0, pmask).  Without p0
 * the cold start applies (those RRHs, the l strongest users of each (m,n),
 * power pmax/(N l)).  xi' starts at max(xi0, 0) (else 0), zeta' at
 * max(zeta0, 0) for streaming users (else 1). */
typedef struct {
  const double* p0;    /* [M][N][K] initial powers */
  const double* xi0;   /* [M] */
  const double* zeta0; /* [K] */
} alloc_warm;

/* Outputs: arrays are caller-allocated (host, or device with
 * ALLOC_OUT_ON_DEVICE); any array pointer may be NULL to skip it.  Scalars
 * are always written to this host struct. */
typedef struct {
  int32_t* sel;        /* [M][N][l] users of (m,n) in SIC decoding order, -1 = empty */
  double* slot_power;  /* [M][N][l] power of those users (W) */
  float* power;        /* [M][N][K] dense powers (W) */
  int32_t* rrh_of_user; /* [K] the RRH whose slots hold the user in sel, -1 = unserved */
  double* xi;          /* [M] */
  double* zeta;        /* [K] (0 for elastic users) */
  double* zeta_sic;    /* [M][N][l(l-1)/2] C14 multiplier of decoding positions (a<b) */
  double* user_rate;   /* [K] r_k (bits/s/Hz, summed over subcarriers) */
  double ee;           /* R/P at the returned allocation (bits/s/Hz/W) */
  double rate_sum, power_sum;
  double viol_qos;     /* C13: sum over streaming users of (1-1e-6) - r_k/Psi_k where positive */
  double viol_budget;  /* C12: sum over RRHs of sum_p/pmax - (1+1e-6) where positive */
  double viol_sic;     /* C14: sum over co-scheduled pairs of margin - 1e-9 where positive */
  int32_t dinkelbach_iters, sweeps;
  uint32_t status_flags;
  int32_t near_ties;   /* near-tie decisions over the solve (alloc_params.tie_rel > 0), else 0 */
} alloc_result;

/* Solve one drop on the context's stream; returns when the results are
 * written (the call synchronises the stream). */
ALLOC_API int alloc_solve(alloc_ctx* ctx, const alloc_problem* prob, const alloc_params* prm,
                const alloc_warm* warm, alloc_result* res);

/* Solve B independent drops of any sizes in one persistent launch: each
 * workgroup takes the next drop from a work queue (largest M*N*K first) and
 * solves it completely (same method and schedule as alloc_solve, reductions
 * over the drop's subcarriers in the workgroup).  probs[b].gain are device
 * pointers with ALLOC_GAIN_ON_DEVICE (each drop its own [M][N][K] array),
 * host pointers otherwise.  results[b] arrays are host pointers (the
 * ALLOC_OUT_ON_DEVICE flag is rejected).  warms is NULL or [B] warm starts
 * (each with NULL members for a cold start).  Any error in any drop's
 * arguments rejects the whole call before work starts. */
ALLOC_API int alloc_solve_batch(alloc_ctx* ctx, int32_t B, const alloc_problem* probs,
                                const alloc_params* prm, const alloc_warm* warms,
                                alloc_result* results);

/* A resident batch: the drops' inputs, state and outputs stay on the device
 * and the batched solve (work-queue reset and the persistent kernel, no host
 * copies) is captured once into a HIP graph that every run replays.  Cold
 * starts only (warms are not taken); results as for alloc_solve_batch.
 * Device gain pointers (ALLOC_GAIN_ON_DEVICE) must stay valid for the life of
 * the batch; host gains are copied in at creation. */
typedef struct alloc_batch alloc_batch;
ALLOC_API int alloc_batch_create(alloc_ctx* ctx, int32_t B, const alloc_problem* probs,
                                 const alloc_params* prm, alloc_batch** out);
/* Replays the captured solve on the context's stream and waits for it. */
ALLOC_API int alloc_batch_run(alloc_batch* batch);
/* Results of the last run (host arrays as in alloc_solve_batch). */
ALLOC_API int alloc_batch_results(alloc_batch* batch, alloc_result* results);
/* Duration of the last run's graph in ms (HIP events on the context's stream). */
ALLOC_API double alloc_batch_last_ms(alloc_batch* batch);
ALLOC_API void alloc_batch_destroy(alloc_batch* batch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * alloc_solve of one cold-started drop that calls no hipMalloc, hipFree or
 * other allocating routine.  Its workspace (the drop's copied inputs, solver
 * state, partials and outputs before they are copied out) is a fixed device
 * array of alloc_noalloc_max_bytes() bytes (64 MiB) that the library holds on
 * every device it runs on until the process ends; a drop whose workspace
 * does not fit (with device gains, the 17 x 1024 x 256 configuration fits)
 * returns ALLOC_ETOOBIG before any work.  Same arguments, method, results
 * and errors as alloc_solve otherwise (no warm start).  Every call on one
 * device shares that array: calls that overlap on one device, from any
 * context or stream, race and must be serialised by the caller. */
ALLOC_API int alloc_solve_noalloc(alloc_ctx* ctx, const alloc_problem* prob, const alloc_params* prm,
                                  alloc_result* res);
ALLOC_API size_t alloc_noalloc_max_bytes(void);

ALLOC_API const char* alloc_strerror(int code);

/* Kernel timing for measurement: when enabled, alloc_solve records HIP events
 * on the context's stream around the persistent solve kernel, and
 * alloc_ctx_last_kernel_ms returns that kernel's duration in milliseconds for
 * the last call (-1 if timing is off or no solve ran). */
ALLOC_API int alloc_ctx_set_timing(alloc_ctx* ctx, int enable);
ALLOC_API double alloc_ctx_last_kernel_ms(alloc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
