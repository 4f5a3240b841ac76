/*
 * FP64 CPU oracle for the energy-efficient PD-NOMA H-CRAN allocator of
 * "Cross-Layer Energy Efficient Resource Allocation in PD-NOMA based H-CRANs:
 * Implementation via GPU" (Mokdad, Azmi, Mokari, Moltafet, Ghaffari-Miab).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, double-precision
 * statement of what the GPU allocator computes.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or constant with the
 * GPU library: every type below is declared here and nowhere else.
 *
 * Method (paper sections):
 *   Sec. II-A   SIC-ordered SINR, rates, power model, energy efficiency E=R/P.
 *   Sec. II-B   M/G/1 delay target -> minimum rate Psi (constraint C9/C13).
 *   Sec. III/IV Dinkelbach: E^{i+1} = R(p^i)/P(p^i), stop at R - E P <= tol.
 *   Sec. IV-A   SCALE lower bound alpha*log2(z)+beta <= log2(1+z), change of
 *               variable p = exp(p_hat), DC treatment of the SIC constraint
 *               C14, Lagrangian closed-form powers (elastic and streaming
 *               closed forms) and subgradient multiplier updates (Alg. 1).
 * The binary RRH/subcarrier constraints (C1/C2/C5/C6) are enforced exactly by
 * selection from the per-triple Lagrangian maximum (the limit of the C10/C11
 * relaxation as its slack goes to zero).
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t M, N, K, l;          /* RRHs (0 = HPN), subcarriers, users, users per (m,n) */
  const float* gain;           /* [M][N][K] Gamma, k fastest (promoted to double) */
  const uint8_t* user_type;    /* [K] 0 elastic, 1 streaming */
  const double* arrival_bps;   /* [K] lambda_k * zbar (bits/s), streaming only */
  const double* delay_s;       /* [K] T_k (s), streaming only */
  const double* pmax_w;        /* [M] */
  const double* eta;           /* [M] amplifier factor */
  const double* pmask_w;       /* [M] spectral mask, NULL -> pmax/N */
  const double* weight;        /* [M][K], NULL -> 1 */
  double noise_w;              /* sigma per subcarrier (W) */
  double bw_hz;                /* B_n */
  double packet_bits;          /* zbar */
  double p_fiber_hpn, p_fiber_lpn, p_circuit_hpn, p_circuit_lpn;
} orc_problem;

typedef struct {
  int32_t max_dinkelbach;        /* cap on Dinkelbach steps */
  int32_t sweeps_per_dinkelbach; /* cap (or exact count) of dual sweeps per step */
  int32_t refit_period;          /* refit alpha/beta every this many sweeps (<=0: never) */
  int32_t fixed_count;           /* 1: exactly sweeps_per_dinkelbach sweeps */
  double tol_dinkelbach;         /* stop when F_i <= tol * R_i */
  double tol_dual;               /* stop the dual loop when max|dp|/pmask and every projected
                                    multiplier subgradient are below tol */
  double step0;                  /* subgradient step delta_v = step0/sqrt(1+v) */
  double tie_rel;                /* relative margin below which a decision is a near-tie */
  int32_t stall_sweeps;          /* end the dual loop after this many sweeps without a
                                    better state (<=0: never; not with fixed_count) */
  double qos_down;               /* lower clip of the relative C13 violation in the
                                    zeta' step (the upper clip is 1) */
} orc_params;

typedef struct {
  const double* p0;    /* [M][N][K] initial powers or NULL */
  const double* xi0;   /* [M] or NULL */
  const double* zeta0; /* [K] or NULL */
} orc_warm;

enum {
  ORC_NOT_CONVERGED = 1u,      /* Dinkelbach stopped at max_dinkelbach */
  ORC_QOS_INFEASIBLE = 2u,     /* C13: a streaming user below (1 - 1e-6) Psi */
  ORC_NEAR_TIE = 4u,           /* some decision had a relative margin <= tie_rel */
  ORC_NONFINITE = 8u,
  ORC_SIC_INFEASIBLE = 16u,    /* C14: a co-scheduled pair with margin above 1e-9 */
  ORC_BUDGET_INFEASIBLE = 64u  /* C12: an RRH above (1 + 1e-6) of its budget */
};

typedef struct {
  int32_t* sel;         /* [M][N][l] users in SIC decoding order, -1 empty */
  double* slot_power;   /* [M][N][l] */
  int32_t* rrh_of_user; /* [K] RRH whose slots hold the user in sel, -1 unserved */
  double* xi;           /* [M] */
  double* zeta;         /* [K] (0 for elastic users) */
  double* zeta_sic;     /* [M][N][l(l-1)/2], pair (a,b) of decoding positions a<b */
  double* user_rate;    /* [K] r_k at exit */
  int32_t* tie_mn;      /* [M][N] or NULL: near-tie decisions of each (m,n) over the solve
                           (decoding order, insertion position, selection order, C14
                           compatibility and margin, H > 0 boundary, power floor) */
  int32_t* tie_user;    /* [K] or NULL: near-tie association and C13-threshold decisions */
  double ee, rate_sum, power_sum;
  double viol_qos, viol_budget, viol_sic; /* violations of C13, C12, C14 at exit */
  int32_t dinkelbach_iters, sweeps;
  uint32_t status_flags;
  int64_t near_ties;
  double min_margin;
  int32_t first_tie_sweep;
  /* optional per-Dinkelbach-step traces, length >= max_dinkelbach, or NULL */
  double* trace_E;
  double* trace_F;
  double* trace_R;
  double* trace_P;
  int32_t* trace_sweeps;
} orc_result;

/* Full solve.  Returns 0, or a negative errno-style code for invalid input. */
int orc_solve(const orc_problem* prob, const orc_params* prm, const orc_warm* warm,
              orc_result* res);

/* Step-level access for property tests. */
typedef struct orc_state orc_state;
orc_state* orc_state_create(const orc_problem* prob, const orc_params* prm,
                            const orc_warm* warm);
void orc_state_destroy(orc_state* st);
void orc_state_set_E(orc_state* st, double E);
void orc_state_reset_scale(orc_state* st);
/* One Jacobi dual sweep at the current E.  Returns the larger of max|dp|/pmask
 * and the largest multiplier step divided by the sweep's step size (its
 * scale factor included: the projected subgradient), or +inf when the sweep
 * moved any user to another RRH. */
double orc_state_sweep(orc_state* st, int32_t v, int32_t refit);
/* Evaluate the current state: true sum rate R, power P, SCALE surrogate rate
 * R_hat (with the current alpha/beta), per-user rates. */
void orc_state_eval(orc_state* st, double* R, double* P, double* R_hat, double* user_rate);
void orc_state_export(orc_state* st, orc_result* res);
/* Raw slot state [M][N][l] in storage order (user or -1, power), and the
 * multipliers; set replaces powers only (selection unchanged). */
void orc_state_get_slots(orc_state* st, int32_t* sel, double* power, double* xi, double* zeta,
                         double* zeta_sic_pairs);
void orc_state_set_powers(orc_state* st, const double* power);
/* Replace multipliers (any may be NULL); zs in the storage slot-pair layout. */
void orc_state_set_multipliers(orc_state* st, const double* xi, const double* zeta,
                               const double* zs);
/* Per-triple Lagrangian maximum H [M][N][K] computed by the last sweep. */
void orc_state_get_H(orc_state* st, double* H);
/* Dissolves the co-scheduled pairs that break C14 at the state, as a solve
 * does before it returns (see repair_subcarrier in oracle.c). */
void orc_state_repair_sic(orc_state* st);

/* Minimum-rate requirement Psi (bits/s/Hz) of a streaming user (Sec. II-B). */
double orc_min_rate(double arrival_bps, double delay_s, double packet_bits, double bw_hz);
/* SCALE coefficients at expansion point z0 (Sec. IV-A). */
void orc_scale_coeffs(double z0, double* alpha, double* beta);
/* Relative SIC margin of a co-scheduled pair (strong s by raw gain, weak w). */
double orc_sic_margin(double g_s, double g_w, double ici_s, double ici_w, double sigma);
/* OpenMP threads of the loops over subcarriers (n < 1: unchanged); returns
 * the previous setting. */
int orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
