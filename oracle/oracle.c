/*
 * FP64 CPU oracle of the PD-NOMA H-CRAN energy-efficiency allocator.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain loops in double precision,
 * one step of the method after another, in the order the paper gives them.
 * Parallelism is limited to an OpenMP loop over subcarriers for work that the
 * method defines per subcarrier; every sum across subcarriers is taken
 * afterwards, serially, in increasing subcarrier order.
 *
 * Notation (Table I): m RRH (0 = HPN), n subcarrier, k user, Gamma channel
 * gain, sigma noise, p power, A RRH association, rho subcarrier allocation
 * (held here as the list "sel" of at most l users per (m,n)), xi' (C12),
 * zeta' (C13), zeta~' (C14) Lagrange multipliers, alpha/beta SCALE
 * coefficients, E the Dinkelbach energy-efficiency parameter.
 *
 * Readings where the paper is silent or ambiguous (each listed with its
 * reason in the design notes):
 *  - decoding order on (m,n) is by normalised gain Gamma/(sigma+ICI),
 *    descending, ties to the lower user index; with it, C14 holds exactly
 *    when raw-gain order and decoding order agree;
 *  - interference prices use the full gradient over all victims, each victim
 *    weighted by mu = 1 (elastic) or zeta'_k (streaming);
 *  - C14 is used as the scale-free margin Omega/nu with
 *    nu = Gamma_w(sigma+ICI_s) + Gamma_s(sigma+ICI_w) taken at the state;
 *  - the binary constraints are met by selection: per (m,n) the users of
 *    RRH m with positive per-triple Lagrangian maximum H are taken in order
 *    of H, each only if every pair it forms with those taken before it meets
 *    C14 at the state's interference, up to l users; per user the RRH with
 *    the largest sum of H over subcarriers, applied from the next sweep;
 *  - subgradient step step0/sqrt(1+v); xi' scaled by N*l/(ln2*pmax_m);
 *    the relative C13 violation clipped to [-qos_down, 1] (a streaming
 *    user's rate jumps between zero and several times its minimum as it
 *    gains or loses a subcarrier, so zeta' falls more slowly than it rises);
 *  - closed-form powers below 1e-20 of the mask are set to zero;
 *  - the dual sweeps are not a descent method, so each Dinkelbach step
 *    returns the best state it visited: feasible for C12-C14 before
 *    infeasible, less C12/C13 violation first, then less C14 violation, then
 *    the larger R - E P (a replacement needs a relative gain of 1e-6); the
 *    dual loop also ends after stall_sweeps sweeps without a better state
 *    (a violation lower by more than 1e-6 relative is progress), and the
 *    next Dinkelbach step restarts from the best; the multipliers xi' and
 *    zeta' continue from the last sweep;
 *  - a warm start's allocation is Dinkelbach's p^0: E^1 = R(p^0)/P(p^0)
 *    whether or not it is feasible (F is strictly decreasing in E with its
 *    root at the optimum, Theorem 1 and Lemma 1, so the iteration converges
 *    from any E; from above the optimum F < 0 and E moves down), and it is
 *    the first step's starting state;
 *  - Dinkelbach's stop test is the root condition |F| <= tol R (F >= 0
 *    whenever E is at most the optimum) on a state that meets C12 and C13;
 *    C14 is enforced through its multiplier and the selection rule (SCA keeps
 *    C13 feasible, Prop. 2; nothing in the method guarantees C14), and the
 *    pairs that still break it when the solve ends are dissolved (see
 *    repair_subcarrier());
 *  - all sweeps are Jacobi: every quantity of a sweep is read from the state
 *    the sweep starts from.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))
#define LN2 0.69314718055994530942
#define MAXL 8
/* Powers below this fraction of the mask are set to exactly zero: decaying
 * closed-form powers would otherwise reach the subnormal range, where the
 * SINR underflows and the SCALE refit produces 0 * log2(0). */
#define POWER_FLOOR_REL 1e-20
/* Feasibility tolerances of an iterate: C13 r >= Psi (1 - QOS_TOL), C12
 * sum p <= pmax (1 + BUDGET_TOL), C14 margin <= SIC_TOL. */
#define QOS_TOL 1e-6
#define BUDGET_TOL 1e-6
#define SIC_TOL 1e-9

/* ------------------------------------------------------------------ basics */

/* log2(1+x) */
static double log2_1p(double x) { return log1p(x) / LN2; }

/* Sec. II-B, constraint C9: Psi = Psi_hat / B_n with
 * Psi_hat = 2 lambda zbar / ((2 + 2 lambda T) - sqrt((2 + 2 lambda T)^2 - 8 lambda T)).
 * With x = lambda T the discriminant is 4(1+x^2), so the denominator is
 * 2(1 - 1/(x + sqrt(1+x^2))), the cancellation-free form used here. */
ORC_API double orc_min_rate(double arrival_bps, double delay_s, double packet_bits,
                            double bw_hz) {
  const double lambda = arrival_bps / packet_bits; /* packets/s */
  const double x = lambda * delay_s;
  const double den = 1.0 - 1.0 / (x + sqrt(1.0 + x * x));
  return (lambda * packet_bits / den) / bw_hz;
}

/* Sec. IV-A, SCALE bound alpha log2 z + beta <= log2(1+z), tight at z0. */
ORC_API void orc_scale_coeffs(double z0, double* alpha, double* beta) {
  *alpha = z0 / (1.0 + z0);
  *beta = log2_1p(z0) - (*alpha) * log2(z0);
}

/* Eq. (SIC_linear) with sigma_k = sigma_k' = sigma: for raw-stronger s and
 * weaker w, Omega = Gamma_w sigma - Gamma_s sigma + Gamma_w ICI_s - Gamma_s ICI_w,
 * and C8/C14 ask Omega <= 0.  Returned divided by the positive scale
 * nu = Gamma_w (sigma + ICI_s) + Gamma_s (sigma + ICI_w). */
/* Threads of the OpenMP loops over subcarriers; returns the previous
 * setting.  n < 1 leaves it unchanged. */
ORC_API int orc_set_threads(int n) {
  const int prev = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return prev;
}

ORC_API double orc_sic_margin(double g_s, double g_w, double ici_s, double ici_w,
                              double sigma) {
  const double omega = g_w * sigma - g_s * sigma + g_w * ici_s - g_s * ici_w;
  const double nu = g_w * (sigma + ici_s) + g_s * (sigma + ici_w);
  return omega / nu;
}

/* ------------------------------------------------------------------- state */

struct orc_state {
  int M, N, K, L;
  double* G; /* [M][N][K] */
  int* elastic;
  double* psi;
  double *pmax, *eta, *pmask;
  double* w; /* [M][K] */
  double sigma, pstatic;
  orc_params prm;
  double E;
  int* A;                     /* [K] */
  int* sel;                   /* [M][N][L] user or -1, in selection-rank order */
  double *p, *al, *be;        /* [M][N][L] */
  double* zs;                 /* [M][N][L][L] multiplier of C14 per slot pair */
  double *xi, *zeta;          /* [M], [K] */
  double* H;                  /* [M][N][K] per-triple Lagrangian maximum */
  double *part_psum, *part_pel; /* [N][M] */
  double *part_r, *part_rh;   /* [N][K] */
  double* part_delta;         /* [N] */
  int64_t* part_ties;         /* [N] */
  double* part_margin;        /* [N] */
  int64_t ties;
  double min_margin;
  int first_tie;
  int sweeps_done;
  int assoc_changed; /* users whose RRH changed in the last sweep */
  int32_t* tie_mn;   /* [M][N] near-tie decisions of (m,n) over the solve */
  int32_t* tie_user; /* [K] near-tie association decisions of each user */
  double* part_sicv; /* [N] C14 violation at the state read by the sweep */
  int* part_moved;   /* [N] the sweep changed a selected set on the subcarrier */
  double* part_dres; /* [N] largest C14 multiplier step / delta_v on the subcarrier */
  int moved;         /* the last sweep changed a selected set or an association */
  /* evaluation of a state (the one the last sweep read, or orc_state_eval's):
   * rate R, power P, violations of C13 (Vq), C12 (Vp), C14 (Vs) */
  double ev_R, ev_P, ev_Vq, ev_Vp, ev_Vs;
};

#define IDX3(st, m, n, k) (((size_t)(m) * (st)->N + (n)) * (st)->K + (k))
#define SLOT(st, m, n, s) (((size_t)(m) * (st)->N + (n)) * (st)->L + (s))
#define PAIR(st, m, n, a, b) ((((size_t)(m) * (st)->N + (n)) * (st)->L + (a)) * (st)->L + (b))

static double mu_of(const orc_state* st, int k) { return st->elastic[k] ? 1.0 : st->zeta[k]; }

static void note_margin(double margin, double tie_rel, int64_t* ties, double* minm) {
  if (margin < *minm) *minm = margin;
  if (margin <= tie_rel) (*ties)++;
}

/* A near-tie of a decision of (m,n) on its subcarrier's thread. */
static void note_mn(orc_state* st, int m, int n, double margin, int64_t* ties, double* minm) {
  if (margin < *minm) *minm = margin;
  if (margin <= st->prm.tie_rel) {
    (*ties)++;
    st->tie_mn[(size_t)m * st->N + n]++;
  }
}

static int validate(const orc_problem* pb) {
  if (!pb || pb->M < 1 || pb->N < 1 || pb->K < 1 || pb->l < 1 || pb->l > MAXL ||
      pb->l > pb->K || pb->M > 64 || pb->K > 4096)
    return -22;
  if (!pb->gain || !pb->user_type || !pb->pmax_w || !pb->eta) return -22;
  if (!(pb->noise_w > 0) || !(pb->bw_hz > 0) || !(pb->packet_bits > 0)) return -22;
  const size_t n3 = (size_t)pb->M * pb->N * pb->K;
  for (size_t i = 0; i < n3; ++i)
    if (!(pb->gain[i] > 0.0f) || !isfinite(pb->gain[i])) return -22;
  for (int m = 0; m < pb->M; ++m) {
    if (!(pb->pmax_w[m] > 0) || !isfinite(pb->pmax_w[m]) || !(pb->eta[m] > 0)) return -22;
    if (pb->pmask_w && !(pb->pmask_w[m] > 0)) return -22;
  }
  for (int k = 0; k < pb->K; ++k) {
    if (pb->user_type[k] > 1) return -22;
    if (pb->user_type[k] == 1) {
      if (!pb->arrival_bps || !pb->delay_s) return -22;
      if (!(pb->arrival_bps[k] > 0) || !(pb->delay_s[k] > 0)) return -22;
    }
  }
  if (pb->weight)
    for (int i = 0; i < pb->M * pb->K; ++i)
      if (!(pb->weight[i] >= 0) || !isfinite(pb->weight[i])) return -22;
  return 0;
}

/* Top-l of users by key desc, ties to the lower user index. */
static void top_by_key(const double* key, const int* users, int cnt, int l, int* out,
                       int* nout) {
  int idx[4096];
  int c = cnt < 4096 ? cnt : 4096;
  for (int i = 0; i < c; ++i) idx[i] = i;
  /* insertion sort: fine for the short lists of one (m,n) */
  for (int i = 1; i < c; ++i) {
    int t = idx[i], j = i - 1;
    while (j >= 0 && (key[idx[j]] < key[t] ||
                      (key[idx[j]] == key[t] && users[idx[j]] > users[t]))) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = t;
  }
  *nout = c < l ? c : l;
  for (int i = 0; i < *nout; ++i) out[i] = idx[i];
}

/* Cold start (initial feasible point of the Dinkelbach iteration, Sec. IV):
 * max-SNR association, strongest l users per (m,n), equal split of pmax. */
static void cold_start(orc_state* st) {
  const int M = st->M, N = st->N, K = st->K, L = st->L;
  for (int k = 0; k < K; ++k) {
    int best = 0;
    double bestv = -1.0;
    for (int m = 0; m < M; ++m) {
      double s = 0.0;
      for (int n = 0; n < N; ++n) s += log2_1p(st->G[IDX3(st, m, n, k)] * st->pmask[m] / st->sigma);
      if (s > bestv) {
        bestv = s;
        best = m;
      }
    }
    st->A[k] = best;
  }
  for (int m = 0; m < M; ++m)
    for (int n = 0; n < N; ++n) {
      double key[4096];
      int users[4096], cnt = 0, pick[MAXL], np;
      for (int k = 0; k < K; ++k)
        if (st->A[k] == m) {
          key[cnt] = st->G[IDX3(st, m, n, k)];
          users[cnt++] = k;
        }
      top_by_key(key, users, cnt, L, pick, &np);
      for (int s = 0; s < L; ++s) {
        const size_t i = SLOT(st, m, n, s);
        st->sel[i] = (s < np) ? users[pick[s]] : -1;
        st->p[i] = (s < np) ? st->pmax[m] / ((double)N * L) : 0.0;
        st->al[i] = 1.0;
        st->be[i] = 0.0;
      }
    }
  for (int m = 0; m < M; ++m) st->xi[m] = 0.0;
  for (int k = 0; k < K; ++k) st->zeta[k] = st->elastic[k] ? 0.0 : 1.0;
  memset(st->zs, 0, sizeof(double) * (size_t)M * N * L * L);
}

/* Warm start: association by the largest total initial power, the l users of
 * largest positive initial power per (m,n), powers clipped to the mask. */
static void warm_start(orc_state* st, const orc_warm* wm) {
  const int M = st->M, N = st->N, K = st->K, L = st->L;
  if (wm->p0) {
    for (int k = 0; k < K; ++k) {
      int best = -1;
      double bestv = 0.0;
      for (int m = 0; m < M; ++m) {
        double s = 0.0;
        for (int n = 0; n < N; ++n) s += wm->p0[IDX3(st, m, n, k)];
        if (s > bestv) {
          bestv = s;
          best = m;
        }
      }
      if (best >= 0) st->A[k] = best; /* else keep the cold-start association */
    }
    for (int m = 0; m < M; ++m)
      for (int n = 0; n < N; ++n) {
        double key[4096];
        int users[4096], cnt = 0, pick[MAXL], np;
        for (int k = 0; k < K; ++k)
          if (st->A[k] == m && wm->p0[IDX3(st, m, n, k)] > 0.0) {
            key[cnt] = wm->p0[IDX3(st, m, n, k)];
            users[cnt++] = k;
          }
        top_by_key(key, users, cnt, L, pick, &np);
        for (int s = 0; s < L; ++s) {
          const size_t i = SLOT(st, m, n, s);
          st->sel[i] = (s < np) ? users[pick[s]] : -1;
          st->p[i] = (s < np) ? fmin(key[pick[s]], st->pmask[m]) : 0.0;
          st->al[i] = 1.0;
          st->be[i] = 0.0;
        }
      }
  }
  if (wm->xi0)
    for (int m = 0; m < M; ++m) st->xi[m] = fmax(wm->xi0[m], 0.0);
  if (wm->zeta0)
    for (int k = 0; k < K; ++k) st->zeta[k] = st->elastic[k] ? 0.0 : fmax(wm->zeta0[k], 0.0);
}

ORC_API orc_state* orc_state_create(const orc_problem* pb, const orc_params* prm,
                                    const orc_warm* warm) {
  if (validate(pb) != 0) return NULL;
  orc_state* st = (orc_state*)calloc(1, sizeof(orc_state));
  const int M = pb->M, N = pb->N, K = pb->K, L = pb->l;
  const size_t n3 = (size_t)M * N * K, ns = (size_t)M * N * L;
  st->M = M;
  st->N = N;
  st->K = K;
  st->L = L;
  st->prm = *prm;
  st->G = (double*)malloc(sizeof(double) * n3);
  for (size_t i = 0; i < n3; ++i) st->G[i] = (double)pb->gain[i];
  st->elastic = (int*)malloc(sizeof(int) * K);
  st->psi = (double*)malloc(sizeof(double) * K);
  for (int k = 0; k < K; ++k) {
    st->elastic[k] = pb->user_type[k] == 0;
    st->psi[k] = st->elastic[k] ? 0.0
                                : orc_min_rate(pb->arrival_bps[k], pb->delay_s[k],
                                               pb->packet_bits, pb->bw_hz);
  }
  st->pmax = (double*)malloc(sizeof(double) * M);
  st->eta = (double*)malloc(sizeof(double) * M);
  st->pmask = (double*)malloc(sizeof(double) * M);
  for (int m = 0; m < M; ++m) {
    st->pmax[m] = pb->pmax_w[m];
    st->eta[m] = pb->eta[m];
    st->pmask[m] = pb->pmask_w ? pb->pmask_w[m] : pb->pmax_w[m] / N; /* Sec. VIII */
  }
  st->w = (double*)malloc(sizeof(double) * M * K);
  for (int i = 0; i < M * K; ++i) st->w[i] = pb->weight ? pb->weight[i] : 1.0;
  st->sigma = pb->noise_w;
  /* Power model (Sec. II-A): P = P_f^H + M_f P_f^L + sum eta p + M_f P_c^L + P_c^H. */
  st->pstatic = pb->p_fiber_hpn + (M - 1) * pb->p_fiber_lpn + (M - 1) * pb->p_circuit_lpn +
                pb->p_circuit_hpn;
  st->E = 0.0;
  st->A = (int*)malloc(sizeof(int) * K);
  st->sel = (int*)malloc(sizeof(int) * ns);
  st->p = (double*)malloc(sizeof(double) * ns);
  st->al = (double*)malloc(sizeof(double) * ns);
  st->be = (double*)malloc(sizeof(double) * ns);
  st->zs = (double*)calloc(ns * L, sizeof(double));
  st->xi = (double*)malloc(sizeof(double) * M);
  st->zeta = (double*)malloc(sizeof(double) * K);
  st->H = (double*)malloc(sizeof(double) * n3);
  st->part_psum = (double*)malloc(sizeof(double) * N * M);
  st->part_pel = (double*)malloc(sizeof(double) * N * M);
  st->part_r = (double*)malloc(sizeof(double) * (size_t)N * K);
  st->part_rh = (double*)malloc(sizeof(double) * (size_t)N * K);
  st->part_delta = (double*)malloc(sizeof(double) * N);
  st->part_ties = (int64_t*)malloc(sizeof(int64_t) * N);
  st->part_margin = (double*)malloc(sizeof(double) * N);
  st->tie_mn = (int32_t*)calloc((size_t)M * N, sizeof(int32_t));
  st->tie_user = (int32_t*)calloc(K, sizeof(int32_t));
  st->part_sicv = (double*)calloc(N, sizeof(double));
  st->part_moved = (int*)calloc(N, sizeof(int));
  st->part_dres = (double*)calloc(N, sizeof(double));
  st->min_margin = INFINITY;
  st->first_tie = -1;
  cold_start(st);
  if (warm) warm_start(st, warm);
  return st;
}

ORC_API void orc_state_destroy(orc_state* st) {
  if (!st) return;
  free(st->G); free(st->elastic); free(st->psi); free(st->pmax); free(st->eta);
  free(st->pmask); free(st->w); free(st->A); free(st->sel); free(st->p); free(st->al);
  free(st->be); free(st->zs); free(st->xi); free(st->zeta); free(st->H);
  free(st->part_psum); free(st->part_pel); free(st->part_r); free(st->part_rh);
  free(st->part_delta); free(st->part_ties); free(st->part_margin);
  free(st->tie_mn); free(st->tie_user); free(st->part_sicv);
  free(st->part_moved);
  free(st->part_dres);
  free(st);
}

ORC_API void orc_state_set_E(orc_state* st, double E) { st->E = E; }

/* Alg. 1 initialisation: alpha = 1, beta = 0 (high-SIR approximation). */
ORC_API void orc_state_reset_scale(orc_state* st) {
  const size_t ns = (size_t)st->M * st->N * st->L;
  for (size_t i = 0; i < ns; ++i) {
    st->al[i] = 1.0;
    st->be[i] = 0.0;
  }
}

/* ------------------------------------------------------- one subcarrier */

/* Evaluation of RRH m's selected users on subcarrier n at the state. */
typedef struct {
  int cnt;
  int slot[MAXL];    /* storage slot at decoding position q */
  int user[MAXL];
  double gt[MAXL];   /* normalised gain Gamma/(sigma+ICI) */
  double pre[MAXL + 1]; /* power of the users decoded before position q */
  double I[MAXL];    /* interference after SIC (Sec. II-A) */
  double gam[MAXL];  /* SINR gamma'' */
  double r[MAXL];    /* log2(1+gamma) */
  double rh[MAXL];   /* SCALE surrogate beta + alpha log2 gamma */
  double c[MAXL];    /* w mu alpha / (ln2 (sigma + I)) */
  double cg[MAXL];   /* c * Gamma_{m,n,user}: price of interference on this user */
} mview;

/* Relative C14 margin of users a, b on (m,n) from u = (sigma + ICI)/Gamma:
 * with s the user of larger raw gain (ties to the lower index) and w the
 * other, Omega/nu = (u_s - u_w)/(u_s + u_w) (the SIC margin of
 * orc_sic_margin divided through by Gamma_s Gamma_w). */
static double pair_margin(double ga, double ua, int ka, double gb, double ub, int kb) {
  const int a_strong = ga > gb || (ga == gb && ka < kb);
  const double us = a_strong ? ua : ub, uw = a_strong ? ub : ua;
  return (us - uw) / (us + uw);
}

/* ICI and per-RRH evaluation on subcarrier n; optionally refits SCALE.
 * With ties != NULL the decoding-order margins are recorded as near-ties of
 * their (m,n).  *sicv receives the C14 violation of the state's pairs. */
static void eval_subcarrier(orc_state* st, int n, int refit, double* ici, mview* vw,
                            int64_t* ties, double* minm, double* sicv) {
  const int M = st->M, K = st->K, L = st->L;
  const double sg = st->sigma;
  double Ptot[64];
  for (int m = 0; m < M; ++m) {
    Ptot[m] = 0.0;
    for (int s = 0; s < L; ++s)
      if (st->sel[SLOT(st, m, n, s)] >= 0) Ptot[m] += st->p[SLOT(st, m, n, s)];
  }
  /* Inter-cell interference: sum over the other RRHs of their total power on n. */
  for (int m = 0; m < M; ++m)
    for (int k = 0; k < K; ++k) {
      double acc = 0.0;
      for (int j = 0; j < M; ++j)
        if (j != m) acc += Ptot[j] * st->G[IDX3(st, j, n, k)];
      ici[(size_t)m * K + k] = acc;
    }
  for (int m = 0; m < M; ++m) {
    mview* v = &vw[m];
    v->cnt = 0;
    for (int s = 0; s < L; ++s) {
      const int k = st->sel[SLOT(st, m, n, s)];
      if (k < 0) continue;
      v->slot[v->cnt] = s;
      v->user[v->cnt] = k;
      v->gt[v->cnt] = st->G[IDX3(st, m, n, k)] / (sg + ici[(size_t)m * K + k]);
      v->cnt++;
    }
    /* decoding order: normalised gain descending, ties to the lower user */
    for (int i = 1; i < v->cnt; ++i) {
      int j = i;
      while (j > 0 && (v->gt[j - 1] < v->gt[j] ||
                       (v->gt[j - 1] == v->gt[j] && v->user[j - 1] > v->user[j]))) {
        int ts = v->slot[j]; v->slot[j] = v->slot[j - 1]; v->slot[j - 1] = ts;
        int tu = v->user[j]; v->user[j] = v->user[j - 1]; v->user[j - 1] = tu;
        double tg = v->gt[j]; v->gt[j] = v->gt[j - 1]; v->gt[j - 1] = tg;
        --j;
      }
    }
    if (ties)
      for (int q = 0; q + 1 < v->cnt; ++q)
        note_mn(st, m, n, (v->gt[q] - v->gt[q + 1]) / v->gt[q], ties, minm);
    v->pre[0] = 0.0;
    for (int q = 0; q < v->cnt; ++q) v->pre[q + 1] = v->pre[q] + st->p[SLOT(st, m, n, v->slot[q])];
    for (int q = 0; q < v->cnt; ++q) {
      const int k = v->user[q];
      const size_t si = SLOT(st, m, n, v->slot[q]);
      const double g = st->G[IDX3(st, m, n, k)];
      /* users decoded earlier (stronger) interfere; weaker ones are cancelled */
      v->I[q] = ici[(size_t)m * K + k] + g * v->pre[q];
      v->gam[q] = st->p[si] * g / (sg + v->I[q]);
      v->r[q] = log2_1p(v->gam[q]);
      if (refit && st->p[si] > 0.0) orc_scale_coeffs(v->gam[q], &st->al[si], &st->be[si]);
      v->rh[q] = (st->p[si] > 0.0) ? st->be[si] + st->al[si] * log2(v->gam[q]) : 0.0;
      v->c[q] = st->w[(size_t)m * K + k] * mu_of(st, k) * st->al[si] / (LN2 * (sg + v->I[q]));
      v->cg[q] = v->c[q] * g;
    }
  }
  /* C14 at the state: every co-scheduled pair's margin above SIC_TOL */
  double viol = 0.0;
  for (int m = 0; m < M; ++m) {
    const mview* v = &vw[m];
    for (int a = 0; a < v->cnt; ++a)
      for (int b = a + 1; b < v->cnt; ++b) {
        const int ka = v->user[a], kb = v->user[b];
        const double ga = st->G[IDX3(st, m, n, ka)], gb = st->G[IDX3(st, m, n, kb)];
        const double om = pair_margin(ga, (sg + ici[(size_t)m * K + ka]) / ga, ka, gb,
                                      (sg + ici[(size_t)m * K + kb]) / gb, kb);
        if (ties) note_mn(st, m, n, fabs(om - SIC_TOL), ties, minm);
        if (om > SIC_TOL) viol += om - SIC_TOL;
      }
  }
  *sicv = viol;
}

/* Per-subcarrier part of one dual sweep (Alg. 1 inner loop body). */
static void sweep_subcarrier(orc_state* st, int n, double delta_v, int refit) {
  const int M = st->M, K = st->K, L = st->L;
  const double sg = st->sigma, tr = st->prm.tie_rel;
  int64_t ties = 0;
  double minm = INFINITY;
  double* ici = (double*)malloc(sizeof(double) * (size_t)M * K);
  mview* vw = (mview*)malloc(sizeof(mview) * M);
  eval_subcarrier(st, n, refit, ici, vw, &ties, &minm, &st->part_sicv[n]);

  /* Partial sums at the state: power per RRH, rates per user. */
  for (int m = 0; m < M; ++m) {
    double ps = 0.0, pe = 0.0;
    for (int q = 0; q < vw[m].cnt; ++q) {
      const double pq = st->p[SLOT(st, m, n, vw[m].slot[q])];
      ps += pq;
      if (st->elastic[vw[m].user[q]]) pe += pq;
    }
    st->part_psum[(size_t)n * M + m] = ps;
    st->part_pel[(size_t)n * M + m] = pe;
  }
  for (int k = 0; k < K; ++k) {
    st->part_r[(size_t)n * K + k] = 0.0;
    st->part_rh[(size_t)n * K + k] = 0.0;
  }
  for (int m = 0; m < M; ++m)
    for (int q = 0; q < vw[m].cnt; ++q) {
      const int k = vw[m].user[q];
      st->part_r[(size_t)n * K + k] += st->w[(size_t)m * K + k] * vw[m].r[q];
      st->part_rh[(size_t)n * K + k] += st->w[(size_t)m * K + k] * vw[m].rh[q];
    }

  /* Inter-cell price: psi-bar' of the closed forms, the marginal rate loss of
   * the users of the other RRHs per watt transmitted by RRH m on n. */
  double pinter[64], psic[64];
  for (int m = 0; m < M; ++m) {
    double acc = 0.0;
    for (int j = 0; j < M; ++j) {
      if (j == m) continue;
      for (int q = 0; q < vw[j].cnt; ++q) acc += vw[j].c[q] * st->G[IDX3(st, m, n, vw[j].user[q])];
    }
    pinter[m] = acc;
    psic[m] = 0.0;
  }

  /* SIC constraint C14 (DC-linearised, affine in the other RRHs' powers):
   * the multiplier of each co-scheduled pair adds zeta~ dOmega/dp_j to the
   * price of RRH j on n; then the pair's subgradient step. */
  double zs_new[64][MAXL][MAXL];
  double dres = 0.0;
  for (int m = 0; m < M; ++m) {
    const mview* v = &vw[m];
    for (int a = 0; a < v->cnt; ++a)
      for (int b = a + 1; b < v->cnt; ++b) {
        int ka = v->user[a], kb = v->user[b];
        const double ga = st->G[IDX3(st, m, n, ka)], gb = st->G[IDX3(st, m, n, kb)];
        /* strong = larger raw gain, ties to the lower user index */
        int ks = ka, kw = kb;
        if (gb > ga || (gb == ga && kb < ka)) {
          ks = kb;
          kw = ka;
        }
        const double gs = st->G[IDX3(st, m, n, ks)], gw = st->G[IDX3(st, m, n, kw)];
        const double is = ici[(size_t)m * K + ks], iw = ici[(size_t)m * K + kw];
        const double om = orc_sic_margin(gs, gw, is, iw, sg);
        const double nu = gw * (sg + is) + gs * (sg + iw);
        const int sa = v->slot[a], sb = v->slot[b];
        const double z = st->zs[PAIR(st, m, n, sa, sb)];
        for (int j = 0; j < M; ++j) {
          if (j == m) continue;
          const double dj = (gw * st->G[IDX3(st, j, n, ks)] - gs * st->G[IDX3(st, j, n, kw)]) / nu;
          psic[j] += z * dj;
        }
        const double zn = fmax(z + delta_v * om, 0.0);
        dres = fmax(dres, fabs(zn - z) / delta_v);
        zs_new[m][sa][sb] = zn;
        zs_new[m][sb][sa] = zn;
      }
  }

  /* Per-triple Lagrangian maximum H and candidate lists. */
  double* cand_Hbuf = (double*)malloc(sizeof(double) * (size_t)M * K);
  int* cand_kbuf = (int*)malloc(sizeof(int) * (size_t)M * K);
  double* cand_pintra = (double*)malloc(sizeof(double) * K); /* intra price on A_k */
#define cand_H(m) (cand_Hbuf + (size_t)(m) * K)
#define cand_k(m) (cand_kbuf + (size_t)(m) * K)
  int ncand[64], nbdry[64];
  for (int m = 0; m < M; ++m) {
    ncand[m] = 0;
    nbdry[m] = 0;
  }
  for (int m = 0; m < M; ++m) {
    const mview* v = &vw[m];
    for (int k = 0; k < K; ++k) {
      const double g = st->G[IDX3(st, m, n, k)];
      const double ik = ici[(size_t)m * K + k];
      int q = -1;
      for (int t = 0; t < v->cnt; ++t)
        if (v->user[t] == k) q = t;
      double Sb, pintra = 0.0;
      if (q >= 0) {
        Sb = v->pre[q];
        for (int t = q + 1; t < v->cnt; ++t) pintra += v->cg[t];
      } else {
        const double gk = g / (sg + ik);
        int pos = 0;
        for (int t = 0; t < v->cnt; ++t) {
          if (v->gt[t] > gk || (v->gt[t] == gk && v->user[t] < k)) pos++;
          note_mn(st, m, n, fabs(v->gt[t] - gk) / fmax(v->gt[t], gk), &ties, &minm);
        }
        Sb = v->pre[pos];
        for (int t = pos; t < v->cnt; ++t) pintra += v->cg[t];
      }
      const double a = g / (sg + ik + g * Sb);
      const double wmu = st->w[(size_t)m * K + k] * mu_of(st, k);
      const double c = (st->elastic[k] ? st->E * st->eta[m] : 0.0) + st->xi[m] + pintra +
                       pinter[m] + psic[m];
      double H = 0.0;
      if (wmu > 0.0) {
        double pt;
        if (c <= 0.0) {
          pt = st->pmask[m];
        } else {
          const double Wl = wmu / (c * LN2);
          const double d = Wl - 1.0 / a;
          if (st->A[k] == m && fabs(d) <= tr * Wl) nbdry[m]++;
          pt = fmin(fmax(d, 0.0), st->pmask[m]);
        }
        if (pt > 0.0) H = wmu * log2_1p(a * pt) - c * pt;
      }
      st->H[IDX3(st, m, n, k)] = H;
      if (st->A[k] == m) {
        cand_pintra[k] = pintra;
        if (H > 0.0) {
          cand_H(m)[ncand[m]] = H;
          cand_k(m)[ncand[m]] = k;
          ncand[m]++;
        }
      }
    }
  }

  int moved = 0;
  /* Selection and closed-form powers for the new selection: RRH m's
   * candidates in order of H (ties to the lower user), each taken only if
   * every pair it forms with the users taken before it meets C14 (margin
   * <= 0 at the state's interference), until l are taken. */
  double dmax = 0.0;
  for (int m = 0; m < M; ++m) {
    const mview* v = &vw[m];
    int chosen[MAXL], np = 0, last = -1;
    int* ord = (int*)malloc(sizeof(int) * (ncand[m] > 0 ? ncand[m] : 1));
    int no = 0;
    top_by_key(cand_H(m), cand_k(m), ncand[m], ncand[m], ord, &no);
    for (int e = 0; e < no && np < L; ++e) {
      const int k = cand_k(m)[ord[e]];
      const double gk = st->G[IDX3(st, m, n, k)], uk = (sg + ici[(size_t)m * K + k]) / gk;
      int ok = 1;
      for (int a = 0; a < np; ++a) {
        const int j = chosen[a];
        const double gj = st->G[IDX3(st, m, n, j)], uj = (sg + ici[(size_t)m * K + j]) / gj;
        const double om = pair_margin(gk, uk, k, gj, uj, j);
        note_mn(st, m, n, fabs(om), &ties, &minm);
        if (om > 0.0) ok = 0;
      }
      if (ok) chosen[np++] = k;
      last = e;
    }
    /* the order of the candidates considered, and the first one not
     * considered, decide the selection */
    for (int e = 0; e <= last && e + 1 < no; ++e) {
      const double h0 = cand_H(m)[ord[e]], h1 = cand_H(m)[ord[e + 1]];
      note_mn(st, m, n, (h0 - h1) / h0, &ties, &minm);
    }
    free(ord);
    if (nbdry[m] > 0 && ncand[m] <= L + nbdry[m]) {
      ties += nbdry[m];
      st->tie_mn[(size_t)m * st->N + n] += nbdry[m];
    }

    int same = np == v->cnt;
    for (int s = 0; s < np && same; ++s) {
      int found = 0;
      for (int t = 0; t < v->cnt; ++t) found |= v->user[t] == chosen[s];
      same = found;
    }
    if (!same) moved = 1;

    int new_user[MAXL];
    double new_p[MAXL], new_al[MAXL], new_be[MAXL];
    for (int s = 0; s < L; ++s) new_user[s] = -1;
    for (int s = 0; s < np; ++s) {
      const int k = chosen[s];
      int old = -1;
      for (int t = 0; t < v->cnt; ++t)
        if (v->user[t] == k) old = v->slot[t];
      double p_old = 0.0, alph = 1.0, bet = 0.0;
      if (old >= 0) {
        const size_t si = SLOT(st, m, n, old);
        p_old = st->p[si];
        alph = st->al[si];
        bet = st->be[si];
      }
      const double wmu = st->w[(size_t)m * K + k] * mu_of(st, k);
      const double pplus = fmax(psic[m], 0.0), pminus = fmax(-psic[m], 0.0);
      const double cp = (st->elastic[k] ? st->E * st->eta[m] : 0.0) + st->xi[m] +
                        cand_pintra[k] + pinter[m] + pplus;
      const double num = wmu * alph / LN2 + p_old * pminus;
      double pn = (cp > 0.0) ? fmin(fmax(num / cp, 0.0), st->pmask[m]) : st->pmask[m];
      const double floor_p = POWER_FLOOR_REL * st->pmask[m];
      if (pn > 0.0) note_mn(st, m, n, fabs(pn - floor_p) / floor_p, &ties, &minm);
      if (pn < floor_p) pn = 0.0;
      new_user[s] = k;
      new_p[s] = pn;
      new_al[s] = alph;
      new_be[s] = bet;
    }
    /* max |p_new - p_old| / pmask over the old and new slots of (m,n) */
    for (int s = 0; s < np; ++s) {
      double p_old = 0.0;
      for (int t = 0; t < v->cnt; ++t)
        if (v->user[t] == new_user[s]) p_old = st->p[SLOT(st, m, n, v->slot[t])];
      dmax = fmax(dmax, fabs(new_p[s] - p_old) / st->pmask[m]);
    }
    for (int t = 0; t < v->cnt; ++t) {
      int kept = 0;
      for (int s = 0; s < np; ++s)
        if (new_user[s] == v->user[t]) kept = 1;
      if (!kept) dmax = fmax(dmax, st->p[SLOT(st, m, n, v->slot[t])] / st->pmask[m]);
    }
    /* C14 multipliers follow their user pair into the new slots. */
    double zmap[MAXL][MAXL];
    for (int a = 0; a < L; ++a)
      for (int b = 0; b < L; ++b) zmap[a][b] = 0.0;
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) {
        if (a == b) continue;
        int oa = -1, ob = -1;
        for (int t = 0; t < v->cnt; ++t) {
          if (v->user[t] == new_user[a]) oa = v->slot[t];
          if (v->user[t] == new_user[b]) ob = v->slot[t];
        }
        if (oa >= 0 && ob >= 0) zmap[a][b] = zs_new[m][oa][ob];
      }
    for (int s = 0; s < L; ++s) {
      const size_t si = SLOT(st, m, n, s);
      st->sel[si] = new_user[s];
      st->p[si] = (s < np) ? new_p[s] : 0.0;
      st->al[si] = (s < np) ? new_al[s] : 1.0;
      st->be[si] = (s < np) ? new_be[s] : 0.0;
      for (int b = 0; b < L; ++b) st->zs[PAIR(st, m, n, s, b)] = zmap[s][b];
    }
  }
  st->part_delta[n] = dmax;
  st->part_moved[n] = moved;
  st->part_dres[n] = dres;
  st->part_ties[n] = ties;
  st->part_margin[n] = minm;
#undef cand_H
#undef cand_k
  free(cand_Hbuf);
  free(cand_kbuf);
  free(cand_pintra);
  free(ici);
  free(vw);
}

/* ------------------------------------------------------------ the sweep */

/* Totals of a state from its per-subcarrier parts, each summed serially in
 * increasing n: the weighted elastic sum rate R (Sec. II-A), the power P of
 * the power model, and the violations of C13 (sum over streaming users of
 * (1 - QOS_TOL) - r_k/Psi_k where positive), C12 (sum over RRHs of
 * sum_p/pmax - (1 + BUDGET_TOL) where positive) and C14 (sum of the pair
 * margins above SIC_TOL).  A threshold decision within tie_rel is a
 * near-tie. */
static int64_t state_totals(orc_state* st, const double* part_r, const double* part_pel,
                            const double* part_psum, const double* part_sicv, double* user_rate) {
  const int M = st->M, N = st->N, K = st->K;
  int64_t ties = 0;
  double Rs = 0.0, Ps = st->pstatic, vq = 0.0, vp = 0.0, vs = 0.0;
  for (int k = 0; k < K; ++k) {
    double r = 0.0;
    for (int n = 0; n < N; ++n) r += part_r[(size_t)n * K + k];
    if (user_rate) user_rate[k] = r;
    if (st->elastic[k]) {
      Rs += r;
    } else {
      const double x = r / st->psi[k];
      if (fabs(x - (1.0 - QOS_TOL)) <= st->prm.tie_rel) {
        ties++;
        st->tie_user[k]++;
      }
      if (x < 1.0 - QOS_TOL) vq += (1.0 - QOS_TOL) - x;
    }
  }
  for (int m = 0; m < M; ++m) {
    double pe = 0.0, ps = 0.0;
    for (int n = 0; n < N; ++n) {
      pe += part_pel[(size_t)n * M + m];
      ps += part_psum[(size_t)n * M + m];
    }
    Ps += st->eta[m] * pe;
    const double y = ps / st->pmax[m];
    if (fabs(y - (1.0 + BUDGET_TOL)) <= st->prm.tie_rel) ties++;
    if (y > 1.0 + BUDGET_TOL) vp += y - (1.0 + BUDGET_TOL);
  }
  for (int n = 0; n < N; ++n) vs += part_sicv[n];
  st->ev_R = Rs;
  st->ev_P = Ps;
  st->ev_Vq = vq;
  st->ev_Vp = vp;
  st->ev_Vs = vs;
  return ties;
}

ORC_API double orc_state_sweep(orc_state* st, int32_t v, int32_t refit) {
  const int M = st->M, N = st->N, K = st->K, L = st->L;
  const double delta_v = st->prm.step0 / sqrt(1.0 + (double)v);
  st->assoc_changed = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int n = 0; n < N; ++n) sweep_subcarrier(st, n, delta_v, refit);

  /* Sums over subcarriers, serially in increasing n. */
  double delta = 0.0;
  int64_t ties = 0;
  st->moved = 0;
  for (int n = 0; n < N; ++n) {
    st->moved |= st->part_moved[n];
    delta = fmax(delta, st->part_delta[n]);
    delta = fmax(delta, st->part_dres[n]);
    ties += st->part_ties[n];
    if (st->part_margin[n] < st->min_margin) st->min_margin = st->part_margin[n];
  }
  /* The state this sweep read: sum rate R, power P, constraint violations. */
  ties += state_totals(st, st->part_r, st->part_pel, st->part_psum, st->part_sicv, NULL);
  /* C12 subgradient: xi'_m <- [xi'_m + delta (sum p - pmax)/pmax * N l/(ln2 pmax)]^+ */
  for (int m = 0; m < M; ++m) {
    double ps = 0.0;
    for (int n = 0; n < N; ++n) ps += st->part_psum[(size_t)n * M + m];
    const double scale = (double)N * L / (LN2 * st->pmax[m]);
    const double xn = fmax(st->xi[m] + delta_v * scale * (ps - st->pmax[m]) / st->pmax[m], 0.0);
    delta = fmax(delta, fabs(xn - st->xi[m]) / (delta_v * scale));
    st->xi[m] = xn;
  }
  /* C13 subgradient on the SCALE surrogate rate of each streaming user; the
   * relative violation (Psi - r_hat)/Psi is clipped to [-qos_down, 1]. */
  for (int k = 0; k < K; ++k) {
    if (st->elastic[k]) continue;
    double rh = 0.0;
    for (int n = 0; n < N; ++n) rh += st->part_rh[(size_t)n * K + k];
    const double viol = fmin(fmax((st->psi[k] - rh) / st->psi[k], -st->prm.qos_down), 1.0);
    const double zn = fmax(st->zeta[k] + delta_v * viol, 0.0);
    delta = fmax(delta, fabs(zn - st->zeta[k]) / delta_v);
    st->zeta[k] = zn;
  }
  /* RRH association from the summed per-triple Lagrangian maxima. */
  for (int k = 0; k < K; ++k) {
    double best = -INFINITY, second = -INFINITY;
    int bm = 0;
    for (int m = 0; m < M; ++m) {
      double s = 0.0;
      for (int n = 0; n < N; ++n) s += st->H[IDX3(st, m, n, k)];
      if (s > best) {
        second = best;
        best = s;
        bm = m;
      } else if (s > second) {
        second = s;
      }
    }
    const int before = st->A[k];
    if (best > 0.0) {
      if (M > 1 && second > 0.0) {
        const int64_t t0 = ties;
        note_margin((best - second) / best, st->prm.tie_rel, &ties, &st->min_margin);
        if (ties > t0) st->tie_user[k]++;
      }
      st->A[k] = bm;
    } else if (st->elastic[k]) {
      st->A[k] = -1;
    }
    if (st->A[k] != before) st->assoc_changed++;
  }
  if (st->assoc_changed) st->moved = 1;
  if (ties > 0) {
    if (st->first_tie < 0) st->first_tie = st->sweeps_done;
    st->ties += ties;
  }
  st->sweeps_done++;
  /* a sweep that moved any user to another RRH has not converged */
  return st->assoc_changed ? INFINITY : delta;
}

ORC_API void orc_state_eval(orc_state* st, double* R, double* P, double* R_hat,
                            double* user_rate) {
  const int M = st->M, N = st->N, K = st->K;
  double* rk = (double*)calloc((size_t)N * K, sizeof(double));
  double* rhk = (double*)calloc((size_t)N * K, sizeof(double));
  double* pe = (double*)calloc((size_t)N * M, sizeof(double));
  double* ps = (double*)calloc((size_t)N * M, sizeof(double));
  double* sv = (double*)calloc((size_t)N, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int n = 0; n < N; ++n) {
    double* ici = (double*)malloc(sizeof(double) * (size_t)M * K);
    mview* vw = (mview*)malloc(sizeof(mview) * M);
    eval_subcarrier(st, n, 0, ici, vw, NULL, NULL, &sv[n]);
    for (int m = 0; m < M; ++m)
      for (int q = 0; q < vw[m].cnt; ++q) {
        const int k = vw[m].user[q];
        const double pq = st->p[SLOT(st, m, n, vw[m].slot[q])];
        rk[(size_t)n * K + k] += st->w[(size_t)m * K + k] * vw[m].r[q];
        rhk[(size_t)n * K + k] += st->w[(size_t)m * K + k] * vw[m].rh[q];
        ps[(size_t)n * M + m] += pq;
        if (st->elastic[k]) pe[(size_t)n * M + m] += pq;
      }
    free(ici);
    free(vw);
  }
  st->ties += state_totals(st, rk, pe, ps, sv, user_rate);
  double Rh = 0.0;
  for (int k = 0; k < K; ++k) {
    double h = 0.0;
    for (int n = 0; n < N; ++n) h += rhk[(size_t)n * K + k];
    if (st->elastic[k]) Rh += h;
  }
  *R = st->ev_R;
  *P = st->ev_P;
  if (R_hat) *R_hat = Rh;
  free(rk);
  free(rhk);
  free(pe);
  free(ps);
  free(sv);
}

/* Final state in the output layout: slots in decoding order. */
ORC_API void orc_state_export(orc_state* st, orc_result* res) {
  const int M = st->M, N = st->N, K = st->K, L = st->L;
  const int NP = L * (L - 1) / 2;
  double* ici = (double*)malloc(sizeof(double) * (size_t)M * K);
  mview* vw = (mview*)malloc(sizeof(mview) * M);
  if (res->rrh_of_user)
    for (int k = 0; k < K; ++k) res->rrh_of_user[k] = -1;
  for (int n = 0; n < N; ++n) {
    double sv;
    eval_subcarrier(st, n, 0, ici, vw, NULL, NULL, &sv);
    for (int m = 0; m < M; ++m) {
      const mview* v = &vw[m];
      if (res->rrh_of_user)
        for (int q = 0; q < v->cnt; ++q) res->rrh_of_user[v->user[q]] = m;
      for (int q = 0; q < L; ++q) {
        const size_t o = SLOT(st, m, n, q);
        if (res->sel) res->sel[o] = (q < v->cnt) ? v->user[q] : -1;
        if (res->slot_power) res->slot_power[o] = (q < v->cnt) ? st->p[SLOT(st, m, n, v->slot[q])] : 0.0;
      }
      if (res->zeta_sic && NP > 0) {
        int pi = 0;
        for (int a = 0; a < L; ++a)
          for (int b = a + 1; b < L; ++b, ++pi) {
            double z = 0.0;
            if (b < v->cnt) z = st->zs[PAIR(st, m, n, v->slot[a], v->slot[b])];
            res->zeta_sic[((size_t)m * N + n) * NP + pi] = z;
          }
      }
    }
  }
  free(ici);
  free(vw);
  if (res->tie_mn)
    for (size_t i = 0; i < (size_t)M * N; ++i) res->tie_mn[i] = st->tie_mn[i];
  if (res->tie_user)
    for (int k = 0; k < K; ++k) res->tie_user[k] = st->tie_user[k];
  if (res->xi)
    for (int m = 0; m < M; ++m) res->xi[m] = st->xi[m];
  if (res->zeta)
    for (int k = 0; k < K; ++k) res->zeta[k] = st->zeta[k];
}

ORC_API void orc_state_get_slots(orc_state* st, int32_t* sel, double* power, double* xi,
                                 double* zeta, double* zs) {
  const size_t ns = (size_t)st->M * st->N * st->L;
  for (size_t i = 0; i < ns; ++i) {
    if (sel) sel[i] = st->sel[i];
    if (power) power[i] = st->p[i];
  }
  if (zs)
    for (size_t i = 0; i < ns * st->L; ++i) zs[i] = st->zs[i];
  if (xi)
    for (int m = 0; m < st->M; ++m) xi[m] = st->xi[m];
  if (zeta)
    for (int k = 0; k < st->K; ++k) zeta[k] = st->zeta[k];
}

ORC_API void orc_state_set_multipliers(orc_state* st, const double* xi, const double* zeta,
                                       const double* zs) {
  if (xi)
    for (int m = 0; m < st->M; ++m) st->xi[m] = xi[m];
  if (zeta)
    for (int k = 0; k < st->K; ++k) st->zeta[k] = zeta[k];
  if (zs) memcpy(st->zs, zs, sizeof(double) * (size_t)st->M * st->N * st->L * st->L);
}

ORC_API void orc_state_get_H(orc_state* st, double* H) {
  memcpy(H, st->H, sizeof(double) * (size_t)st->M * st->N * st->K);
}

ORC_API void orc_state_set_powers(orc_state* st, const double* power) {
  const size_t ns = (size_t)st->M * st->N * st->L;
  for (size_t i = 0; i < ns; ++i)
    if (st->sel[i] >= 0) st->p[i] = power[i];
}

/* ---------------------------------------------------------- C14 repair */

/* Makes subcarrier n of the state meet C14 (Sec. II-B, C8/C14: a
 * co-scheduled pair is SIC-decodable only when its raw-gain and
 * normalised-gain orders agree).  While a pair breaks it at the state's
 * interference, the pair of largest margin (RRHs in increasing order, then
 * pairs in decoding order, the first of equal margins) loses one user: the
 * elastic one when exactly one is elastic (streaming users keep the rates
 * C13 asks for), otherwise the one of lower rate on the subcarrier (the
 * higher user index on equal rates).  Its slot is emptied with its C14
 * multipliers.  Every round removes a user, so the loop ends. */
static void repair_subcarrier(orc_state* st, int n, double* ici, mview* vw) {
  const int M = st->M, K = st->K, L = st->L;
  const double sg = st->sigma;
  for (;;) {
    double sv, best = SIC_TOL;
    int bm = -1, ba = 0, bb = 0;
    eval_subcarrier(st, n, 0, ici, vw, NULL, NULL, &sv);
    for (int m = 0; m < M; ++m) {
      const mview* v = &vw[m];
      for (int a = 0; a < v->cnt; ++a)
        for (int b = a + 1; b < v->cnt; ++b) {
          const int ka = v->user[a], kb = v->user[b];
          const double ga = st->G[IDX3(st, m, n, ka)], gb = st->G[IDX3(st, m, n, kb)];
          const double om = pair_margin(ga, (sg + ici[(size_t)m * K + ka]) / ga, ka, gb,
                                        (sg + ici[(size_t)m * K + kb]) / gb, kb);
          note_mn(st, m, n, fabs(om - best) / fmax(fabs(best), SIC_TOL), &st->part_ties[n], &st->part_margin[n]);
          if (om > best) {
            best = om;
            bm = m;
            ba = a;
            bb = b;
          }
        }
    }
    if (bm < 0) return;
    const mview* v = &vw[bm];
    const int ea = st->elastic[v->user[ba]], eb = st->elastic[v->user[bb]];
    int drop;
    if (ea != eb) {
      drop = ea ? ba : bb;
    } else {
      const double ra = v->r[ba], rb = v->r[bb];
      note_mn(st, bm, n, fabs(ra - rb) / fmax(fmax(ra, rb), DBL_MIN), &st->part_ties[n],
              &st->part_margin[n]);
      if (ra != rb)
        drop = ra < rb ? ba : bb;
      else
        drop = v->user[ba] > v->user[bb] ? ba : bb;
    }
    const int s = v->slot[drop];
    const size_t si = SLOT(st, bm, n, s);
    st->sel[si] = -1;
    st->p[si] = 0.0;
    st->al[si] = 1.0;
    st->be[si] = 0.0;
    for (int b = 0; b < L; ++b) {
      st->zs[PAIR(st, bm, n, s, b)] = 0.0;
      st->zs[PAIR(st, bm, n, b, s)] = 0.0;
    }
  }
}

static void repair_sic(orc_state* st) {
  const int M = st->M, N = st->N, K = st->K;
#pragma omp parallel for schedule(dynamic, 1)
  for (int n = 0; n < N; ++n) {
    double* ici = (double*)malloc(sizeof(double) * (size_t)M * K);
    mview* vw = (mview*)malloc(sizeof(mview) * M);
    st->part_ties[n] = 0;
    st->part_margin[n] = INFINITY;
    repair_subcarrier(st, n, ici, vw);
    free(ici);
    free(vw);
  }
  for (int n = 0; n < N; ++n) {
    st->ties += st->part_ties[n];
    if (st->part_margin[n] < st->min_margin) st->min_margin = st->part_margin[n];
  }
}

ORC_API void orc_state_repair_sic(orc_state* st) { repair_sic(st); }

/* ---------------------------------------------------------- full solve */

/* Primal state of an iterate: association, selection, powers, SCALE
 * coefficients and the C14 multipliers that live with the slot pairs.  The
 * multipliers xi' and zeta' are not part of it: they continue from the last
 * sweep. */
typedef struct {
  int* A;
  int* sel;
  double *p, *al, *be, *zs;
} orc_snap;

static void snap_alloc(const orc_state* st, orc_snap* s) {
  const size_t ns = (size_t)st->M * st->N * st->L;
  s->A = (int*)malloc(sizeof(int) * st->K);
  s->sel = (int*)malloc(sizeof(int) * ns);
  s->p = (double*)malloc(sizeof(double) * ns);
  s->al = (double*)malloc(sizeof(double) * ns);
  s->be = (double*)malloc(sizeof(double) * ns);
  s->zs = (double*)malloc(sizeof(double) * ns * st->L);
}

static void snap_free(orc_snap* s) {
  free(s->A);
  free(s->sel);
  free(s->p);
  free(s->al);
  free(s->be);
  free(s->zs);
}

static void snap_copy(const orc_state* st, int* A, int* sel, double* p, double* al, double* be,
                      double* zs, const int* A0, const int* sel0, const double* p0,
                      const double* al0, const double* be0, const double* zs0) {
  const size_t ns = (size_t)st->M * st->N * st->L;
  memcpy(A, A0, sizeof(int) * st->K);
  memcpy(sel, sel0, sizeof(int) * ns);
  memcpy(p, p0, sizeof(double) * ns);
  memcpy(al, al0, sizeof(double) * ns);
  memcpy(be, be0, sizeof(double) * ns);
  memcpy(zs, zs0, sizeof(double) * ns * st->L);
}

static void snap_take(const orc_state* st, orc_snap* s) {
  snap_copy(st, s->A, s->sel, s->p, s->al, s->be, s->zs, st->A, st->sel, st->p, st->al, st->be,
            st->zs);
}

static void snap_put(orc_state* st, const orc_snap* s) {
  snap_copy(st, st->A, st->sel, st->p, st->al, st->be, st->zs, s->A, s->sel, s->p, s->al, s->be,
            s->zs);
}

static void snap_assign(const orc_state* st, orc_snap* d, const orc_snap* s) {
  snap_copy(st, d->A, d->sel, d->p, d->al, d->be, d->zs, s->A, s->sel, s->p, s->al, s->be, s->zs);
}

/* Relative change of the violation that separates two iterates in the
 * ranking below. */
#define VIOL_REL 1e-6

/* Violations Va against Vb: -1 when Va is lower by more than VIOL_REL
 * (relative), 1 when higher, 0 otherwise (zero only equals zero). */
static int cmp_viol(double Va, double Vb, double tie_rel, int64_t* ties, double* minm) {
  if (Va == 0.0 && Vb == 0.0) return 0;
  if (Va == 0.0) return -1;
  if (Vb == 0.0) return 1;
  const double lo = Vb * (1.0 - VIOL_REL), hi = Vb * (1.0 + VIOL_REL);
  note_margin(fmin(fabs(Va - lo), fabs(Va - hi)) / Vb, tie_rel, ties, minm);
  if (Va < lo) return -1;
  if (Va > hi) return 1;
  return 0;
}

/* Ranking of the iterate a just evaluated against the best iterate b of the
 * Dinkelbach step: less C12/C13 violation V first, then less C14 violation
 * V2 (feasible = both zero), then the larger Dinkelbach objective
 * f = R - E P.  *replace: a becomes the best; *progress: it is better by more
 * than the violation band or, at equal violation, by more than rel times the
 * best's rate R_b (rel = the Dinkelbach tolerance: smaller gains are below
 * what the outer loop resolves).  moved: a and b differ in a selected set or
 * an association (otherwise choosing between them by f is no discrete
 * decision). */
static void rank_iterate(double Va, double Va2, double fa, double Vb, double Vb2, double fb,
                         double Rb, double rel, int moved, double tie_rel, int64_t* ties,
                         double* minm, int* replace, int* progress) {
  int c = cmp_viol(Va, Vb, tie_rel, ties, minm);
  if (c == 0) c = cmp_viol(Va2, Vb2, tie_rel, ties, minm);
  if (c != 0) {
    *replace = *progress = c < 0;
    return;
  }
  const double thr = rel * fabs(Rb);
  if (Rb != 0.0) {
    note_margin(fabs(fa - fb - thr) / fabs(Rb), tie_rel, ties, minm);
    if (moved) note_margin(fabs(fa - fb) / fabs(Rb), tie_rel, ties, minm);
  }
  *replace = fa > fb;
  *progress = fa - fb > thr;
}

/* Dinkelbach outer loop (Sec. III-IV) around the dual sweeps of Alg. 1.
 * Step i runs dual sweeps at E^i from the previous step's returned state and
 * returns the best state it visited (see rank_iterate()); F_i = R - E^i P at
 * that state; the solve stops when that state meets C12 and C13 and
 * |F_i| <= tol_dinkelbach R, otherwise E^{i+1} = R/P of that state. */
ORC_API int orc_solve(const orc_problem* pb, const orc_params* prm, const orc_warm* warm,
                      orc_result* res) {
  const int rc = validate(pb);
  if (rc != 0) return rc;
  orc_state* st = orc_state_create(pb, prm, warm);
  if (!st) return -12;
  const int K = st->K;
  uint32_t flags = 0;
  double R = 0.0, P = st->pstatic;
  int i = 0, total = 0;
  double* rate = (double*)malloc(sizeof(double) * K);
  orc_snap cur, best;
  snap_alloc(st, &cur);
  snap_alloc(st, &best);
  st->E = 0.0; /* E^0 = 0 */
  /* A warm initial allocation is Dinkelbach's p^0: a first step without
   * sweeps evaluates it, E^1 = R(p^0)/P(p^0), and the sweeps start from it. */
  int eval_only = (warm && warm->p0) ? 1 : 0;
  for (;;) {
    int v = 0;
    if (eval_only) {
      orc_state_eval(st, &R, &P, NULL, rate);
    } else {
      orc_state_reset_scale(st);
      int have_best = 0, stall = 0, moved = 0;
      double bV = 0.0, bV2 = 0.0, bf = 0.0, bR = 0.0;
      for (;;) {
        const int refit = prm->refit_period > 0 && (v % prm->refit_period) == 0;
        snap_take(st, &cur);
        const double d = orc_state_sweep(st, v, refit);
        ++v;
        ++total;
        if (isnan(d)) {
          flags |= ORC_NONFINITE;
          break;
        }
        /* the state read by this sweep against the best so far ("moved":
         * a sweep since the best changed a selected set or an association) */
        const double V = st->ev_Vq + st->ev_Vp, V2 = st->ev_Vs;
        const double f = st->ev_R - st->E * st->ev_P;
        int replace = 1, progress = 1;
        if (have_best)
          rank_iterate(V, V2, f, bV, bV2, bf, bR, prm->tol_dinkelbach, moved, prm->tie_rel,
                       &st->ties, &st->min_margin, &replace, &progress);
        if (replace) {
          snap_assign(st, &best, &cur);
          have_best = 1;
          bV = V;
          bV2 = V2;
          bf = f;
          bR = st->ev_R;
          moved = 0;
        }
        stall = progress ? 0 : stall + 1;
        moved |= st->moved;
        if (v >= prm->sweeps_per_dinkelbach) break;
        if (!prm->fixed_count) {
          if (fabs(d - prm->tol_dual) <= 1e-6 * prm->tol_dual) st->ties++;
          if (d < prm->tol_dual) break;
          if (prm->stall_sweeps > 0 && stall >= prm->stall_sweeps) break;
        }
      }
      if (have_best) snap_put(st, &best);
      orc_state_eval(st, &R, &P, NULL, rate);
    }
    const double F = R - st->E * P;
    if (res->trace_E) res->trace_E[i] = st->E;
    if (res->trace_F) res->trace_F[i] = F;
    if (res->trace_R) res->trace_R[i] = R;
    if (res->trace_P) res->trace_P[i] = P;
    if (res->trace_sweeps) res->trace_sweeps[i] = v;
    ++i;
    if (flags & ORC_NONFINITE) break;
    if (eval_only) {
      eval_only = 0;
      if (i >= prm->max_dinkelbach) {
        flags |= ORC_NOT_CONVERGED;
        break;
      }
      st->E = R / P;
      continue;
    }
    /* Dinkelbach's test applies to iterates that meet C12 and C13; an
     * infeasible step is followed by another (the multipliers keep moving
     * towards feasibility) */
    const int feasible = st->ev_Vq == 0.0 && st->ev_Vp == 0.0;
    if (fabs(fabs(F) - prm->tol_dinkelbach * R) <= 1e-6 * prm->tol_dinkelbach * fabs(R)) st->ties++;
    if (feasible && fabs(F) <= prm->tol_dinkelbach * R) break;
    if (i >= prm->max_dinkelbach) {
      flags |= ORC_NOT_CONVERGED;
      break;
    }
    st->E = R / P; /* E^{i+1} = R(p^i)/P(p^i) */
  }
  snap_free(&cur);
  snap_free(&best);
  /* the returned allocation meets C14: pairs that still break it are
   * dissolved, and the allocation is evaluated again */
  if (st->ev_Vs > 0.0 && !(flags & ORC_NONFINITE)) {
    repair_sic(st);
    orc_state_eval(st, &R, &P, NULL, rate);
  }
  orc_state_export(st, res);
  if (st->ev_Vq > 0.0) flags |= ORC_QOS_INFEASIBLE;
  if (st->ev_Vp > 0.0) flags |= ORC_BUDGET_INFEASIBLE;
  if (st->ev_Vs > 0.0) flags |= ORC_SIC_INFEASIBLE;
  for (int k = 0; k < K; ++k) {
    if (res->user_rate) res->user_rate[k] = rate[k];
    if (!isfinite(rate[k])) flags |= ORC_NONFINITE;
  }
  if (st->ties > 0) flags |= ORC_NEAR_TIE;
  res->ee = (P > 0.0) ? R / P : 0.0;
  res->rate_sum = R;
  res->power_sum = P;
  res->viol_qos = st->ev_Vq;
  res->viol_budget = st->ev_Vp;
  res->viol_sic = st->ev_Vs;
  res->dinkelbach_iters = i;
  res->sweeps = total;
  res->status_flags = flags;
  res->near_ties = st->ties;
  res->min_margin = st->min_margin;
  res->first_tie_sweep = st->first_tie;
  free(rate);
  orc_state_destroy(st);
  return 0;
}
