/*
 * Seeded synthetic channel drops for the two-tier PD-NOMA H-CRAN downlink.
 *
 * This file generates INPUTS only: geometry, path loss, shadowing, Rayleigh
 * fading and streaming traffic.  It contains none of the allocator's
 * arithmetic (no minimum rate, no SINR, no power model).  Both the FP64
 * reference and the GPU library consume what it writes.
 *
 * Randomness comes from the Philox4x32-10 counter-based generator
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11), written here from its published definition.  Every random number
 * is addressed by (stream tag, element index, drop index) under a key made of
 * (seed, configuration id), so the output does not depend on thread count or
 * call order.
 *
 * Channel model (system model, Sec. II-A: one HPN at the cell centre and M_f
 * LPNs; Gamma = |h|^2 per RRH, user and subcarrier):
 *   HPN path loss 128.1 + 37.6 log10(d_km) dB, LPN 140.7 + 36.7 log10(d_km) dB,
 *   log-normal shadowing per (RRH, user), Exp(1) Rayleigh power per
 *   (RRH, subcarrier, user), distance clamped below at min_dist_m.
 * The paper's own simulation channel (Sec. VIII: chi * d^-3 with chi ~ Exp(1))
 * is path_loss_model = 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYNTH_API __attribute__((visibility("default")))

/* ---------------------------------------------------------------- Philox */

static inline void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

SYNTH_API void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                                   uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof c);
}

/* Stream tags: one per kind of random quantity. */
enum {
  TAG_LPN_POS = 1,
  TAG_USER_POS = 2,
  TAG_SHADOW = 3,
  TAG_FADING = 4,
  TAG_TRAFFIC = 5,
  TAG_TYPE = 6,
  TAG_SIZES = 7
};

typedef struct {
  uint32_t key[2];
  uint32_t drop_lo, drop_hi;
} rng_t;

static rng_t rng_make(uint64_t seed, int32_t cfg_id, uint64_t drop) {
  rng_t r;
  r.key[0] = (uint32_t)(seed & 0xffffffffu);
  r.key[1] = (uint32_t)(seed >> 32) ^ ((uint32_t)cfg_id * 0x85EBCA6Bu);
  r.drop_lo = (uint32_t)(drop & 0xffffffffu);
  r.drop_hi = (uint32_t)(drop >> 32);
  return r;
}

/* Two uniforms in the open interval (0,1), 53 bits each, for element idx. */
static void rng_u2(const rng_t* r, uint32_t tag, uint64_t idx, double u[2]) {
  /* counter = (idx low, idx high ^ tag<<24, drop low, drop high) */
  uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32) ^ (tag << 24), r->drop_lo,
                     r->drop_hi};
  uint32_t o[4];
  synth_philox4x32_10(ctr, r->key, o);
  const double two53 = 9007199254740992.0;
  const uint64_t a = ((uint64_t)(o[0] >> 5) << 26) | (uint64_t)(o[1] >> 6);
  const uint64_t b = ((uint64_t)(o[2] >> 5) << 26) | (uint64_t)(o[3] >> 6);
  u[0] = ((double)a + 0.5) / two53;
  u[1] = ((double)b + 0.5) / two53;
}

/* Standard normal by Box-Muller on one uniform pair (first output). */
static double rng_normal(const rng_t* r, uint32_t tag, uint64_t idx) {
  double u[2];
  rng_u2(r, tag, idx, u);
  return sqrt(-2.0 * log(u[0])) * cos(6.283185307179586 * u[1]);
}

/* ---------------------------------------------------------------- recipe */

typedef struct {
  int32_t cfg_id;      /* part of the RNG key */
  int32_t M;           /* RRHs, index 0 = HPN */
  int32_t N;           /* subcarriers */
  int32_t K;           /* users */
  int32_t K_s;         /* streaming users (types drawn by seeded permutation) */
  int32_t path_loss_model; /* 0: HPN/LPN dB formulas, 1: chi*d^-exponent */
  double cell_radius_m;
  double lpn_ring_min_m, lpn_ring_max_m;
  double cluster_radius_m;
  double cluster_fraction; /* share of users dropped near an LPN */
  double min_dist_m;
  double shadow_db;
  double path_loss_exponent; /* model 1 only */
  double bw_hz;              /* subcarrier bandwidth B_n */
  double noise_dbm_hz;
  double pmax_hpn_dbm, pmax_lpn_dbm;
  double eta_hpn, eta_lpn;
  double rate_bps_lo, rate_bps_hi; /* streaming arrival rate lambda*zbar */
  double delay_lo_s, delay_hi_s;   /* streaming delay target T */
  double packet_bits;
} synth_recipe;

typedef struct {
  float* gain;         /* [M][N][K], k fastest */
  uint8_t* user_type;  /* [K] 0 elastic, 1 streaming */
  double* arrival_bps; /* [K] (0 for elastic) */
  double* delay_s;     /* [K] (0 for elastic) */
  double* pmax_w;      /* [M] */
  double* eta;         /* [M] */
  double* noise_w;     /* [1] noise power per subcarrier */
  double* rrh_xy;      /* [M][2] or NULL */
  double* user_xy;     /* [K][2] or NULL */
} synth_out;

static double dbm_to_w(double dbm) { return pow(10.0, (dbm - 30.0) / 10.0); }

/* Uniform point in an annulus [r0, r1] around (cx, cy). */
static void point_in_annulus(const rng_t* r, uint32_t tag, uint64_t idx, double cx,
                             double cy, double r0, double r1, double* x, double* y) {
  double u[2];
  rng_u2(r, tag, idx, u);
  const double rad = sqrt(r0 * r0 + u[0] * (r1 * r1 - r0 * r0));
  const double th = 6.283185307179586 * u[1];
  *x = cx + rad * cos(th);
  *y = cy + rad * sin(th);
}

SYNTH_API int synth_drop(const synth_recipe* rc, uint64_t seed, uint64_t drop,
                         const synth_out* out) {
  const int M = rc->M, N = rc->N, K = rc->K;
  if (M < 1 || N < 1 || K < 1 || rc->K_s < 0 || rc->K_s > K) return -22;
  const rng_t rg = rng_make(seed, rc->cfg_id, drop);

  /* RRH positions: HPN at the origin, LPNs uniform in an annulus. */
  double rx[64], ry[64];
  if (M > 64) return -22;
  rx[0] = 0.0;
  ry[0] = 0.0;
  for (int m = 1; m < M; ++m)
    point_in_annulus(&rg, TAG_LPN_POS, (uint64_t)m, 0.0, 0.0, rc->lpn_ring_min_m,
                     rc->lpn_ring_max_m, &rx[m], &ry[m]);

  /* Users: the first round(cluster_fraction*K) are clustered round-robin
   * around the LPNs, the rest uniform in the cell disc. */
  int n_clu = (M > 1) ? (int)floor(rc->cluster_fraction * K) : 0;
  double ux_buf[4096], uy_buf[4096];
  if (K > 4096) return -22;
  for (int k = 0; k < K; ++k) {
    if (k < n_clu) {
      const int m = 1 + (k % (M - 1));
      point_in_annulus(&rg, TAG_USER_POS, (uint64_t)k, rx[m], ry[m], 0.0,
                       rc->cluster_radius_m, &ux_buf[k], &uy_buf[k]);
    } else {
      point_in_annulus(&rg, TAG_USER_POS, (uint64_t)k, 0.0, 0.0, 0.0, rc->cell_radius_m,
                       &ux_buf[k], &uy_buf[k]);
    }
  }

  /* User types: a seeded permutation picks which K_s users stream. */
  {
    int perm[4096];
    for (int k = 0; k < K; ++k) perm[k] = k;
    for (int k = K - 1; k > 0; --k) { /* Fisher-Yates */
      double u[2];
      rng_u2(&rg, TAG_TYPE, (uint64_t)k, u);
      int j = (int)floor(u[0] * (double)(k + 1));
      if (j > k) j = k;
      int t = perm[k];
      perm[k] = perm[j];
      perm[j] = t;
    }
    for (int k = 0; k < K; ++k) out->user_type[k] = 0;
    for (int s = 0; s < rc->K_s; ++s) out->user_type[perm[s]] = 1;
  }

  for (int k = 0; k < K; ++k) {
    if (out->user_type[k]) {
      double u[2];
      rng_u2(&rg, TAG_TRAFFIC, (uint64_t)k, u);
      out->arrival_bps[k] = rc->rate_bps_lo + u[0] * (rc->rate_bps_hi - rc->rate_bps_lo);
      out->delay_s[k] = rc->delay_lo_s + u[1] * (rc->delay_hi_s - rc->delay_lo_s);
    } else {
      out->arrival_bps[k] = 0.0;
      out->delay_s[k] = 0.0;
    }
  }

  for (int m = 0; m < M; ++m) {
    out->pmax_w[m] = dbm_to_w(m == 0 ? rc->pmax_hpn_dbm : rc->pmax_lpn_dbm);
    out->eta[m] = (m == 0) ? rc->eta_hpn : rc->eta_lpn;
  }
  out->noise_w[0] = dbm_to_w(rc->noise_dbm_hz) * rc->bw_hz;
  if (out->rrh_xy)
    for (int m = 0; m < M; ++m) {
      out->rrh_xy[2 * m] = rx[m];
      out->rrh_xy[2 * m + 1] = ry[m];
    }
  if (out->user_xy)
    for (int k = 0; k < K; ++k) {
      out->user_xy[2 * k] = ux_buf[k];
      out->user_xy[2 * k + 1] = uy_buf[k];
    }

  /* Large-scale gain per (m,k): path loss and shadowing. */
  double* large = (double*)malloc(sizeof(double) * (size_t)M * (size_t)K);
  if (!large) return -12;
  for (int m = 0; m < M; ++m)
    for (int k = 0; k < K; ++k) {
      double dx = ux_buf[k] - rx[m], dy = uy_buf[k] - ry[m];
      double d = sqrt(dx * dx + dy * dy);
      if (d < rc->min_dist_m) d = rc->min_dist_m;
      double g;
      if (rc->path_loss_model == 0) {
        const double dkm = d / 1000.0;
        const double pl = (m == 0) ? 128.1 + 37.6 * log10(dkm) : 140.7 + 36.7 * log10(dkm);
        const double sh = rc->shadow_db * rng_normal(&rg, TAG_SHADOW, (uint64_t)m * K + k);
        g = pow(10.0, -(pl + sh) / 10.0);
      } else {
        g = pow(d, -rc->path_loss_exponent);
      }
      large[(size_t)m * K + k] = g;
    }

  /* Small-scale Rayleigh power per (m,n,k): Exp(1) = -ln U. */
  const int64_t total = (int64_t)M * N * K;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < total; e += 2) {
    double u[2];
    rng_u2(&rg, TAG_FADING, (uint64_t)(e >> 1), u);
    for (int t = 0; t < 2 && e + t < total; ++t) {
      const int64_t i = e + t;
      const int k = (int)(i % K);
      const int m = (int)(i / ((int64_t)N * K));
      out->gain[i] = (float)(large[(size_t)m * K + k] * (-log(u[t])));
    }
  }
  free(large);
  return 0;
}

/* Sizes of a ragged batch: M = 1 + U{mf_lo..mf_hi}, N from n_choices, K = U{k_lo..k_hi}. */
SYNTH_API void synth_batch_sizes(uint64_t seed, int32_t cfg_id, int32_t B, int32_t mf_lo,
                                 int32_t mf_hi, const int32_t* n_choices, int32_t n_n,
                                 int32_t k_lo, int32_t k_hi, int32_t* M, int32_t* N,
                                 int32_t* K) {
  const rng_t rg = rng_make(seed, cfg_id, 0xFFFFFFFFull);
  for (int b = 0; b < B; ++b) {
    double u[2], v[2];
    rng_u2(&rg, TAG_SIZES, (uint64_t)b * 2, u);
    rng_u2(&rg, TAG_SIZES, (uint64_t)b * 2 + 1, v);
    int mf = mf_lo + (int)floor(u[0] * (mf_hi - mf_lo + 1));
    if (mf > mf_hi) mf = mf_hi;
    int ni = (int)floor(u[1] * n_n);
    if (ni >= n_n) ni = n_n - 1;
    int kk = k_lo + (int)floor(v[0] * (k_hi - k_lo + 1));
    if (kk > k_hi) kk = k_hi;
    M[b] = 1 + mf;
    N[b] = n_choices[ni];
    K[b] = kk;
  }
}
