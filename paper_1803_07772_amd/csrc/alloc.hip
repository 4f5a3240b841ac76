// MI355X (gfx950) allocator kernels and the C ABI declared in include/alloc.h.
//
// One drop is solved by a persistent cooperative grid.  Workgroup b owns the
// subcarriers n = b, b + G, ... (G = grid size): everything the method
// defines per subcarrier (inter-cell interference, SIC decoding order,
// SINRs, SCALE refit, prices, closed-form powers, per-triple Lagrangian
// maxima, selection, the C14 multipliers of the subcarrier's pairs) is local
// to the workgroup that owns it, staged in LDS.  The couplings across
// subcarriers -- the RRH budget multiplier xi', the streaming multipliers
// zeta', the RRH association A and the Dinkelbach parameter E -- are reduced
// once per sweep from per-workgroup partials written in a fixed order.
// Every workgroup runs the same loop control on the same reduced values, so
// the whole Dinkelbach / dual / SCALE schedule stays on the device.
//
// Arithmetic is IEEE double on gains stored as float32.  Reductions are in a
// fixed order (no floating-point atomics), so results are deterministic.

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "alloc.h"

namespace cg = cooperative_groups;

namespace {

constexpr double kLn2 = 0.69314718055994530942;
constexpr int kMaxL = 4;
constexpr int kMaxM = 32;
constexpr int kMaxK = 1024;
constexpr int kMaxMK = 4608;
constexpr int kBlock = 512;
// Closed-form powers below this fraction of the mask become exactly zero, so
// decaying powers never reach the subnormal range.
constexpr double kPowerFloorRel = 1e-20;

enum Mode : int { kSweep = 0, kEval = 1, kDone = 2 };

// Loop-control state.  Every workgroup holds an identical copy.
struct Ctrl {
  double E;       // Dinkelbach parameter of the current step
  double R, P;    // rate and power of the last evaluated state
  int i;          // Dinkelbach steps completed
  int v;          // sweeps done in the current step
  int mode;
  int total;      // sweeps done in total
  int reset;      // next sweep starts a Dinkelbach step
  int pass;       // passes (sweeps and evaluations) done
  uint32_t flags;
};

struct Sched {
  int max_d, sweeps, refit_period, fixed, churn;
  double tol_d, tol_dual, step0;
};

// Device view of one drop: inputs, state, per-workgroup partials.
struct Drop {
  int M, N, K, L, NP;
  const float* G;          // [M][N][K]
  const double* psi;       // [K] minimum rate (0 elastic)
  const uint8_t* elastic;  // [K]
  const double* pmax;      // [M]
  const double* eta;       // [M]
  const double* pmask;     // [M]
  const double* w;         // [M][K] or nullptr (all ones)
  double sigma, pstatic;
  int* A;                  // [K]
  int* sel;                // [M][N][L] storage order
  double* p;               // [M][N][L]
  double* al;              // [M][N][L]
  double* be;              // [M][N][L]
  double* zs;              // [M][N][L][L]
  double* xi;              // [M]
  double* zeta;            // [K]
  int* churn_sel;          // [M][N]
  int* churn_A;            // [K]
  // partials, one row per workgroup
  double* S_part;          // [G][M][K] association metric
  double* r_part;          // [G][K] true rate
  double* rh_part;         // [G][K] SCALE surrogate rate
  double* psum_part;       // [G][M] power, all users
  double* pel_part;        // [G][M] power, elastic users
  double* R_part;          // [G] weighted elastic rate
  double* d_part;          // [G] max |dp|/pmask
  int* chg_count;          // [2] association changes, indexed by pass parity
  double* red;             // [4] R, P, delta (written by workgroup 0)
  double* user_rate;       // [K]
  // decoding-order copies of the last evaluated state
  int* out_sel;            // [M][N][L]
  double* out_p;           // [M][N][L]
  double* out_zs;          // [M][N][NP]
  Ctrl* ctrl;              // final control state for the host
};

// LDS carve-up for one workgroup.
struct Lds {
  float* g;       // [M][K] gains of the current subcarrier
  double* u;      // [M][K] (sigma + ICI)/Gamma
  double* Sacc;   // [M][K] association metric summed over my subcarriers
  double* mu;     // [K] 1 (elastic) or zeta'
  double* Hc;     // [K] H of user k on its own RRH
  double* pic;    // [K] intra-cell price of user k on its own RRH
  double* racc;   // [K]
  double* rhacc;  // [K]
  int* Al;        // [K]
  int* grp;       // [K] users grouped by RRH
  int* grp_off;   // [M+1]
  int* grpk;      // [K] rank of a user within its RRH group
  int* wcnt;      // [kBlock/64][M] per-wave group counts
  int* gcur;      // [M]
  // slots of the current subcarrier, storage order
  int* su;        // [M][L]
  double* sp;     // [M][L]
  double* sal;    // [M][L]
  double* sbe;    // [M][L]
  double* szs;    // [M][L][L]
  double* szn;    // [M][L][L] after this sweep's subgradient step
  // per-RRH view in decoding order
  int* vcnt;      // [M]
  int* vslot;     // [M][L]
  int* vuser;     // [M][L]
  double* vu;     // [M][L]
  double* vpre;   // [M][L+1]
  double* vc;     // [M][L]
  double* vcg;    // [M][L]
  double* vT;     // [M][L+1] suffix sums of vcg
  double* Ptot;   // [M]
  double* pinter; // [M]
  double* psic;   // [M]
  double* contrib; // [M][M]
  double* xi;     // [M]
  double* psacc;  // [M]
  double* peacc;  // [M]
  double* Racc;   // [M]
  double* dmax;   // [M]
  int* churn;     // [M]
  double* red;    // [kBlock] scratch for reductions
  double* tmp;    // [M+2] reduction results
};

__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~size_t(7); }

__host__ __device__ inline size_t lds_bytes(int M, int K, int L) {
  size_t b = 0;
  b += align8(sizeof(float) * M * K);
  b += 2 * sizeof(double) * M * K;
  b += 5 * sizeof(double) * K;
  b += 2 * sizeof(int) * K + align8(sizeof(int) * (M + 1));
  b += align8(sizeof(int) * M * L) + 3 * sizeof(double) * M * L;
  b += 2 * sizeof(double) * M * L * L;
  b += align8(sizeof(int) * M) + 2 * align8(sizeof(int) * M * L);
  b += 3 * sizeof(double) * M * L + 2 * sizeof(double) * M * (L + 1);
  b += 9 * sizeof(double) * M + sizeof(double) * M * M;
  b += align8(sizeof(int) * M);
  b += sizeof(double) * kBlock;
  b += align8(sizeof(int) * K) + align8(sizeof(int) * (kBlock / 64) * M) + align8(sizeof(int) * M);
  b += sizeof(double) * (M + 2);
  return b + 64;
}

__device__ Lds carve(char* base, int M, int K, int L) {
  Lds s;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base + o;
    o += align8(bytes);
    return p;
  };
  s.g = (float*)take(sizeof(float) * M * K);
  s.u = (double*)take(sizeof(double) * M * K);
  s.Sacc = (double*)take(sizeof(double) * M * K);
  s.mu = (double*)take(sizeof(double) * K);
  s.Hc = (double*)take(sizeof(double) * K);
  s.pic = (double*)take(sizeof(double) * K);
  s.racc = (double*)take(sizeof(double) * K);
  s.rhacc = (double*)take(sizeof(double) * K);
  s.Al = (int*)take(sizeof(int) * K);
  s.grp = (int*)take(sizeof(int) * K);
  s.grp_off = (int*)take(sizeof(int) * (M + 1));
  s.grpk = (int*)take(sizeof(int) * K);
  s.wcnt = (int*)take(sizeof(int) * (kBlock / 64) * M);
  s.gcur = (int*)take(sizeof(int) * M);
  s.su = (int*)take(sizeof(int) * M * L);
  s.sp = (double*)take(sizeof(double) * M * L);
  s.sal = (double*)take(sizeof(double) * M * L);
  s.sbe = (double*)take(sizeof(double) * M * L);
  s.szs = (double*)take(sizeof(double) * M * L * L);
  s.szn = (double*)take(sizeof(double) * M * L * L);
  s.vcnt = (int*)take(sizeof(int) * M);
  s.vslot = (int*)take(sizeof(int) * M * L);
  s.vuser = (int*)take(sizeof(int) * M * L);
  s.vu = (double*)take(sizeof(double) * M * L);
  s.vpre = (double*)take(sizeof(double) * M * (L + 1));
  s.vc = (double*)take(sizeof(double) * M * L);
  s.vcg = (double*)take(sizeof(double) * M * L);
  s.vT = (double*)take(sizeof(double) * M * (L + 1));
  s.Ptot = (double*)take(sizeof(double) * M);
  s.pinter = (double*)take(sizeof(double) * M);
  s.psic = (double*)take(sizeof(double) * M);
  s.contrib = (double*)take(sizeof(double) * M * M);
  s.xi = (double*)take(sizeof(double) * M);
  s.psacc = (double*)take(sizeof(double) * M);
  s.peacc = (double*)take(sizeof(double) * M);
  s.Racc = (double*)take(sizeof(double) * M);
  s.dmax = (double*)take(sizeof(double) * M);
  s.churn = (int*)take(sizeof(int) * M);
  s.red = (double*)take(sizeof(double) * kBlock);
  s.tmp = (double*)take(sizeof(double) * (M + 2));
  return s;
}

__device__ inline double log2_1p(double x) { return log1p(x) / kLn2; }

// Loop-control inputs cross workgroups (and XCDs): stored and loaded with
// device-scope atomics so every workgroup reads the same value after a grid
// barrier.
__device__ inline void store_shared(double* p, double v) {
  __hip_atomic_store((unsigned long long*)p, __double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double load_shared(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load((unsigned long long*)p, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
}
__device__ inline void store_shared(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int load_shared(const int* p) {
  return __hip_atomic_load((int*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------- per sweep

// Start of a pass: multipliers, association and RRH groups into LDS,
// accumulators cleared.
__device__ void begin_pass(const Drop& d, Lds& s) {
  const int M = d.M, K = d.K, tid = threadIdx.x, nth = blockDim.x;
  for (int k = tid; k < K; k += nth) {
    s.mu[k] = d.elastic[k] ? 1.0 : d.zeta[k];
    s.Al[k] = d.A[k];
    s.racc[k] = 0.0;
    s.rhacc[k] = 0.0;
  }
  for (int i = tid; i < M * K; i += nth) s.Sacc[i] = 0.0;
  for (int m = tid; m < M; m += nth) {
    s.xi[m] = d.xi[m];
    s.psacc[m] = 0.0;
    s.peacc[m] = 0.0;
    s.Racc[m] = 0.0;
    s.dmax[m] = 0.0;
  }
  __syncthreads();
  // Users grouped by RRH in ascending user order: each wave ranks its lanes
  // with ballots, per-wave counts are scanned in wave order.
  const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;
  for (int base = 0; base < K; base += nth) {
    const int k = base + tid;
    const int a = (k < K) ? s.Al[k] : -1;
    int rank = 0;
    for (int m = 0; m < M; ++m) {
      const unsigned long long bal = __ballot(a == m);
      if (a == m) rank = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) s.wcnt[wave * M + m] = __popcll(bal);
    }
    __syncthreads();
    if (tid < M) {  // running start of group m for each wave of this chunk
      const int m = tid;
      int run = (base == 0) ? 0 : s.gcur[m];
      for (int w = 0; w < nwaves; ++w) {
        const int c = s.wcnt[w * M + m];
        s.wcnt[w * M + m] = run;  // exclusive prefix within group m
        run += c;
      }
      s.gcur[m] = run;
    }
    __syncthreads();
    if (a >= 0) s.grpk[k] = s.wcnt[wave * M + a] + rank;  // rank of k within its group
    __syncthreads();
  }
  if (tid == 0) {
    int off = 0;
    for (int m = 0; m < M; ++m) {
      s.grp_off[m] = off;
      off += s.gcur[m];
    }
    s.grp_off[M] = off;
  }
  __syncthreads();
  for (int k = tid; k < K; k += nth)
    if (s.Al[k] >= 0) s.grp[s.grp_off[s.Al[k]] + s.grpk[k]] = k;
  __syncthreads();
}

struct PassConst {
  double E, delta_v;
  int refit, reset, update, write_out;
};

// One subcarrier of a sweep (update) or of an evaluation pass (no update).
__device__ void subcarrier(const Drop& d, const Sched& sc, const PassConst& pc, Lds& s, int n) {
  const int M = d.M, N = d.N, K = d.K, L = d.L, tid = threadIdx.x, nth = blockDim.x;
  const double sg = d.sigma;

  // 1. gains and slot state into LDS
  for (int i = tid; i < M * K; i += nth) {
    const int m = i / K, k = i - m * K;
    s.g[i] = d.G[((size_t)m * N + n) * K + k];
  }
  for (int i = tid; i < M * L; i += nth) {
    const int m = i / L, q = i - m * L;
    const size_t gi = ((size_t)m * N + n) * L + q;
    s.su[i] = d.sel[gi];
    s.sp[i] = d.p[gi];
    s.sal[i] = pc.reset ? 1.0 : d.al[gi];
    s.sbe[i] = pc.reset ? 0.0 : d.be[gi];
  }
  for (int i = tid; i < M * L * L; i += nth) {
    s.szs[i] = d.zs[(size_t)n * L * L + (size_t)(i / (L * L)) * N * L * L + (i % (L * L))];
    s.szn[i] = 0.0;
  }
  for (int m = tid; m < M; m += nth) s.churn[m] = pc.reset ? 0 : d.churn_sel[(size_t)m * N + n];
  __syncthreads();

  // 2. total power per RRH on n
  for (int m = tid; m < M; m += nth) {
    double acc = 0.0;
    for (int q = 0; q < L; ++q)
      if (s.su[m * L + q] >= 0) acc += s.sp[m * L + q];
    s.Ptot[m] = acc;
  }
  __syncthreads();

  // 3. inter-cell interference as exclusive prefix + suffix over RRHs (no
  //    subtraction), stored as u = (sigma + ICI)/Gamma
  for (int k = tid; k < K; k += nth) {
    double suf = 0.0;
    for (int m = M - 1; m >= 0; --m) {
      s.u[m * K + k] = suf;
      suf += s.Ptot[m] * (double)s.g[m * K + k];
    }
    double pre = 0.0;
    for (int m = 0; m < M; ++m) {
      const double gm = (double)s.g[m * K + k];
      const double ici = pre + s.u[m * K + k];
      pre += s.Ptot[m] * gm;
      s.u[m * K + k] = (sg + ici) / gm;
    }
  }
  __syncthreads();

  // 4. per RRH: decoding order, SINR, rates, SCALE refit, prices
  for (int m = tid; m < M; m += nth) {
    int cnt = 0, slot[kMaxL], usr[kMaxL];
    double uu[kMaxL];
    for (int q = 0; q < L; ++q) {
      const int k = s.su[m * L + q];
      if (k < 0) continue;
      slot[cnt] = q;
      usr[cnt] = k;
      uu[cnt] = s.u[m * K + k];
      ++cnt;
    }
    for (int i = 1; i < cnt; ++i)  // normalised gain descending = u ascending
      for (int j = i; j > 0 && (uu[j - 1] > uu[j] || (uu[j - 1] == uu[j] && usr[j - 1] > usr[j])); --j) {
        double tu = uu[j]; uu[j] = uu[j - 1]; uu[j - 1] = tu;
        int ti = usr[j]; usr[j] = usr[j - 1]; usr[j - 1] = ti;
        ti = slot[j]; slot[j] = slot[j - 1]; slot[j - 1] = ti;
      }
    double pre = 0.0, ps = 0.0, pe = 0.0, Rm = 0.0;
    for (int t = 0; t < cnt; ++t) {
      const int k = usr[t], q = slot[t];
      const double pq = s.sp[m * L + q];
      const double wmk = d.w ? d.w[(size_t)m * K + k] : 1.0;
      const double gam = pq / (uu[t] + pre);
      const double r = log2_1p(gam);
      double a = s.sal[m * L + q], b = s.sbe[m * L + q];
      if (pc.refit && pq > 0.0) {
        a = gam / (1.0 + gam);
        b = r - a * log2(gam);
        s.sal[m * L + q] = a;
        s.sbe[m * L + q] = b;
      }
      const double rh = (pq > 0.0) ? b + a * log2(gam) : 0.0;
      const double cg = wmk * s.mu[k] * a / (kLn2 * (uu[t] + pre));
      s.vslot[m * L + t] = q;
      s.vuser[m * L + t] = k;
      s.vu[m * L + t] = uu[t];
      s.vpre[m * (L + 1) + t] = pre;
      s.vcg[m * L + t] = cg;
      s.vc[m * L + t] = cg / (double)s.g[m * K + k];
      s.racc[k] += wmk * r;  // a user holds at most one slot per subcarrier
      s.rhacc[k] += wmk * rh;
      ps += pq;
      if (d.elastic[k]) {
        pe += pq;
        Rm += wmk * r;
      }
      pre += pq;
    }
    s.vpre[m * (L + 1) + cnt] = pre;
    s.vcnt[m] = cnt;
    s.psacc[m] += ps;
    s.peacc[m] += pe;
    s.Racc[m] += Rm;
    if (pc.write_out) {
      for (int t = 0; t < L; ++t) {
        const size_t o = ((size_t)m * N + n) * L + t;
        d.out_sel[o] = t < cnt ? usr[t] : -1;
        d.out_p[o] = t < cnt ? s.sp[m * L + slot[t]] : 0.0;
      }
      int pi = 0;
      for (int a = 0; a < L; ++a)
        for (int b = a + 1; b < L; ++b, ++pi)
          d.out_zs[((size_t)m * N + n) * d.NP + pi] =
              (b < cnt) ? s.szs[m * L * L + slot[a] * L + slot[b]] : 0.0;
    }
  }
  __syncthreads();
  if (!pc.update) return;

  // 5. inter-cell price and the C14 terms of this subcarrier's pairs
  for (int m = tid; m < M; m += nth) {
    double acc = 0.0;
    for (int j = 0; j < M; ++j) {
      if (j == m) continue;
      for (int t = 0; t < s.vcnt[j]; ++t) acc += s.vc[j * L + t] * (double)s.g[m * K + s.vuser[j * L + t]];
    }
    s.pinter[m] = acc;
    for (int j = 0; j < M; ++j) s.contrib[m * M + j] = 0.0;
    const int cnt = s.vcnt[m];
    for (int a = 0; a < cnt; ++a)
      for (int b = a + 1; b < cnt; ++b) {
        const int ka = s.vuser[m * L + a], kb = s.vuser[m * L + b];
        const double ga = s.g[m * K + ka], gb = s.g[m * K + kb];
        const bool swap = gb > ga || (gb == ga && kb < ka);  // strong = larger raw gain
        const int ps_ = swap ? b : a, pw_ = swap ? a : b;
        const int ks = s.vuser[m * L + ps_], kw = s.vuser[m * L + pw_];
        const double us = s.vu[m * L + ps_], uw = s.vu[m * L + pw_];
        const double om = (us - uw) / (us + uw);  // Omega / nu
        const int sa = s.vslot[m * L + a], sb = s.vslot[m * L + b];
        const double z = s.szs[m * L * L + sa * L + sb];
        const double gs = s.g[m * K + ks], gw = s.g[m * K + kw];
        for (int j = 0; j < M; ++j) {
          if (j == m) continue;
          const double dj = ((double)s.g[j * K + ks] / gs - (double)s.g[j * K + kw] / gw) / (us + uw);
          s.contrib[m * M + j] += z * dj;
        }
        const double zn = fmax(z + pc.delta_v * om, 0.0);
        s.szn[m * L * L + sa * L + sb] = zn;
        s.szn[m * L * L + sb * L + sa] = zn;
      }
  }
  __syncthreads();
  for (int j = tid; j < M; j += nth) {
    double acc = 0.0;
    for (int m = 0; m < M; ++m)
      if (m != j) acc += s.contrib[m * M + j];
    s.psic[j] = acc;
    const int cnt = s.vcnt[j];
    s.vT[j * (L + 1) + cnt] = 0.0;
    for (int t = cnt - 1; t >= 0; --t) s.vT[j * (L + 1) + t] = s.vT[j * (L + 1) + t + 1] + s.vcg[j * L + t];
  }
  __syncthreads();

  // 6. per-triple Lagrangian maximum H for every (m,k)
  for (int i = tid; i < M * K; i += nth) {
    const int m = i / K, k = i - m * K;
    const double u = s.u[i];
    const int cnt = s.vcnt[m];
    int q = -1;
    for (int t = 0; t < cnt; ++t)
      if (s.vuser[m * L + t] == k) q = t;
    double Sb, pin;
    if (q >= 0) {
      Sb = s.vpre[m * (L + 1) + q];
      pin = s.vT[m * (L + 1) + q + 1];
    } else {
      int pos = 0;
      for (int t = 0; t < cnt; ++t) {
        const double ut = s.vu[m * L + t];
        if (ut < u || (ut == u && s.vuser[m * L + t] < k)) ++pos;
      }
      Sb = s.vpre[m * (L + 1) + pos];
      pin = s.vT[m * (L + 1) + pos];
    }
    const double wmu = (d.w ? d.w[(size_t)m * K + k] : 1.0) * s.mu[k];
    const double c = (d.elastic[k] ? pc.E * d.eta[m] : 0.0) + s.xi[m] + pin + s.pinter[m] + s.psic[m];
    double H = 0.0;
    if (wmu > 0.0) {
      const double ainv = u + Sb;
      double pt;
      if (c <= 0.0) {
        pt = d.pmask[m];
      } else {
        const double Wl = wmu / (c * kLn2);
        pt = fmin(fmax(Wl - ainv, 0.0), d.pmask[m]);
      }
      if (pt > 0.0) H = wmu * log2_1p(pt / ainv) - c * pt;
    }
    s.Sacc[i] += H;
    if (s.Al[k] == m) {
      s.Hc[k] = H;
      s.pic[k] = pin;
    }
  }
  __syncthreads();

  // 7. selection, closed-form powers, C14 multipliers follow their pairs
  for (int m = tid; m < M; m += nth) {
    const int cnt = s.vcnt[m];
    const bool frozen = sc.churn > 0 && s.churn[m] >= sc.churn;
    int chosen[kMaxL], np = 0;
    if (frozen) {
      for (int t = 0; t < cnt; ++t)
        if (s.Al[s.vuser[m * L + t]] == m) chosen[np++] = s.vuser[m * L + t];
    } else {
      double bh[kMaxL];
      for (int e = s.grp_off[m]; e < s.grp_off[m + 1]; ++e) {
        const int k = s.grp[e];
        const double h = s.Hc[k];
        if (!(h > 0.0)) continue;
        int t = np < L ? np : L;
        while (t > 0 && (bh[t - 1] < h || (bh[t - 1] == h && chosen[t - 1] > k))) {
          if (t < L) {
            bh[t] = bh[t - 1];
            chosen[t] = chosen[t - 1];
          }
          --t;
        }
        if (t < L) {
          bh[t] = h;
          chosen[t] = k;
          if (np < L) ++np;
        }
      }
      bool same = (np == cnt);
      for (int a = 0; a < np && same; ++a) {
        bool f = false;
        for (int t = 0; t < cnt; ++t) f = f || (s.vuser[m * L + t] == chosen[a]);
        same = f;
      }
      if (!same) s.churn[m]++;
    }
    const double pplus = fmax(s.psic[m], 0.0), pminus = fmax(-s.psic[m], 0.0);
    double dm = s.dmax[m];
    int nu_[kMaxL];
    double np_[kMaxL], na_[kMaxL], nb_[kMaxL];
    int oldslot[kMaxL];
    for (int a = 0; a < np; ++a) {
      const int k = chosen[a];
      int old = -1;
      for (int t = 0; t < cnt; ++t)
        if (s.vuser[m * L + t] == k) old = s.vslot[m * L + t];
      double p_old = 0.0, alph = 1.0, bet = 0.0;
      if (old >= 0) {
        p_old = s.sp[m * L + old];
        alph = s.sal[m * L + old];
        bet = s.sbe[m * L + old];
      }
      const double wmu = (d.w ? d.w[(size_t)m * K + k] : 1.0) * s.mu[k];
      const double cp = (d.elastic[k] ? pc.E * d.eta[m] : 0.0) + s.xi[m] + s.pic[k] + s.pinter[m] + pplus;
      const double num = wmu * alph / kLn2 + p_old * pminus;
      double pn = (cp > 0.0) ? fmin(fmax(num / cp, 0.0), d.pmask[m]) : d.pmask[m];
      if (pn < kPowerFloorRel * d.pmask[m]) pn = 0.0;
      nu_[a] = k;
      np_[a] = pn;
      na_[a] = alph;
      nb_[a] = bet;
      oldslot[a] = old;
      dm = fmax(dm, fabs(pn - p_old) / d.pmask[m]);
    }
    for (int t = 0; t < cnt; ++t) {
      bool kept = false;
      for (int a = 0; a < np; ++a) kept = kept || (nu_[a] == s.vuser[m * L + t]);
      if (!kept) dm = fmax(dm, s.sp[m * L + s.vslot[m * L + t]] / d.pmask[m]);
    }
    s.dmax[m] = dm;
    const size_t base = ((size_t)m * N + n) * L;
    for (int a = 0; a < L; ++a) {
      d.sel[base + a] = a < np ? nu_[a] : -1;
      d.p[base + a] = a < np ? np_[a] : 0.0;
      d.al[base + a] = a < np ? na_[a] : 1.0;
      d.be[base + a] = a < np ? nb_[a] : 0.0;
      for (int b = 0; b < L; ++b) {
        double z = 0.0;
        if (a < np && b < np && a != b && oldslot[a] >= 0 && oldslot[b] >= 0)
          z = s.szn[m * L * L + oldslot[a] * L + oldslot[b]];
        d.zs[(base + a) * L + b] = z;
      }
    }
    d.churn_sel[(size_t)m * N + n] = s.churn[m];
  }
  __syncthreads();
}

// Per-workgroup partials after its subcarriers.
__device__ void write_partials(const Drop& d, const Lds& s, int b) {
  const int M = d.M, K = d.K, tid = threadIdx.x, nth = blockDim.x;
  for (int i = tid; i < M * K; i += nth) d.S_part[(size_t)b * M * K + i] = s.Sacc[i];
  for (int k = tid; k < K; k += nth) {
    d.r_part[(size_t)b * K + k] = s.racc[k];
    d.rh_part[(size_t)b * K + k] = s.rhacc[k];
  }
  for (int m = tid; m < M; m += nth) {
    d.psum_part[(size_t)b * M + m] = s.psacc[m];
    d.pel_part[(size_t)b * M + m] = s.peacc[m];
  }
  if (tid == 0) {
    double R = 0.0, dm = 0.0;
    for (int m = 0; m < M; ++m) {
      R += s.Racc[m];
      dm = fmax(dm, s.dmax[m]);
    }
    d.R_part[b] = R;
    d.d_part[b] = dm;
  }
}

// Sums (or maxima) over workgroups g of v(g, m) = base[g*gs + m*ms] for
// m < M, in a fixed order: strided partial sums per (m, chunk), then a tree
// over chunks.  Result in out[m] (LDS), visible to all threads on return.
template <bool kMax>
__device__ void reduce_groups(Lds& s, const double* base, int G, int M, size_t gs, size_t ms,
                              double* out) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int chunks = nth / M;
  if (tid < M * chunks) {
    const int m = tid % M, c = tid / M;
    double acc = 0.0;
    for (int g = c; g < G; g += chunks) {
      const double v = base[(size_t)g * gs + (size_t)m * ms];
      acc = kMax ? fmax(acc, v) : acc + v;
    }
    s.red[tid] = acc;
  }
  __syncthreads();
  for (int st = 1; st < chunks; st <<= 1) {
    if (tid < M * chunks) {
      const int c = tid / M;
      if ((c % (2 * st)) == 0 && c + st < chunks) {
        const double o = s.red[tid + st * M];
        s.red[tid] = kMax ? fmax(s.red[tid], o) : s.red[tid] + o;
      }
    }
    __syncthreads();
  }
  if (tid < M) out[tid] = s.red[tid];
  __syncthreads();
}

// Reductions across workgroups: users k = b, b+G, ... per workgroup;
// workgroup 0 also does the per-RRH and scalar sums.
__device__ void reduce_pass(const Drop& d, const Sched& sc, const Ctrl& c, Lds& s, int b, int G,
                            bool update, double delta_v) {
  const int M = d.M, K = d.K, tid = threadIdx.x;
  const int par = c.pass & 1;
  int changes = 0;
  if (b == 0 && tid == 0) store_shared(&d.chg_count[par ^ 1], 0);  // next pass's counter
  for (int k = b; k < K; k += G) {
    reduce_groups<false>(s, d.r_part + k, G, 1, K, 0, s.tmp);
    reduce_groups<false>(s, d.rh_part + k, G, 1, K, 0, s.tmp + 1);
    if (update) reduce_groups<false>(s, d.S_part + k, G, M, (size_t)M * K, K, s.tmp + 2);
    if (tid == 0) {
      const double r = s.tmp[0], rh = s.tmp[1];
      d.user_rate[k] = r;
      if (update) {
        double best = -INFINITY;
        int bm = 0;
        for (int m = 0; m < M; ++m)
          if (s.tmp[2 + m] > best) {
            best = s.tmp[2 + m];
            bm = m;
          }
        int ch_A = c.reset ? 0 : d.churn_A[k];
        const int before = d.A[k];
        if (!(sc.churn > 0 && ch_A >= sc.churn)) {
          int after = before;
          if (best > 0.0)
            after = bm;
          else if (d.elastic[k])
            after = -1;
          if (after != before) {
            d.A[k] = after;
            ++ch_A;
            ++changes;
          }
        }
        d.churn_A[k] = ch_A;
        if (!d.elastic[k]) {
          const double viol = fmin(fmax((d.psi[k] - rh) / d.psi[k], -1.0), 1.0);
          d.zeta[k] = fmax(d.zeta[k] + delta_v * viol, 0.0);
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && changes > 0)
    __hip_atomic_fetch_add(&d.chg_count[par], changes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (b == 0) {
    // per-RRH sums, xi' step, R, P, max delta (fixed-order trees)
    reduce_groups<false>(s, d.psum_part, G, M, M, 1, s.psacc);
    reduce_groups<false>(s, d.pel_part, G, M, M, 1, s.peacc);
    reduce_groups<false>(s, d.R_part, G, 1, 1, 0, s.tmp);
    reduce_groups<true>(s, d.d_part, G, 1, 1, 0, s.tmp + 1);
    if (update)
      for (int m = tid; m < M; m += blockDim.x) {
        const double ps = s.psacc[m];
        const double scale = (double)d.N * d.L / (kLn2 * d.pmax[m]);
        d.xi[m] = fmax(d.xi[m] + delta_v * scale * (ps - d.pmax[m]) / d.pmax[m], 0.0);
      }
    if (tid == 0) {
      double P = d.pstatic;
      for (int m = 0; m < M; ++m) P += d.eta[m] * s.peacc[m];
      store_shared(&d.red[0], s.tmp[0]);
      store_shared(&d.red[1], P);
      store_shared(&d.red[2], s.tmp[1]);
    }
  }
}

// Loop control, identical in every workgroup (mirrors the Dinkelbach and
// dual-loop stopping rules).
__device__ void control(const Drop& d, const Sched& sc, Ctrl& c, int G) {
  const double R = load_shared(&d.red[0]), P = load_shared(&d.red[1]), dm = load_shared(&d.red[2]);
  if (c.mode == kSweep) {
    const int changes = load_shared(&d.chg_count[c.pass & 1]);
    c.v += 1;
    c.total += 1;
    c.reset = 0;
    const double delta = changes > 0 ? INFINITY : dm;
    bool end = c.v >= sc.sweeps;
    if (isnan(delta)) {
      c.flags |= ALLOC_NONFINITE;
      end = true;
    }
    if (!sc.fixed && delta < sc.tol_dual) end = true;
    if (end) c.mode = kEval;
  } else if (c.mode == kEval) {
    c.R = R;
    c.P = P;
    const double F = R - c.E * P;
    c.i += 1;
    if (c.flags & ALLOC_NONFINITE) {
      c.mode = kDone;
    } else if (F <= sc.tol_d * R) {
      c.mode = kDone;
    } else if (c.i >= sc.max_d) {
      c.flags |= ALLOC_NOT_CONVERGED;
      c.mode = kDone;
    } else {
      c.E = R / P;
      c.v = 0;
      c.reset = 1;
      c.mode = kSweep;
    }
  }
}

__global__ void __launch_bounds__(kBlock) solve_kernel(Drop d, Sched sc) {
  extern __shared__ __align__(16) char smem[];
  Lds s = carve(smem, d.M, d.K, d.L);
  cg::grid_group grid = cg::this_grid();
  const int b = blockIdx.x, G = gridDim.x;
  Ctrl c = *d.ctrl;
  while (c.mode != kDone) {
    const bool update = c.mode == kSweep;
    PassConst pc;
    pc.E = c.E;
    pc.delta_v = sc.step0 / sqrt(1.0 + (double)c.v);
    pc.refit = update && sc.refit_period > 0 && (c.v % sc.refit_period) == 0;
    pc.reset = update && c.reset;
    pc.update = update;
    pc.write_out = !update;
    begin_pass(d, s);
    for (int n = b; n < d.N; n += G) subcarrier(d, sc, pc, s, n);
    write_partials(d, s, b);
    grid.sync();
    reduce_pass(d, sc, c, s, b, G, update, pc.delta_v);
    grid.sync();
    control(d, sc, c, G);
    c.pass += 1;
    if (b == 0 && threadIdx.x == 0) *d.ctrl = c;
  }
}

// ------------------------------------------------------------ initial point

// Cold start, part 1: per (m,k) the sum over n of log2(1 + Gamma pmask/sigma),
// summed in increasing n; part 2 picks the best RRH per user.
__global__ void cold_assoc_kernel(Drop d, double* snr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.M * d.K) return;
  const int m = i / d.K, k = i - m * d.K;
  double acc = 0.0;
  for (int n = 0; n < d.N; ++n)
    acc += log2_1p((double)d.G[((size_t)m * d.N + n) * d.K + k] * d.pmask[m] / d.sigma);
  snr[i] = acc;
}

__global__ void cold_pick_kernel(Drop d, const double* snr, const double* p0sum) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.K) return;
  int best = 0;
  double bv = -1.0;
  for (int m = 0; m < d.M; ++m) {
    const double v = snr[(size_t)m * d.K + k];
    if (v > bv) {
      bv = v;
      best = m;
    }
  }
  if (p0sum) {  // warm start: largest total initial power, if any
    int wb = -1;
    double wv = 0.0;
    for (int m = 0; m < d.M; ++m) {
      const double v = p0sum[(size_t)m * d.K + k];
      if (v > wv) {
        wv = v;
        wb = m;
      }
    }
    if (wb >= 0) best = wb;
  }
  d.A[k] = best;
  d.churn_A[k] = 0;
  d.zeta[k] = d.elastic[k] ? 0.0 : 1.0;
}

// Strongest l users of RRH m on n (by Gamma, or by initial power when warm).
__global__ void cold_select_kernel(Drop d, const double* p0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.M * d.N) return;
  const int m = i / d.N, n = i - m * d.N, L = d.L;
  int bk[kMaxL];
  double bv[kMaxL];
  int cnt = 0;
  for (int k = 0; k < d.K; ++k) {
    if (d.A[k] != m) continue;
    double v;
    if (p0) {
      v = p0[((size_t)m * d.N + n) * d.K + k];
      if (!(v > 0.0)) continue;
    } else {
      v = d.G[((size_t)m * d.N + n) * d.K + k];
    }
    int t = cnt < L ? cnt : L;
    while (t > 0 && (bv[t - 1] < v || (bv[t - 1] == v && bk[t - 1] > k))) {
      if (t < L) {
        bv[t] = bv[t - 1];
        bk[t] = bk[t - 1];
      }
      --t;
    }
    if (t < L) {
      bv[t] = v;
      bk[t] = k;
      if (cnt < L) ++cnt;
    }
  }
  const size_t base = ((size_t)m * d.N + n) * L;
  for (int a = 0; a < L; ++a) {
    d.sel[base + a] = a < cnt ? bk[a] : -1;
    double pa = 0.0;
    if (a < cnt) pa = p0 ? fmin(bv[a], d.pmask[m]) : d.pmax[m] / ((double)d.N * L);
    d.p[base + a] = pa;
    d.al[base + a] = 1.0;
    d.be[base + a] = 0.0;
    for (int b = 0; b < L; ++b) d.zs[(base + a) * L + b] = 0.0;
  }
  d.churn_sel[i] = 0;
}

__global__ void p0_sum_kernel(Drop d, const double* p0, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.M * d.K) return;
  const int m = i / d.K, k = i - m * d.K;
  double acc = 0.0;
  for (int n = 0; n < d.N; ++n) acc += p0[((size_t)m * d.N + n) * d.K + k];
  out[i] = acc;
}

// Dense [M][N][K] powers from the decoding-order slots.
__global__ void dense_kernel(Drop d, float* out) {
  const size_t total = (size_t)d.M * d.N * d.K;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = 0.0f;
}

__global__ void scatter_kernel(Drop d, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.M * d.N) return;
  const int m = i / d.N, n = i - m * d.N;
  for (int a = 0; a < d.L; ++a) {
    const int k = d.out_sel[(size_t)i * d.L + a];
    if (k >= 0) out[((size_t)m * d.N + n) * d.K + k] = (float)d.out_p[(size_t)i * d.L + a];
  }
}

}  // namespace

// ==================================================================== host

struct alloc_ctx {
  int device;
  hipStream_t stream;
  char* ws;         // device workspace
  size_t ws_bytes;
  int cus;
  size_t lds_max;
  int timing;
  hipEvent_t ev0, ev1;
  double last_ms;
};

namespace {

// Minimum rate (Sec. II-B, C9): Psi = lambda zbar / (B_n (1 - 1/(x + sqrt(1+x^2)))),
// x = lambda T -- the smaller root of the delay quadratic without cancellation.
double min_rate(double arrival_bps, double delay_s, double packet_bits, double bw_hz) {
  const double lambda = arrival_bps / packet_bits;
  const double x = lambda * delay_s;
  return (arrival_bps / (1.0 - 1.0 / (x + sqrt(1.0 + x * x)))) / bw_hz;
}

int validate(const alloc_problem* pb, const alloc_params* prm) {
  if (!pb || !prm) return ALLOC_EINVAL;
  if (pb->M < 1 || pb->N < 1 || pb->K < 1 || pb->l < 1 || pb->l > pb->K) return ALLOC_EINVAL;
  if (!pb->gain || !pb->user_type || !pb->pmax_w || !pb->eta) return ALLOC_EINVAL;
  if (!(pb->noise_w > 0) || !(pb->bw_hz > 0) || !(pb->packet_bits > 0)) return ALLOC_EINVAL;
  if (!std::isfinite(pb->noise_w)) return ALLOC_EINVAL;
  if (pb->M > kMaxM || pb->l > kMaxL || pb->K > kMaxK || pb->M * pb->K > kMaxMK) return ALLOC_ETOOBIG;
  if (prm->sweeps_per_dinkelbach < 1 || prm->max_dinkelbach < 1 || prm->max_groups < 0) return ALLOC_EINVAL;
  for (int m = 0; m < pb->M; ++m) {
    if (!(pb->pmax_w[m] > 0) || !std::isfinite(pb->pmax_w[m])) return ALLOC_EINVAL;
    if (!(pb->eta[m] > 0) || !std::isfinite(pb->eta[m])) return ALLOC_EINVAL;
    if (pb->pmask_w && !(pb->pmask_w[m] > 0)) return ALLOC_EINVAL;
  }
  for (int k = 0; k < pb->K; ++k) {
    if (pb->user_type[k] > 1) return ALLOC_EINVAL;
    if (pb->user_type[k] == 1) {
      if (!pb->arrival_bps || !pb->delay_s) return ALLOC_EINVAL;
      if (!(pb->arrival_bps[k] > 0) || !(pb->delay_s[k] > 0)) return ALLOC_EINVAL;
      if (!std::isfinite(pb->arrival_bps[k]) || !std::isfinite(pb->delay_s[k])) return ALLOC_EINVAL;
    }
  }
  if (pb->weight)
    for (int i = 0; i < pb->M * pb->K; ++i)
      if (!(pb->weight[i] >= 0) || !std::isfinite(pb->weight[i])) return ALLOC_EINVAL;
  return ALLOC_OK;
}

struct Layout {
  size_t off[48];
  int n = 0;
  size_t total = 0;
  size_t add(size_t bytes) {
    const size_t o = total;
    off[n++] = o;
    total += (bytes + 255) & ~size_t(255);
    return o;
  }
};

}  // namespace

extern "C" {

void alloc_params_default(alloc_params* p) {
  p->max_dinkelbach = 20;
  p->sweeps_per_dinkelbach = 200;
  p->refit_period = 1;
  p->fixed_count = 1;
  p->churn_limit = 8;
  p->tol_dinkelbach = 1e-6;
  p->tol_dual = 1e-7;
  p->step0 = 0.1;
  p->flags = 0;
  p->max_groups = 0;
}

int alloc_ctx_set_timing(alloc_ctx* ctx, int enable) {
  if (!ctx) return ALLOC_EINVAL;
  ctx->timing = enable != 0;
  return ALLOC_OK;
}

double alloc_ctx_last_kernel_ms(alloc_ctx* ctx) { return ctx ? ctx->last_ms : -1.0; }

const char* alloc_strerror(int code) {
  switch (code) {
    case ALLOC_OK: return "ok";
    case ALLOC_EINVAL: return "invalid argument";
    case ALLOC_ENOMEM: return "device memory allocation failed";
    case ALLOC_EDEVICE: return "HIP runtime error";
    case ALLOC_ETOOBIG: return "problem exceeds a kernel limit (M<=32, l<=4, K<=1024, M*K<=4608)";
    default: return "unknown error";
  }
}

int alloc_ctx_create(int device, void* hip_stream, alloc_ctx** out) {
  if (!out) return ALLOC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return ALLOC_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return ALLOC_EDEVICE;
  alloc_ctx* c = new alloc_ctx;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->cus = prop.multiProcessorCount;
  c->lds_max = prop.sharedMemPerBlock;
  c->timing = 0;
  c->last_ms = -1.0;
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    delete c;
    return ALLOC_EDEVICE;
  }
  if (hipFuncSetAttribute((const void*)solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)c->lds_max) != hipSuccess) {
    delete c;
    return ALLOC_EDEVICE;
  }
  *out = c;
  return ALLOC_OK;
}

void alloc_ctx_destroy(alloc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->ws) (void)hipFree(c->ws);
  (void)hipEventDestroy(c->ev0);
  (void)hipEventDestroy(c->ev1);
  delete c;
}

int alloc_solve(alloc_ctx* ctx, const alloc_problem* pb, const alloc_params* prm,
                const alloc_warm* warm, alloc_result* res) {
  if (!ctx || !res) return ALLOC_EINVAL;
  int rc = validate(pb, prm);
  if (rc != ALLOC_OK) return rc;
  const int M = pb->M, N = pb->N, K = pb->K, L = pb->l, NP = L * (L - 1) / 2;
  const size_t lds = lds_bytes(M, K, L);
  if (lds > ctx->lds_max) return ALLOC_ETOOBIG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ALLOC_EDEVICE;
  const bool gain_dev = prm->flags & ALLOC_GAIN_ON_DEVICE;
  const bool out_dev = prm->flags & ALLOC_OUT_ON_DEVICE;
  if (!gain_dev) {  // host gains are validated here; device gains by the caller's contract
    const size_t n3 = (size_t)M * N * K;
    for (size_t i = 0; i < n3; ++i)
      if (!(pb->gain[i] > 0.0f) || !std::isfinite(pb->gain[i])) return ALLOC_EINVAL;
  }

  // grid: one workgroup per subcarrier up to what can be co-resident
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)solve_kernel, kBlock, lds) !=
      hipSuccess)
    return ALLOC_EDEVICE;
  if (per_cu < 1) return ALLOC_ETOOBIG;
  int G = std::min(N, per_cu * ctx->cus);
  if (prm->max_groups > 0) G = std::min(G, prm->max_groups);

  // host-side constants (FP64)
  std::vector<double> psi(K, 0.0), pmask(M), w;
  std::vector<uint8_t> el(K);
  for (int k = 0; k < K; ++k) {
    el[k] = pb->user_type[k] == 0;
    if (!el[k]) psi[k] = min_rate(pb->arrival_bps[k], pb->delay_s[k], pb->packet_bits, pb->bw_hz);
  }
  for (int m = 0; m < M; ++m) pmask[m] = pb->pmask_w ? pb->pmask_w[m] : pb->pmax_w[m] / N;
  const double pstatic = pb->p_fiber_hpn + (M - 1) * pb->p_fiber_lpn + (M - 1) * pb->p_circuit_lpn +
                         pb->p_circuit_hpn;

  // workspace layout
  const size_t n3 = (size_t)M * N * K, ns = (size_t)M * N * L;
  Layout lay;
  const size_t oG = lay.add(gain_dev ? 0 : sizeof(float) * n3);
  const size_t oPsi = lay.add(sizeof(double) * K);
  const size_t oEl = lay.add(K);
  const size_t oPmax = lay.add(sizeof(double) * M);
  const size_t oEta = lay.add(sizeof(double) * M);
  const size_t oPmask = lay.add(sizeof(double) * M);
  const size_t oW = lay.add(pb->weight ? sizeof(double) * M * K : 0);
  const size_t oA = lay.add(sizeof(int) * K);
  const size_t oSel = lay.add(sizeof(int) * ns);
  const size_t oP = lay.add(sizeof(double) * ns);
  const size_t oAl = lay.add(sizeof(double) * ns);
  const size_t oBe = lay.add(sizeof(double) * ns);
  const size_t oZs = lay.add(sizeof(double) * ns * L);
  const size_t oXi = lay.add(sizeof(double) * M);
  const size_t oZeta = lay.add(sizeof(double) * K);
  const size_t oChS = lay.add(sizeof(int) * M * N);
  const size_t oChA = lay.add(sizeof(int) * K);
  const size_t oSp = lay.add(sizeof(double) * G * M * K);
  const size_t oRp = lay.add(sizeof(double) * G * K);
  const size_t oRhp = lay.add(sizeof(double) * G * K);
  const size_t oPsp = lay.add(sizeof(double) * G * M);
  const size_t oPep = lay.add(sizeof(double) * G * M);
  const size_t oRP = lay.add(sizeof(double) * G);
  const size_t oDp = lay.add(sizeof(double) * G);
  const size_t oChg = lay.add(sizeof(int) * 2);
  const size_t oRed = lay.add(sizeof(double) * 4);
  const size_t oUr = lay.add(sizeof(double) * K);
  const size_t oOs = lay.add(sizeof(int) * ns);
  const size_t oOp = lay.add(sizeof(double) * ns);
  const size_t oOz = lay.add(sizeof(double) * (size_t)M * N * (NP > 0 ? NP : 1));
  const size_t oCtrl = lay.add(sizeof(Ctrl));
  const size_t oSnr = lay.add(sizeof(double) * M * K);
  const size_t oP0 = lay.add(warm && warm->p0 ? sizeof(double) * n3 : 0);
  const size_t oP0s = lay.add(warm && warm->p0 ? sizeof(double) * M * K : 0);
  if (lay.total > ctx->ws_bytes) {
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (hipMalloc((void**)&ctx->ws, lay.total) != hipSuccess) return ALLOC_ENOMEM;
    ctx->ws_bytes = lay.total;
  }
  char* ws = ctx->ws;
  hipStream_t st = ctx->stream;
  auto h2d = [&](size_t off, const void* src, size_t bytes) {
    return bytes == 0 || hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  bool ok = true;
  if (!gain_dev) ok = ok && h2d(oG, pb->gain, sizeof(float) * n3);
  ok = ok && h2d(oPsi, psi.data(), sizeof(double) * K) && h2d(oEl, el.data(), K) &&
       h2d(oPmax, pb->pmax_w, sizeof(double) * M) && h2d(oEta, pb->eta, sizeof(double) * M) &&
       h2d(oPmask, pmask.data(), sizeof(double) * M);
  if (pb->weight) ok = ok && h2d(oW, pb->weight, sizeof(double) * M * K);
  if (warm && warm->p0) ok = ok && h2d(oP0, warm->p0, sizeof(double) * n3);
  Ctrl c0;
  memset(&c0, 0, sizeof c0);
  c0.mode = kSweep;
  c0.reset = 1;
  ok = ok && h2d(oCtrl, &c0, sizeof c0);
  static const int zeros2[2] = {0, 0};
  ok = ok && h2d(oChg, zeros2, sizeof zeros2);
  if (!ok) return ALLOC_EDEVICE;

  Drop d;
  d.M = M; d.N = N; d.K = K; d.L = L; d.NP = NP;
  d.G = gain_dev ? pb->gain : (const float*)(ws + oG);
  d.psi = (const double*)(ws + oPsi);
  d.elastic = (const uint8_t*)(ws + oEl);
  d.pmax = (const double*)(ws + oPmax);
  d.eta = (const double*)(ws + oEta);
  d.pmask = (const double*)(ws + oPmask);
  d.w = pb->weight ? (const double*)(ws + oW) : nullptr;
  d.sigma = pb->noise_w;
  d.pstatic = pstatic;
  d.A = (int*)(ws + oA);
  d.sel = (int*)(ws + oSel);
  d.p = (double*)(ws + oP);
  d.al = (double*)(ws + oAl);
  d.be = (double*)(ws + oBe);
  d.zs = (double*)(ws + oZs);
  d.xi = (double*)(ws + oXi);
  d.zeta = (double*)(ws + oZeta);
  d.churn_sel = (int*)(ws + oChS);
  d.churn_A = (int*)(ws + oChA);
  d.S_part = (double*)(ws + oSp);
  d.r_part = (double*)(ws + oRp);
  d.rh_part = (double*)(ws + oRhp);
  d.psum_part = (double*)(ws + oPsp);
  d.pel_part = (double*)(ws + oPep);
  d.R_part = (double*)(ws + oRP);
  d.d_part = (double*)(ws + oDp);
  d.chg_count = (int*)(ws + oChg);
  d.red = (double*)(ws + oRed);
  d.user_rate = (double*)(ws + oUr);
  d.out_sel = (int*)(ws + oOs);
  d.out_p = (double*)(ws + oOp);
  d.out_zs = (double*)(ws + oOz);
  d.ctrl = (Ctrl*)(ws + oCtrl);

  // initial point
  if (hipMemsetAsync(d.xi, 0, sizeof(double) * M, st) != hipSuccess) return ALLOC_EDEVICE;
  const double* p0 = (warm && warm->p0) ? (const double*)(ws + oP0) : nullptr;
  double* p0s = p0 ? (double*)(ws + oP0s) : nullptr;
  const int tb = 256;
  hipLaunchKernelGGL(cold_assoc_kernel, dim3((M * K + tb - 1) / tb), dim3(tb), 0, st, d,
                     (double*)(ws + oSnr));
  if (p0) hipLaunchKernelGGL(p0_sum_kernel, dim3((M * K + tb - 1) / tb), dim3(tb), 0, st, d, p0, p0s);
  hipLaunchKernelGGL(cold_pick_kernel, dim3((K + tb - 1) / tb), dim3(tb), 0, st, d,
                     (const double*)(ws + oSnr), (const double*)p0s);
  hipLaunchKernelGGL(cold_select_kernel, dim3((M * N + tb - 1) / tb), dim3(tb), 0, st, d, p0);
  if (warm && (warm->xi0 || warm->zeta0)) {
    std::vector<double> xi0(M, 0.0), z0(K, 0.0);
    if (warm->xi0)
      for (int m = 0; m < M; ++m) xi0[m] = std::max(warm->xi0[m], 0.0);
    if (warm->xi0 && !h2d(oXi, xi0.data(), sizeof(double) * M)) return ALLOC_EDEVICE;
    if (warm->zeta0) {
      for (int k = 0; k < K; ++k) z0[k] = el[k] ? 0.0 : std::max(warm->zeta0[k], 0.0);
      if (!h2d(oZeta, z0.data(), sizeof(double) * K)) return ALLOC_EDEVICE;
    }
  }
  if (hipGetLastError() != hipSuccess) return ALLOC_EDEVICE;

  Sched sc;
  sc.max_d = prm->max_dinkelbach;
  sc.sweeps = prm->sweeps_per_dinkelbach;
  sc.refit_period = prm->refit_period;
  sc.fixed = prm->fixed_count;
  sc.churn = prm->churn_limit;
  sc.tol_d = prm->tol_dinkelbach;
  sc.tol_dual = prm->tol_dual;
  sc.step0 = prm->step0;
  void* args[] = {(void*)&d, (void*)&sc};
  if (ctx->timing && hipEventRecord(ctx->ev0, st) != hipSuccess) return ALLOC_EDEVICE;
  if (hipLaunchCooperativeKernel((const void*)solve_kernel, dim3(G), dim3(kBlock), args, lds, st) !=
      hipSuccess)
    return ALLOC_EDEVICE;
  if (ctx->timing && hipEventRecord(ctx->ev1, st) != hipSuccess) return ALLOC_EDEVICE;

  // outputs
  const hipMemcpyKind kind = out_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  auto d2o = [&](void* dst, const void* src, size_t bytes) {
    return !dst || hipMemcpyAsync(dst, src, bytes, kind, st) == hipSuccess;
  };
  ok = d2o(res->sel, d.out_sel, sizeof(int) * ns) && d2o(res->slot_power, d.out_p, sizeof(double) * ns) &&
       d2o(res->rrh_of_user, d.A, sizeof(int) * K) && d2o(res->xi, d.xi, sizeof(double) * M) &&
       d2o(res->zeta, d.zeta, sizeof(double) * K) && d2o(res->user_rate, d.user_rate, sizeof(double) * K);
  if (NP > 0) ok = ok && d2o(res->zeta_sic, d.out_zs, sizeof(double) * M * N * NP);
  if (!ok) return ALLOC_EDEVICE;
  if (res->power) {
    float* dense = res->power;
    float* tmp = nullptr;
    if (!out_dev) {
      if (hipMallocAsync((void**)&tmp, sizeof(float) * n3, st) != hipSuccess) return ALLOC_ENOMEM;
      dense = tmp;
    }
    hipLaunchKernelGGL(dense_kernel, dim3(std::min<size_t>((n3 + tb - 1) / tb, 65535)), dim3(tb), 0, st, d,
                       dense);
    hipLaunchKernelGGL(scatter_kernel, dim3((M * N + tb - 1) / tb), dim3(tb), 0, st, d, dense);
    if (tmp) {
      if (hipMemcpyAsync(res->power, tmp, sizeof(float) * n3, hipMemcpyDeviceToHost, st) != hipSuccess)
        return ALLOC_EDEVICE;
      (void)hipFreeAsync(tmp, st);
    }
  }
  Ctrl cf;
  if (hipMemcpyAsync(&cf, d.ctrl, sizeof cf, hipMemcpyDeviceToHost, st) != hipSuccess) return ALLOC_EDEVICE;
  std::vector<double> ur(K);
  if (hipMemcpyAsync(ur.data(), d.user_rate, sizeof(double) * K, hipMemcpyDeviceToHost, st) != hipSuccess)
    return ALLOC_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return ALLOC_EDEVICE;
  ctx->last_ms = -1.0;
  if (ctx->timing) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) != hipSuccess) return ALLOC_EDEVICE;
    ctx->last_ms = ms;
  }
  uint32_t flags = cf.flags;
  for (int k = 0; k < K; ++k) {
    if (!el[k] && ur[k] < psi[k] * (1.0 - 1e-6)) flags |= ALLOC_QOS_INFEASIBLE;
    if (!std::isfinite(ur[k])) flags |= ALLOC_NONFINITE;
  }
  res->ee = cf.P > 0.0 ? cf.R / cf.P : 0.0;
  res->rate_sum = cf.R;
  res->power_sum = cf.P;
  res->dinkelbach_iters = cf.i;
  res->sweeps = cf.total;
  res->status_flags = flags;
  return ALLOC_OK;
}

}  // extern "C"
