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
#include "ctx.h"
#include "logs.h"

namespace cg = cooperative_groups;

// Fixed workspace of alloc_solve_noalloc (callers that cannot allocate):
// every device the library runs on holds one copy, at its own address, until
// the process ends.  Host code never uses this name as an address: each
// context looks up its device's copy once (hipGetSymbolAddress, in
// alloc_ctx_create) and passes that pointer to the kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr double kLn2 = 0.69314718055994530942;
constexpr int kMaxL = 4;
constexpr int kMaxM = 32;
constexpr int kMaxK = 1024;
constexpr int kMaxMK = 4608;
constexpr int kBlock = 1024;     // largest workgroup of the batched solver
constexpr int kGridBlock = 512;  // workgroup of the grid solver
// Closed-form powers below this fraction of the mask become exactly zero, so
// decaying powers never reach the subnormal range.
constexpr double kPowerFloorRel = 1e-20;

// Feasibility of an evaluated state: C13 r_k >= Psi_k (1 - kQosTol), C12
// sum p <= pmax (1 + kBudgetTol), C14 pair margin <= kSicTol.  Two nonzero
// violations within kViolRel of each other rank as equal.
constexpr double kQosTol = 1e-6;
constexpr double kBudgetTol = 1e-6;
constexpr double kSicTol = 1e-9;
constexpr double kViolRel = 1e-6;

// kRepair: dissolve the C14 pairs the returned state still breaks; kFinal:
// evaluate the repaired state.
enum Mode : int { kSweep = 0, kEval = 1, kDone = 2, kRepair = 3, kFinal = 4 };

// Loop-control state.  Every workgroup holds an identical copy.
//
// The dual sweeps are not a descent method, so a Dinkelbach step returns the
// best state it visited: feasible (C12-C14) before infeasible, less C12/C13
// violation first, then less C14 violation, then the larger R - E P.  The
// primal state (association, selection, powers, SCALE coefficients, C14
// multipliers) lives in three buffers: the one the next pass reads (rd), the
// one a sweep writes (wr) and the best state of the step (best).  After a
// sweep its output becomes the state to read; the state it read becomes the
// best or is free for the next sweep's output: a pointer rotation, no copies.
struct Ctrl {
  double E;           // Dinkelbach parameter of the current step
  double R, P;        // rate and power of the last evaluated state
  double Vq, Vp, Vs;  // its violations of C13, C12, C14
  double bV, bV2;     // best state of the step: C12 + C13 and C14 violation,
  double bf, bR;      //   R - E P and R
  int i;              // Dinkelbach steps completed
  int v;              // sweeps done in the current step
  int mode;
  int total;          // sweeps done in total
  int reset;          // next sweep starts a Dinkelbach step
  int pass;           // passes (sweeps and evaluations) done
  int rd, wr, best;   // state buffers (0..2)
  int have_best;      // best is set in this step
  int stall;          // sweeps since the last gain of the best
  int first_eval;     // the next evaluation is the warm start's p^0
  uint32_t flags;
};

struct Sched {
  int max_d, sweeps, refit_period, fixed, stall, tile;
  int sdev;  // grid solver: association sums in S_part's row of the workgroup
  double tol_d, tol_dual, step0, qos_down;
  double tie_rel;  // > 0: count near-tie decisions in Drop::ties
};

// Reduced values of one pass, the input of the loop control.
struct Eval {
  double R, P;        // weighted elastic rate, power of the state read
  double Vq, Vp, Vs;  // its violations of C13, C12, C14
  double dm;          // largest |dp|/pmask and C14 multiplier step / delta
  double xres, zres;  // largest xi' and zeta' steps / their step sizes
  int changes;        // users whose association the sweep changed
};

// Division by a run-time invariant d by multiply-high and shifts
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Fig. 4.1): exact for every 32-bit numerator.
struct Div {
  uint32_t m, s1, s2;
  __host__ __device__ uint32_t div(uint32_t n) const {
    const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
    return (t + ((n - t) >> s1)) >> s2;
  }
};

__host__ __device__ inline Div make_div(uint32_t d) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;  // ceil(log2 d)
  Div r;
  r.m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
  r.s1 = l < 1 ? l : 1;
  r.s2 = l > 0 ? l - 1 : 0;
  return r;
}

// Divisors of the per-subcarrier item loops of one drop.
struct Divs {
  Div K, M, L, MK, ML, MLL, LL, MM;
  Div K4, MK4;  // K/4 and M*K/4 (when K is a multiple of 4)
};

inline Divs make_divs(int M, int K, int L) {
  Divs v;
  v.K = make_div(K);
  v.M = make_div(M);
  v.L = make_div(L);
  v.MK = make_div(M * K);
  v.ML = make_div(M * L);
  v.MLL = make_div(M * L * L);
  v.LL = make_div(L * L);
  v.MM = make_div(M * M);
  v.K4 = make_div(K % 4 == 0 ? K / 4 : 1);
  v.MK4 = make_div(K % 4 == 0 ? M * K / 4 : 1);
  return v;
}

// Device view of one drop: inputs, state, per-workgroup partials.
struct Drop {
  int M, N, K, L, NP;
  Divs dv;                 // divisors of the item loops
  const float* G;          // [M][N][K]
  const double* psi;       // [K] minimum rate (0 elastic)
  const uint8_t* elastic;  // [K]
  const double* pmax;      // [M]
  const double* eta;       // [M]
  const double* pmask;     // [M]
  const double* w;         // [M][K] or nullptr (all ones)
  double sigma, pstatic;
  // primal state, three buffers each (see Ctrl)
  int* A;                  // [3][K] association
  int* sel;                // [3][M][N][L] storage order
  double* p;               // [3][M][N][L]
  double* al;              // [3][M][N][L]
  double* be;              // [3][M][N][L]
  double* zs;              // [3][M][N][L][L]
  double* xi;              // [M]
  double* zeta;            // [K]
  // partials, one row per workgroup
  double* S_part;          // [G][M][K] association metric
  double* r_part;          // [G][K] true rate
  double* rh_part;         // [G][K] SCALE surrogate rate
  double* psum_part;       // [G][M] power, all users
  double* pel_part;        // [G][M] power, elastic users
  double* R_part;          // [G] weighted elastic rate
  double* d_part;          // [G] max |dp|/pmask
  double* sv_part;         // [G] C14 violation
  double* vq_part;         // [G] C13 violation of the workgroup's users
  double* zr_part;         // [G] largest zeta' step of its users / delta
  int* chg_count;          // [2] association changes, indexed by pass parity
  double* red;             // [8] R, P, dm, xres, Vp, Vs (written by workgroup 0)
  double* user_rate;       // [K]
  // decoding-order copies of the last evaluated state
  int* out_sel;            // [M][N][L]
  double* out_p;           // [M][N][L]
  double* out_zs;          // [M][N][NP]
  Ctrl* ctrl;              // final control state for the host
  int tile;                // subcarriers per LDS tile (batched solver)
  int gvec4;               // K % 4 == 0 and G 16-byte aligned: gains load four at a time
  int wave;                // batched solver, one-workgroup drops: subcarriers per wave tile
                           // (each wave runs its own subcarriers), 0 = workgroup tiles
  const double* p0;        // batched solver, warm start (device, may be null):
  const double* xi0;       //   initial powers [M][N][K], xi' [M], zeta' [K]
  const double* zeta0;
  int start_eval;          // the initial allocation is Dinkelbach's p^0 (warm start)
  int sdev;                // batched solver: tiles sum the association metric into
                           // S_part's row of the slot (device memory), not LDS
  int group;               // batched solver: workgroups that solve the drop together
  unsigned* bar;           // [3] their barrier: arrivals, generation, broken
  unsigned* ties;          // near-tie decisions (Sched::tie_rel > 0), zeroed before the solve
};

// Pointers into the workgroup's LDS: 32-bit addresses, direct LDS access.
#define LDS __attribute__((address_space(3)))
// Device memory reached through the drop descriptor: global (not generic)
// accesses, so loads complete in order and are waited for one by one.
#define GLB __attribute__((address_space(1)))
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ GLB T* gl(T* p) {
  return (GLB T*)p;
}

// One near-tie decision (rare: only where a margin is within tie_rel).
__device__ __forceinline__ void note_tie(const Drop& d) {
  __hip_atomic_fetch_add(gl(d.ties), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS carve-up for one workgroup.  The table of array pointers itself sits in
// LDS (written once per drop by thread 0): the pointers are reloaded from
// there as needed instead of occupying registers or spilling.  Arrays marked [T] have one row per
// subcarrier of the tile being processed.
struct Lds {
  LDS float* g;       // [T][M][K] gains
  LDS double* u;      // [T][M][K] (sigma + ICI)/Gamma
  LDS double* Sacc;   // [M][K] association metric summed over my subcarriers
                      // (with Sg: only the pass's reduced sums, in u's storage)
  double* Sg;         // [M][K] in device memory, the slot's own row, or null:
                      // where the tiles sum the association metric when the
                      // LDS it would take is better spent on subcarriers
  LDS double* mu;     // [K] 1 (elastic) or zeta'
  LDS double* racc;   // [K]
  LDS double* rhacc;  // [K]
  LDS int* Al;        // [K]
  LDS int* el;        // [K] 1 elastic
  LDS int* grp;       // [K] users grouped by RRH
  LDS int* grpk;      // [K] rank of a user within its RRH group
  LDS int* grp_off;   // [M+1]
  LDS int* wcnt;      // [waves][M] per-wave group counts
  LDS int* gcur;      // [M]
  LDS double* Hc;     // [T][K] H of user k on its own RRH
  LDS double* pic;    // [T][K] intra-cell price of user k on its own RRH
  LDS double* rk;     // [T][K] rate of user k on the subcarrier
  LDS double* rhk;    // [T][K] surrogate rate
  LDS int* su;        // [T][M][L] slots, storage order
  LDS double* sp;     // [T][M][L]
  LDS double* sal;    // [T][M][L]
  LDS double* sbe;    // [T][M][L]
  LDS double* szs;    // [T][M][L][L]
  LDS double* szn;    // [T][M][L][L] after this sweep's subgradient step
  LDS int* vcnt;      // [T][M] per-RRH view in decoding order
  LDS int* vslot;     // [T][M][L]
  LDS int* vuser;     // [T][M][L]
  LDS double* vu;     // [T][M][L]
  LDS double* vpre;   // [T][M][L+1]
  LDS double* vc;     // [T][M][L]
  LDS double* vcg;    // [T][M][L]
  LDS double* vr;     // [T][M][L]
  LDS double* vT;     // [T][M][L+1] suffix sums of vcg
  LDS double* Ptot;   // [T][M]
  LDS double* pinter; // [T][M]
  LDS double* psic;   // [T][M]
  LDS double* tps;    // [T][M]
  LDS double* tpe;    // [T][M]
  LDS double* tR;     // [T][M]
  LDS double* tsv;    // [T][M] C14 violation of RRH m's pairs
  LDS double* uc;     // [T][K] u of user k on its own RRH
  LDS float* gc;      // [T][K] gain of user k on its own RRH
  LDS int* ord;       // [T][K] each RRH group's candidates in order of H
  LDS double* pij;    // [T][M][M]
  LDS double* contrib; // [T][M][M]
  LDS double* xi;     // [M]
  LDS double* eta;    // [M]
  LDS double* pmask;  // [M]
  LDS double* psacc;  // [M]
  LDS double* peacc;  // [M]
  LDS double* Racc;   // [M]
  LDS double* dmax;   // [M]
  LDS double* svacc;  // [M] C14 violation
  LDS double* red;    // [threads / 64] one value per wave (block_sum)
  LDS double* tmp;    // [M+2] reduction results
};

__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~size_t(7); }

// Parts of the carve-up: arrays read by every team during a pass, the pass
// accumulators, and the per-tile arrays.
enum LdsPart : int { kShared = 1, kAccum = 2, kTile = 4, kAllParts = 7 };

// Lays the arrays of `parts` out from `base`; returns the bytes used (the
// other pointers are left null).  With base == nullptr it only measures
// (host side).
__host__ __device__ inline size_t carve_lds(LDS char* base, int M, int K, int L, int T, int nth, Lds* out,
                                            int parts = kAllParts, bool sdev = false) {
  Lds s;
  s.Sg = nullptr;
  size_t o = 0;
  int part = kAllParts;
  auto take = [&](size_t bytes) {
    if (!(parts & part)) return (LDS char*)nullptr;
    LDS char* p = base ? base + o : nullptr;
    o += align8(bytes);
    return p;
  };
  const size_t TM = (size_t)T * M, TML = TM * L, TK = (size_t)T * K;
  part = kTile;
  // Arrays whose live ranges within a tile do not overlap share storage: H
  // and the intra-cell price of each user on its own RRH (steps 6-7) take
  // the gains' place (steps 1-5); the inter-cell and C14 price terms (step
  // 5) the per-user rates' (steps 1-4), and so does the candidates' order
  // (steps 6-7).
  {
    if (parts & kTile) o = (o + 15) & ~size_t(15);  // the gains take 16-byte stores
    LDS char* r = take(std::max(sizeof(float) * TM * K, sizeof(double) * 2 * TK));
    s.g = (LDS float*)r;
    s.Hc = (LDS double*)r;
    s.pic = r ? s.Hc + TK : nullptr;
  }
  s.u = (LDS double*)take(sizeof(double) * TM * K);
  // with the sums in device memory, the pass's reduced sums (after the
  // tiles, when u is dead) take u's place: T*M*K >= M*K
  if (sdev) s.Sacc = s.u;
  {
    LDS char* r = take(std::max(sizeof(double) * 2 * TK, sizeof(double) * 2 * TM * M));
    s.rk = (LDS double*)r;
    s.rhk = r ? s.rk + TK : nullptr;
    s.pij = (LDS double*)r;
    s.contrib = r ? s.pij + TM * M : nullptr;
    s.ord = (LDS int*)r;
  }
  {
    LDS char* r = take(sizeof(double) * 2 * TML);
    s.vc = (LDS double*)r;
    s.vcg = r ? s.vc + TML : nullptr;
  }
  s.uc = (LDS double*)take(sizeof(double) * TK);
  s.gc = (LDS float*)take(sizeof(float) * TK);
  part = kAccum;
  if (!sdev) s.Sacc = (LDS double*)take(sizeof(double) * M * K);
  s.racc = (LDS double*)take(sizeof(double) * K);
  s.rhacc = (LDS double*)take(sizeof(double) * K);
  s.psacc = (LDS double*)take(sizeof(double) * M);
  s.peacc = (LDS double*)take(sizeof(double) * M);
  s.Racc = (LDS double*)take(sizeof(double) * M);
  s.dmax = (LDS double*)take(sizeof(double) * M);
  s.svacc = (LDS double*)take(sizeof(double) * M);
  part = kShared;
  s.mu = (LDS double*)take(sizeof(double) * K);
  s.Al = (LDS int*)take(sizeof(int) * K);
  s.el = (LDS int*)take(sizeof(int) * K);
  s.grp = (LDS int*)take(sizeof(int) * K);
  s.grpk = (LDS int*)take(sizeof(int) * K);
  s.grp_off = (LDS int*)take(sizeof(int) * (M + 1));
  s.wcnt = (LDS int*)take(sizeof(int) * (nth / 64) * M);
  s.gcur = (LDS int*)take(sizeof(int) * M);
  s.xi = (LDS double*)take(sizeof(double) * M);
  s.eta = (LDS double*)take(sizeof(double) * M);
  s.pmask = (LDS double*)take(sizeof(double) * M);
  s.red = (LDS double*)take(sizeof(double) * (nth / 64));
  s.tmp = (LDS double*)take(sizeof(double) * (M + 2));
  part = kTile;
  s.su = (LDS int*)take(sizeof(int) * TML);
  s.sp = (LDS double*)take(sizeof(double) * TML);
  s.sal = (LDS double*)take(sizeof(double) * TML);
  s.sbe = (LDS double*)take(sizeof(double) * TML);
  s.szs = (LDS double*)take(sizeof(double) * TML * L);
  s.szn = (LDS double*)take(sizeof(double) * TML * L);
  s.vcnt = (LDS int*)take(sizeof(int) * TM);
  s.vslot = (LDS int*)take(sizeof(int) * TML);
  s.vuser = (LDS int*)take(sizeof(int) * TML);
  s.vu = (LDS double*)take(sizeof(double) * TML);
  s.vpre = (LDS double*)take(sizeof(double) * TM * (L + 1));
  s.vr = (LDS double*)take(sizeof(double) * TML);
  s.vT = (LDS double*)take(sizeof(double) * TM * (L + 1));
  s.Ptot = (LDS double*)take(sizeof(double) * TM);
  s.pinter = (LDS double*)take(sizeof(double) * TM);
  s.psic = (LDS double*)take(sizeof(double) * TM);
  s.tps = (LDS double*)take(sizeof(double) * TM);
  s.tpe = (LDS double*)take(sizeof(double) * TM);
  s.tR = (LDS double*)take(sizeof(double) * TM);
  s.tsv = (LDS double*)take(sizeof(double) * TM);
  if (out) *out = s;
  return o;
}

// Bytes kept for one table of array pointers in the dynamic LDS (the
// host's pointers are wider than the device's 32-bit LDS addresses).
constexpr size_t kTabBytes = 512;
static_assert(sizeof(Lds) <= kTabBytes, "an LDS pointer table outgrew its space");

// Wave-tile carve-up for W waves with T subcarriers each: the W waves' pointer
// tables (kTabBytes each, at base), the shared arrays and the workgroup's
// accumulators once, then per wave its tile arrays and its own accumulators
// (its table points at the shared arrays).  The workgroup table's u (scratch
// before the first pass) is wave 0's.  Only drops with wave tiles pay for
// the tables.
__host__ __device__ inline size_t carve_waves(LDS char* base, int M, int K, int L, int T, int W, Lds* common) {
  Lds c;
  size_t o = (size_t)W * kTabBytes;
  o += carve_lds(base ? base + o : nullptr, M, K, L, 0, 64 * W, &c, kShared | kAccum);
  for (int w = 0; w < W; ++w) {
    Lds v;
    o = (o + 15) & ~size_t(15);
    o += carve_lds(base ? base + o : nullptr, M, K, L, T, 64 * W, &v, kTile | kAccum);
    v.mu = c.mu;
    v.Al = c.Al;
    v.el = c.el;
    v.grp = c.grp;
    v.grpk = c.grpk;
    v.grp_off = c.grp_off;
    v.wcnt = c.wcnt;
    v.gcur = c.gcur;
    v.xi = c.xi;
    v.eta = c.eta;
    v.pmask = c.pmask;
    v.red = c.red;
    v.tmp = c.tmp;
    if (w == 0) c.u = v.u;
    if (base) ((Lds*)base)[w] = v;
  }
  if (common) *common = c;
  return o;
}

__device__ inline double log2_1p(double x) { return alloc_logs::log2_1p_d(x); }
__device__ inline double log2_(double x) { return alloc_logs::log2_d(x); }

// init + at(0) + at(1) + ... + at(n-1), added in that order; the loads of
// each group of eight are issued together (at() is called on clamped
// indices only).
template <class F>
__device__ __forceinline__ double seq_sum(int n, double init, F&& at) {
  double acc = init;
  for (int t0 = 0; t0 < n; t0 += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = at(min(t0 + j, n - 1));
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (t0 + j < n) acc += v[j];
  }
  return acc;
}

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

// Start of a pass: multipliers, association (of state buffer rd) and RRH
// groups into LDS, accumulators cleared.
__device__ void begin_pass(const Drop& d, Lds& s, int rd) {
  const int M = d.M, K = d.K, tid = threadIdx.x, nth = blockDim.x;
  for (int k = tid; k < K; k += nth) {
    s.el[k] = gl(d.elastic)[k];
    s.mu[k] = gl(d.elastic)[k] ? 1.0 : gl(d.zeta)[k];
    s.Al[k] = gl(d.A)[(size_t)rd * K + k];
    s.racc[k] = 0.0;
    s.rhacc[k] = 0.0;
  }
  // the sums in device memory are cleared (and later summed) by the thread
  // that owns each item in the tiles' step 6: i = tid, tid + nth, ...
  if (GLB double* const Sg = gl(s.Sg))
    for (int i = tid; i < M * K; i += nth) Sg[i] = 0.0;
  else
    for (int i = tid; i < M * K; i += nth) s.Sacc[i] = 0.0;
  for (int m = tid; m < M; m += nth) {
    s.xi[m] = gl(d.xi)[m];
    s.eta[m] = gl(d.eta)[m];
    s.pmask[m] = gl(d.pmask)[m];
    s.psacc[m] = 0.0;
    s.peacc[m] = 0.0;
    s.Racc[m] = 0.0;
    s.dmax[m] = 0.0;
    s.svacc[m] = 0.0;
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

__device__ __forceinline__ int mul24(int a, int b) { return (int)__umul24(a, b); }
__device__ __forceinline__ int mad24(int a, int b, int c) { return mul24(a, b) + c; }

struct PassConst {
  double E, delta_v;
  int refit, reset, update, write_out;
  int rd, wr;  // state buffer read, and written by a sweep
};

// The threads that run one tile together: the whole workgroup (barriers), or
// one wave (lanes run in lockstep and a wave's LDS operations complete in
// order, so a fence against compiler reordering is all it needs).
struct BlockTeam {
  int tid, nth;
  __device__ void sync() const { __syncthreads(); }
};
struct WaveTeam {
  int tid;
  static constexpr int nth = 64;
  __device__ void sync() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// One subcarrier of a sweep (update) or of an evaluation pass (no update).
// Indexing of the per-tile LDS arrays (s = subcarrier within the tile).
// (LDS indices stay below 2^24: 24-bit multiply-adds, full rate, instead of
// 32-bit multiplies)
#define IX_MK(s, m, k) mad24(mad24((s), M, (m)), K, (k))
#define IX_ML(s, m, q) mad24(mad24((s), M, (m)), L, (q))
#define IX_ML1(s, m, t) mad24(mad24((s), M, (m)), L + 1, (t))
#define IX_MLL(s, m, a, b) mad24(mad24(mad24((s), M, (m)), L, (a)), L, (b))
#define IX_SM(s, m) mad24((s), M, (m))
#define IX_SMM(s, m, j) mad24(mad24((s), M, (m)), M, (j))
#define IX_SK(s, k) mad24((s), K, (k))

// One tile of ns subcarriers n = n0, n0 + nstep, ... of a sweep (update) or
// of an evaluation pass (no update).  Everything here is defined per
// subcarrier; the tile only gives each barrier interval more independent work.
// kItemH: step 6 runs one item per (t, m, k) and sums over t afterwards (the
// batched solver's tiles span many subcarriers); otherwise one item per
// (m, k) loops over t.  Both add the tile's H values in subcarrier order.
template <bool kItemH, class Team>
__device__ void tile(const Team& tm, const Drop& d, const Sched& sc, const PassConst& pc, Lds& s, int n0,
                     int nstep, int ns) {
  const int M = d.M, N = d.N, K = d.K, L = d.L, tid = tm.tid, nth = tm.nth;
  const Divs& dv = d.dv;
  const double sg = d.sigma;
  // state buffers: slot arrays [M][N][L], pair multipliers [M][N][L][L]
  const size_t nsl = (size_t)M * N * L;
  GLB const int* rsel = gl(d.sel) + pc.rd * nsl;
  GLB const double* rp = gl(d.p) + pc.rd * nsl;
  GLB const double* ral = gl(d.al) + pc.rd * nsl;
  GLB const double* rbe = gl(d.be) + pc.rd * nsl;
  GLB const double* rzs = gl(d.zs) + pc.rd * nsl * L;
#define NOF(t) (n0 + (t) * nstep)

  // 1. gains, slot state and per-RRH totals into LDS.  Within a round every
  //    global load is issued before the first LDS store (the round waits for
  //    memory once); the totals come from unconditional loads.
  {
    constexpr int kG = 6;  // gains per thread per round (four-wide: kQ)
    constexpr int kQ = 2;
    const bool vec4 = d.gvec4;
    const int K4 = K >> 2;
    const int nG = ns * M * K, nG4 = ns * M * K4, nS = ns * M * L, nZ = nS * L, nP = ns * M;
    const int rounds = max(vec4 ? (nG4 + kQ * nth - 1) / (kQ * nth) : (nG + kG * nth - 1) / (kG * nth),
                           (max(nZ, nP) + nth - 1) / nth);
    for (int r0 = 0; r0 < rounds; ++r0) {
      float gv[kG];
      f32x4 gq[kQ];
      int gqi[kQ];
      if (vec4) {
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
          const int i = tid + (r0 * kQ + j) * nth;
          gqi[j] = -1;
          if (i < nG4) {
            const int t = dv.MK4.div(i), r = i - mul24(t, M * K4), m = dv.K4.div(r), c = r - mul24(m, K4);
            gq[j] = *(GLB const f32x4*)(gl(d.G) + ((size_t)m * N + NOF(t)) * K + 4 * c);
            gqi[j] = IX_MK(t, m, 4 * c);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < kG; ++j) {
          const int i = tid + (r0 * kG + j) * nth;
          if (i < nG) {
            const int t = dv.MK.div(i), r = i - mul24(t, M * K), m = dv.K.div(r), k = r - mul24(m, K);
            gv[j] = gl(d.G)[((size_t)m * N + NOF(t)) * K + k];
          }
        }
      }
      const int i = tid + r0 * nth;
      int sel = -1;
      double p = 0.0, al = 1.0, be = 0.0, z = 0.0, pq[kMaxL];
      int sq[kMaxL];
      if (i < nS) {
        const int t = dv.ML.div(i), r = i - mul24(t, M * L), m = dv.L.div(r), q = r - mul24(m, L);
        const size_t gi = ((size_t)m * N + NOF(t)) * L + q;
        sel = rsel[gi];
        p = rp[gi];
        if (!pc.reset) {
          al = ral[gi];
          be = rbe[gi];
        }
      }
      if (i < nZ) {
        const int t = dv.MLL.div(i), r = i - mul24(t, M * L * L), m = dv.LL.div(r), ab = r - mul24(m, L * L);
        z = rzs[((size_t)m * N + NOF(t)) * L * L + ab];
      }
      if (i < nP) {
        const int t = dv.M.div(i), m = i - mul24(t, M);
        const size_t gi = ((size_t)m * N + NOF(t)) * L;
#pragma unroll
        for (int q = 0; q < kMaxL; ++q) {
          sq[q] = q < L ? rsel[gi + q] : -1;
          pq[q] = q < L ? rp[gi + q] : 0.0;
        }
      }
      if (vec4) {
#pragma unroll
        for (int j = 0; j < kQ; ++j)
          if (gqi[j] >= 0) *(LDS f32x4*)(s.g + gqi[j]) = gq[j];
      } else {
#pragma unroll
        for (int j = 0; j < kG; ++j) {
          const int ij = tid + (r0 * kG + j) * nth;
          if (ij < nG) s.g[ij] = gv[j];
        }
      }
      if (i < nS) {
        s.su[i] = sel;
        s.sp[i] = p;
        s.sal[i] = al;
        s.sbe[i] = be;
      }
      if (i < nZ) {
        s.szs[i] = z;
        s.szn[i] = 0.0;
      }
      if (i < nP) {
        double acc = 0.0;  // total power of RRH m on the subcarrier
#pragma unroll
        for (int q = 0; q < kMaxL; ++q)
          if (sq[q] >= 0) acc += pq[q];
        s.Ptot[i] = acc;
      }
    }
  }
  for (int i = tid; i < ns * K; i += nth) {
    s.rk[i] = 0.0;
    s.rhk[i] = 0.0;
  }
  tm.sync();

  // 2. inter-cell interference as exclusive prefix + suffix over RRHs (no
  //    subtraction), stored as u = (sigma + ICI)/Gamma
  for (int i = tid; i < ns * K; i += nth) {
    const int t = dv.K.div(i), k = i - mul24(t, K);
    double suf = 0.0;
    for (int m = M - 1; m >= 0; --m) {
      s.u[IX_MK(t, m, k)] = suf;
      suf += s.Ptot[IX_SM(t, m)] * (double)s.g[IX_MK(t, m, k)];
    }
    double pre = 0.0;
    const int own = s.Al[k];
    for (int m = 0; m < M; ++m) {
      const float gf = s.g[IX_MK(t, m, k)];
      const double gm = (double)gf;
      const double ici = pre + s.u[IX_MK(t, m, k)];
      pre += s.Ptot[IX_SM(t, m)] * gm;
      const double uu = (sg + ici) / gm;
      s.u[IX_MK(t, m, k)] = uu;
      if (m == own) {  // kept for the C14 test of the selection (step 7)
        s.uc[i] = uu;
        s.gc[i] = gf;
      }
    }
  }
  tm.sync();

  // 3. SIC decoding order of each RRH's users: normalised gain descending
  //    (u ascending), ties to the lower user; position by rank
  for (int i = tid; i < ns * M * L; i += nth) {
    const int t = dv.ML.div(i), r = i - mul24(t, M * L), m = dv.L.div(r), q = r - mul24(m, L);
    const int k = s.su[i];
    if (k < 0) continue;
    const double uq = s.u[IX_MK(t, m, k)];
    int pos = 0;
    for (int q2 = 0; q2 < L; ++q2) {
      const int k2 = s.su[IX_ML(t, m, q2)];
      if (q2 == q || k2 < 0) continue;
      const double u2 = s.u[IX_MK(t, m, k2)];
      if (u2 < uq || (u2 == uq && k2 < k)) ++pos;
      if (sc.tie_rel > 0.0 && k2 > k && fabs(u2 - uq) <= sc.tie_rel * fmax(u2, uq)) note_tie(d);
    }
    s.vslot[IX_ML(t, m, pos)] = q;
    s.vuser[IX_ML(t, m, pos)] = k;
    s.vu[IX_ML(t, m, pos)] = uq;
  }
  for (int i = tid; i < ns * M; i += nth) {
    int cnt = 0;
    for (int q = 0; q < L; ++q) cnt += s.su[i * L + q] >= 0;
    s.vcnt[i] = cnt;
  }
  tm.sync();

  // 4. per selected user: SINR, rate, SCALE refit and surrogate, price c
  for (int i = tid; i < ns * M * L; i += nth) {
    const int t = dv.ML.div(i), r = i - mul24(t, M * L), m = dv.L.div(r), a = r - mul24(m, L);
    if (a >= s.vcnt[IX_SM(t, m)]) continue;
    double pre = 0.0;
    for (int a2 = 0; a2 < a; ++a2) pre += s.sp[IX_ML(t, m, s.vslot[IX_ML(t, m, a2)])];
    const int k = s.vuser[i], q = s.vslot[i];
    const double pq = s.sp[IX_ML(t, m, q)];
    const double wmk = d.w ? gl(d.w)[(size_t)m * K + k] : 1.0;
    const double uu = s.vu[i];
    const double gam = pq / (uu + pre);
    const double rr = log2_1p(gam);
    double al = s.sal[IX_ML(t, m, q)], be = s.sbe[IX_ML(t, m, q)];
    if (pc.refit && pq > 0.0) {
      al = gam / (1.0 + gam);
      be = rr - al * log2_(gam);
      s.sal[IX_ML(t, m, q)] = al;
      s.sbe[IX_ML(t, m, q)] = be;
    }
    const double rh = (pq > 0.0) ? be + al * log2_(gam) : 0.0;
    const double cg = wmk * s.mu[k] * al / (kLn2 * (uu + pre));
    s.vpre[IX_ML1(t, m, a)] = pre;
    s.vcg[i] = cg;
    s.vc[i] = cg / (double)s.g[IX_MK(t, m, k)];
    s.vr[i] = wmk * rr;
    s.rk[IX_SK(t, k)] = wmk * rr;  // a user holds at most one slot per subcarrier
    s.rhk[IX_SK(t, k)] = wmk * rh;
    if (pc.write_out) {
      const size_t o = ((size_t)m * N + NOF(t)) * L + a;
      gl(d.out_sel)[o] = k;
      gl(d.out_p)[o] = pq;
    }
  }
  tm.sync();
  for (int i = tid; i < ns * M; i += nth) {
    const int t = dv.M.div(i), m = i - mul24(t, M);
    const int cnt = s.vcnt[i];
    double ps = 0.0, pe = 0.0, Rm = 0.0;
    for (int a = 0; a < cnt; ++a) {
      const double pq = s.sp[IX_ML(t, m, s.vslot[IX_ML(t, m, a)])];
      ps += pq;
      if (s.el[s.vuser[IX_ML(t, m, a)]]) {
        pe += pq;
        Rm += s.vr[IX_ML(t, m, a)];
      }
    }
    s.vpre[IX_ML1(t, m, cnt)] = ps;
    s.tps[i] = ps;
    s.tpe[i] = pe;
    s.tR[i] = Rm;
    // C14 at the state: each co-scheduled pair's relative margin
    // (u_s - u_w)/(u_s + u_w), s the user of larger raw gain (ties to the
    // lower index), counted above kSicTol
    double sv = 0.0;
    for (int a = 0; a < cnt; ++a)
      for (int b = a + 1; b < cnt; ++b) {
        const int ka = s.vuser[IX_ML(t, m, a)], kb = s.vuser[IX_ML(t, m, b)];
        const float ga = s.g[IX_MK(t, m, ka)], gb = s.g[IX_MK(t, m, kb)];
        const bool swap = gb > ga || (gb == ga && kb < ka);
        const double us = swap ? s.vu[IX_ML(t, m, b)] : s.vu[IX_ML(t, m, a)];
        const double uw = swap ? s.vu[IX_ML(t, m, a)] : s.vu[IX_ML(t, m, b)];
        if (us > uw) {  // a positive margin (the only kind counted)
          const double om = (us - uw) / (us + uw);
          if (om > kSicTol) sv += om - kSicTol;
        }
      }
    s.tsv[i] = sv;
    if (pc.write_out) {
      for (int a = cnt; a < L; ++a) {
        const size_t o = ((size_t)m * N + NOF(t)) * L + a;
        gl(d.out_sel)[o] = -1;
        gl(d.out_p)[o] = 0.0;
      }
      int pi = 0;
      for (int a = 0; a < L; ++a)
        for (int b = a + 1; b < L; ++b, ++pi)
          gl(d.out_zs)[((size_t)m * N + NOF(t)) * d.NP + pi] =
              (b < cnt) ? s.szs[IX_MLL(t, m, s.vslot[IX_ML(t, m, a)], s.vslot[IX_ML(t, m, b)])] : 0.0;
    }
  }
  // tile sums of the per-user rates into the pass accumulators, in
  // subcarrier order (the rates are complete since the barrier above)
  for (int k = tid; k < K; k += nth) {
    s.racc[k] += seq_sum(ns, 0.0, [&](int t) { return s.rk[IX_SK(t, k)]; });
    s.rhacc[k] += seq_sum(ns, 0.0, [&](int t) { return s.rhk[IX_SK(t, k)]; });
  }
  // (the barrier also ends the reads of the rates, whose storage step 5
  // reuses)
  tm.sync();
  // tile sums of the per-RRH powers and elastic rates of the loop above; on
  // a sweep they run in step 5's barrier interval, which does not touch them
  auto rrh_sums = [&]() {
    for (int m = tid; m < M; m += nth) {
      s.psacc[m] = seq_sum(ns, s.psacc[m], [&](int t) { return s.tps[IX_SM(t, m)]; });
      s.peacc[m] = seq_sum(ns, s.peacc[m], [&](int t) { return s.tpe[IX_SM(t, m)]; });
      s.Racc[m] = seq_sum(ns, s.Racc[m], [&](int t) { return s.tR[IX_SM(t, m)]; });
      s.svacc[m] = seq_sum(ns, s.svacc[m], [&](int t) { return s.tsv[IX_SM(t, m)]; });
    }
  };
  if (!pc.update) {
    rrh_sums();
    tm.sync();
    return;
  }

  // 5. inter-cell price and C14 terms per (RRH m, other RRH j)
  for (int i = tid; i < ns * M * M; i += nth) {
    const int t = dv.MM.div(i), r = i - mul24(t, M * M), m = dv.M.div(r), j = r - mul24(m, M);
    double inter = 0.0, sic = 0.0;
    if (j != m) {
      const int cj = s.vcnt[IX_SM(t, j)];
      for (int a = 0; a < cj; ++a)
        inter += s.vc[IX_ML(t, j, a)] * (double)s.g[IX_MK(t, m, s.vuser[IX_ML(t, j, a)])];
      // pairs of RRH m: their margins move with the power of RRH j (a pair
      // whose multiplier is zero adds nothing: skipped)
      const int cnt = s.vcnt[IX_SM(t, m)];
      for (int a = 0; a < cnt; ++a)
        for (int b = a + 1; b < cnt; ++b) {
          const double z = s.szs[IX_MLL(t, m, s.vslot[IX_ML(t, m, a)], s.vslot[IX_ML(t, m, b)])];
          if (z == 0.0) continue;
          const int ka = s.vuser[IX_ML(t, m, a)], kb = s.vuser[IX_ML(t, m, b)];
          const double ga = s.g[IX_MK(t, m, ka)], gb = s.g[IX_MK(t, m, kb)];
          const bool swap = gb > ga || (gb == ga && kb < ka);  // strong = larger raw gain
          const int ks = swap ? kb : ka, kw = swap ? ka : kb;
          const double us = swap ? s.vu[IX_ML(t, m, b)] : s.vu[IX_ML(t, m, a)];
          const double uw = swap ? s.vu[IX_ML(t, m, a)] : s.vu[IX_ML(t, m, b)];
          const double gs = swap ? gb : ga, gw = swap ? ga : gb;
          const double dj = ((double)s.g[IX_MK(t, j, ks)] / gs - (double)s.g[IX_MK(t, j, kw)] / gw) / (us + uw);
          sic += z * dj;
        }
    }
    s.pij[i] = inter;
    s.contrib[i] = sic;
  }
  // subgradient step of each pair's C14 multiplier on the margin Omega/nu
  for (int i = tid; i < ns * M * L * L; i += nth) {
    const int t = dv.MLL.div(i), r = i - mul24(t, M * L * L), m = dv.LL.div(r), rl = dv.L.div(r), a = rl - mul24(dv.L.div(rl), L),
              b = r - mul24(rl, L);
    if (!(a < b && b < s.vcnt[IX_SM(t, m)])) continue;
    const int ka = s.vuser[IX_ML(t, m, a)], kb = s.vuser[IX_ML(t, m, b)];
    const double ga = s.g[IX_MK(t, m, ka)], gb = s.g[IX_MK(t, m, kb)];
    const bool swap = gb > ga || (gb == ga && kb < ka);
    const double us = swap ? s.vu[IX_ML(t, m, b)] : s.vu[IX_ML(t, m, a)];
    const double uw = swap ? s.vu[IX_ML(t, m, a)] : s.vu[IX_ML(t, m, b)];
    const int sa = s.vslot[IX_ML(t, m, a)], sb = s.vslot[IX_ML(t, m, b)];
    const double z = s.szs[IX_MLL(t, m, sa, sb)];
    if (z == 0.0 && !(us > uw)) {  // a zero multiplier and a margin <= 0: it stays 0
      s.szn[IX_MLL(t, m, sa, sb)] = 0.0;
      s.szn[IX_MLL(t, m, sb, sa)] = 0.0;
      continue;
    }
    const double om = (us - uw) / (us + uw);
    const double zn = fmax(z + pc.delta_v * om, 0.0);
    s.szn[IX_MLL(t, m, sa, sb)] = zn;
    s.szn[IX_MLL(t, m, sb, sa)] = zn;
    // the projected subgradient joins the power changes in the dual loop's
    // stopping test (an order-free integer maximum, as below)
    const double dz = fabs(zn - z) / pc.delta_v;
    if (dz == dz)
      __hip_atomic_fetch_max((LDS unsigned long long*)(s.dmax + m), (unsigned long long)__double_as_longlong(dz),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  rrh_sums();
  tm.sync();
  for (int i = tid; i < ns * M; i += nth) {
    const int t = dv.M.div(i), m = i - mul24(t, M);
    double inter = 0.0, sic = 0.0;
    for (int j = 0; j < M; ++j) {
      inter += s.pij[IX_SMM(t, m, j)];
      if (j != m) sic += s.contrib[IX_SMM(t, j, m)];
    }
    s.pinter[i] = inter;
    s.psic[i] = sic;
    const int cnt = s.vcnt[i];
    s.vT[IX_ML1(t, m, cnt)] = 0.0;
    for (int a = cnt - 1; a >= 0; --a) s.vT[IX_ML1(t, m, a)] = s.vT[IX_ML1(t, m, a + 1)] + s.vcg[IX_ML(t, m, a)];
  }
  tm.sync();

  // near-ties of where each user would enter its RRH's decoding order (a
  // separate loop, so that the sweep without counting carries none of it)
  if (sc.tie_rel > 0.0) {
    for (int i = tid; i < ns * M * K; i += nth) {
      const int t = dv.MK.div(i), r = i - mul24(t, M * K), m = dv.K.div(r), k = r - mul24(m, K);
      const double u = s.u[IX_MK(t, m, k)];
      const int cnt = s.vcnt[IX_SM(t, m)];
      for (int a = 0; a < cnt; ++a) {
        const double ua = s.vu[IX_ML(t, m, a)];
        if (s.vuser[IX_ML(t, m, a)] != k && fabs(ua - u) <= sc.tie_rel * fmax(ua, u)) note_tie(d);
      }
    }
  }

  // 6. per-triple Lagrangian maximum H (the candidates' order starts empty:
  //    its storage held the price terms read after step 5)
  for (int i = tid; i < ns * K; i += nth) s.ord[i] = -1;
  auto h_item = [&](int t, int m, int k, double u) -> double {
    const double wmu = (d.w ? gl(d.w)[(size_t)m * K + k] : 1.0) * s.mu[k];
    const int cnt = s.vcnt[IX_SM(t, m)];
    int q = -1, pos = 0;
    for (int a = 0; a < cnt; ++a) {
      const int ka = s.vuser[IX_ML(t, m, a)];
      const double ua = s.vu[IX_ML(t, m, a)];
      if (ka == k) q = a;
      if (ua < u || (ua == u && ka < k)) ++pos;
    }
    const double Sb = s.vpre[IX_ML1(t, m, q >= 0 ? q : pos)];
    const double pin = s.vT[IX_ML1(t, m, q >= 0 ? q + 1 : pos)];
    const double c =
        (s.el[k] ? pc.E * s.eta[m] : 0.0) + s.xi[m] + pin + s.pinter[IX_SM(t, m)] + s.psic[IX_SM(t, m)];
    double H = 0.0;
    if (wmu > 0.0) {
      const double ainv = u + Sb;
      double pt;
      if (c <= 0.0) {
        pt = s.pmask[m];
      } else {
        const double Wl = wmu / (c * kLn2);
        pt = fmin(fmax(Wl - ainv, 0.0), s.pmask[m]);
      }
      if (pt > 0.0) H = wmu * log2_1p(pt / ainv) - c * pt;
    }
    if (s.Al[k] == m) {  // H in the user's place within its RRH group
      s.Hc[IX_SK(t, s.grp_off[m] + s.grpk[k])] = H;
      s.pic[IX_SK(t, k)] = pin;
    }
    return H;
  };
  if (kItemH) {
    // H replaces the triple's own u (nothing later in the pass reads u)
    for (int i = tid; i < ns * M * K; i += nth) {
      const int t = dv.MK.div(i), r = i - mul24(t, M * K), m = dv.K.div(r), k = r - mul24(m, K);
      s.u[i] = h_item(t, m, k, s.u[i]);
    }
    tm.sync();
    // (the selection below runs in the same barrier interval)
    GLB double* const Sg = gl(s.Sg);
    for (int i = tid; i < M * K; i += nth) {
      const double Hsum = seq_sum(ns, 0.0, [&](int t) { return s.u[t * M * K + i]; });
      if (Sg) Sg[i] += Hsum;
      else s.Sacc[i] += Hsum;
    }
  } else {
    GLB double* const Sg = gl(s.Sg);
    for (int i = tid; i < M * K; i += nth) {
      const int m = dv.K.div(i), k = i - mul24(m, K);
      double Hsum = 0.0;
      for (int t = 0; t < ns; ++t) Hsum += h_item(t, m, k, s.u[IX_MK(t, m, k)]);
      if (Sg) Sg[i] += Hsum;
      else s.Sacc[i] += Hsum;
    }
    tm.sync();
  }

  // 7. selection.  Each candidate (H > 0 on its own RRH) takes the place of
  //    its rank within its RRH group (H desc, user asc: a group holds its
  //    users in increasing order, so positions order them as indices do) ...
  for (int i = tid; i < ns * K; i += nth) {
    const int t = dv.K.div(i), k = i - mul24(t, K);
    const int m = s.Al[k];
    if (m < 0) continue;
    const int e0 = s.grp_off[m], e1 = s.grp_off[m + 1], ek = e0 + s.grpk[k];
    const double h = s.Hc[IX_SK(t, ek)];
    if (!(h > 0.0)) continue;
    int rank = 0;
    for (int e = e0; e < e1; ++e) {
      const double hj = s.Hc[IX_SK(t, e)];
      rank += (hj > h) || (hj == h && e < ek);
    }
    s.ord[IX_SK(t, e0 + rank)] = k;
    if (sc.tie_rel > 0.0 && rank < L) {  // k and the next candidate in H order
      double gap = INFINITY;
      for (int e = e0; e < e1; ++e) {
        const double hj = s.Hc[IX_SK(t, e)];
        if (e != ek && hj > 0.0 && (hj < h || (hj == h && e > ek))) gap = fmin(gap, h - hj);
      }
      if (gap <= sc.tie_rel * h) note_tie(d);
    }
  }
  tm.sync();
  // ... then, one item per slot, each (subcarrier, RRH)'s new selection
  // (settled by each of its slot items alone, so no barrier follows), its
  // closed-form powers and the C14 multipliers' move into the new slots.
  // The candidates are taken in order, each only if every pair it forms with
  // those taken before it meets C14 (margin <= 0 at the state's
  // interference), until l are taken (Sec. II-B, C8/C14).
  for (int i = tid; i < ns * M * L; i += nth) {
    const int t = dv.ML.div(i), r = i - mul24(t, M * L), m = dv.L.div(r), a = r - mul24(m, L);
    const int sm = IX_SM(t, m);
    const int cnt = s.vcnt[sm];
    int vk[kMaxL], vq[kMaxL], ch[kMaxL];
    double cu[kMaxL];
    float cgn[kMaxL];
#pragma unroll
    for (int b = 0; b < kMaxL; ++b) {
      vk[b] = b < cnt ? s.vuser[IX_ML(t, m, b)] : -1;
      vq[b] = b < cnt ? s.vslot[IX_ML(t, m, b)] : -1;
      ch[b] = -1;
      cu[b] = 0.0;
      cgn[b] = 0.0f;
    }
    int np = 0;
    {
      const int base = s.grp_off[m], gn = s.grp_off[m + 1] - base;
      for (int e = 0; e < gn && np < L; ++e) {
        const int k = s.ord[IX_SK(t, base + e)];
        if (k < 0) break;
        const double uk = s.uc[IX_SK(t, k)];
        const float gk = s.gc[IX_SK(t, k)];
        bool ok = true;
#pragma unroll
        for (int b = 0; b < kMaxL; ++b)
          if (b < np) {
            const bool kstrong = gk > cgn[b] || (gk == cgn[b] && k < ch[b]);
            const double us = kstrong ? uk : cu[b], uw = kstrong ? cu[b] : uk;
            // the margin (us - uw)/(us + uw) is positive exactly when
            // us > uw (both positive)
            if (us > uw) ok = false;
          }
        if (ok) {
#pragma unroll
          for (int b = 0; b < kMaxL; ++b)
            if (b == np) {
              ch[b] = k;
              cu[b] = uk;
              cgn[b] = gk;
            }
          ++np;
        }
      }
    }
    int old[kMaxL];  // each new entry's slot before this sweep (-1 if new)
#pragma unroll
    for (int b = 0; b < kMaxL; ++b) {
      old[b] = -1;
#pragma unroll
      for (int b2 = 0; b2 < kMaxL; ++b2)
        if (b < np && b2 < cnt && vk[b2] == ch[b]) old[b] = vq[b2];
    }
    double dm = 0.0;
    int k = -1;
    double pn = 0.0, alph = 1.0, bet = 0.0;
    if (a < np) {
      k = ch[a];
      double p_old = 0.0;
      if (old[a] >= 0) {
        p_old = s.sp[IX_ML(t, m, old[a])];
        alph = s.sal[IX_ML(t, m, old[a])];
        bet = s.sbe[IX_ML(t, m, old[a])];
      }
      const double wmu = (d.w ? gl(d.w)[(size_t)m * K + k] : 1.0) * s.mu[k];
      const double ps = s.psic[sm];
      const double pplus = fmax(ps, 0.0), pminus = fmax(-ps, 0.0);
      const double cp = (s.el[k] ? pc.E * s.eta[m] : 0.0) + s.xi[m] + s.pic[IX_SK(t, k)] + s.pinter[sm] + pplus;
      const double num = wmu * alph / kLn2 + p_old * pminus;
      pn = (cp > 0.0) ? fmin(fmax(num / cp, 0.0), s.pmask[m]) : s.pmask[m];
      if (pn < kPowerFloorRel * s.pmask[m]) pn = 0.0;
      dm = fabs(pn - p_old) / s.pmask[m];
    }
    if (a < cnt) {  // an incumbent that leaves the selection
      const int kt = vk[a];
      bool kept = false;
#pragma unroll
      for (int b = 0; b < kMaxL; ++b) kept = kept || (b < np && ch[b] == kt);
      if (!kept) dm = fmax(dm, s.sp[IX_ML(t, m, vq[a])] / s.pmask[m]);
    }
    // largest power change of RRH m: dm >= 0, so the bit patterns order as
    // the values and an integer maximum is exact and order-free (NaN is
    // skipped, as the maximum over the values would skip it)
    if (dm == dm)
      __hip_atomic_fetch_max((LDS unsigned long long*)(s.dmax + m), (unsigned long long)__double_as_longlong(dm),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    // the new state goes to buffer wr
    const size_t gi = pc.wr * nsl + ((size_t)m * N + NOF(t)) * L + a;
    gl(d.sel)[gi] = k;
    gl(d.p)[gi] = pn;
    gl(d.al)[gi] = alph;
    gl(d.be)[gi] = bet;
    // the C14 multipliers of this new slot's pairs, from the pairs' old slots
#pragma unroll
    for (int b = 0; b < kMaxL; ++b)
      if (b < L) {
        double z = 0.0;
        if (a < np && b < np && a != b && old[a] >= 0 && old[b] >= 0) z = s.szn[IX_MLL(t, m, old[a], old[b])];
        gl(d.zs)[(gi * L) + b] = z;
      }
  }
  tm.sync();
#undef NOF
}

// Per-workgroup partials after its subcarriers.
__device__ void write_partials(const Drop& d, const Lds& s, int b) {
  const int M = d.M, K = d.K, tid = threadIdx.x, nth = blockDim.x;
  if (!s.Sg)  // else the tiles summed into this row already
    for (int i = tid; i < M * K; i += nth) gl(d.S_part)[(size_t)b * M * K + i] = s.Sacc[i];
  for (int k = tid; k < K; k += nth) {
    gl(d.r_part)[(size_t)b * K + k] = s.racc[k];
    gl(d.rh_part)[(size_t)b * K + k] = s.rhacc[k];
  }
  for (int m = tid; m < M; m += nth) {
    gl(d.psum_part)[(size_t)b * M + m] = s.psacc[m];
    gl(d.pel_part)[(size_t)b * M + m] = s.peacc[m];
  }
  if (tid == 0) {
    double R = 0.0, dm = 0.0, sv = 0.0;
    for (int m = 0; m < M; ++m) {
      R += s.Racc[m];
      dm = fmax(dm, s.dmax[m]);
      sv += s.svacc[m];
    }
    gl(d.R_part)[b] = R;
    gl(d.d_part)[b] = dm;
    gl(d.sv_part)[b] = sv;
  }
}


// C13 violation of one user: (1 - kQosTol) - r/Psi where positive, for a
// streaming user.
__device__ inline double qos_viol(double r, double psi) {
  const double x = r / psi;
  return x < 1.0 - kQosTol ? (1.0 - kQosTol) - x : 0.0;
}

// Subgradient step of zeta' on the SCALE surrogate rate: the relative C13
// violation (Psi - r_hat)/Psi clipped to [-qos_down, 1]; returns the new
// value, *res the step over delta.
__device__ inline double zeta_step(double z, double psi, double rh, double delta_v, double qos_down, double* res) {
  const double viol = fmin(fmax((psi - rh) / psi, -qos_down), 1.0);
  const double zn = fmax(z + delta_v * viol, 0.0);
  *res = fabs(zn - z) / delta_v;
  return zn;
}

// Subgradient step of xi'_m on the C12 budget, scaled by N l/(ln2 pmax);
// returns the new value, *res the step over (delta scale).
__device__ inline double xi_step(double x, double ps, double pmax, int N, int L, double delta_v, double* res) {
  const double scale = (double)N * L / (kLn2 * pmax);
  const double xn = fmax(x + delta_v * scale * (ps - pmax) / pmax, 0.0);
  *res = fabs(xn - x) / (delta_v * scale);
  return xn;
}

// The association of one user from its summed Lagrangian maxima S[m]
// (stride ms): the RRH of the largest positive sum (ties to the lower RRH);
// without one an elastic user is unserved and a streaming user keeps its RRH.
template <class F>
__device__ inline int assoc_of(int M, int before, bool elastic, F&& S) {
  double best = -INFINITY;
  int bm = 0;
  for (int m = 0; m < M; ++m)
    if (S(m) > best) {
      best = S(m);
      bm = m;
    }
  if (best > 0.0) return bm;
  return elastic ? -1 : before;
}

// Whether the best and second-best RRH of a user are within tie_rel of each
// other (both with a positive sum of H).
template <class F>
__device__ inline bool assoc_near_tie(int M, double tie_rel, F&& S) {
  double best = -INFINITY, second = -INFINITY;
  for (int m = 0; m < M; ++m) {
    const double v = S(m);
    if (v > best) {
      second = best;
      best = v;
    } else if (v > second) {
      second = v;
    }
  }
  return best > 0.0 && second > 0.0 && best - second <= tie_rel * best;
}

// Reductions across workgroups: users k = b, b+G, ... per workgroup (rates,
// association into buffer wr, zeta' steps, partial C13 violation);
// workgroup 0 also does the per-RRH and scalar sums.
// Sum over the workgroup of one value per thread, by a fixed tree (wave
// shuffles, then the waves in order); the total is returned to thread 0.
__device__ double block_sum(double v, Lds& s) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();  // s.red may still be read by the caller's previous use
  if (lane == 0) s.red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) t += s.red[w];
  return t;
}

// Reductions over the G workgroups of a grid or group.  Up to this many
// workgroups, one thread sums an item's G partials in workgroup order; above
// it a wave does (lane l takes workgroups l, l + 64, ..., then a fixed
// butterfly, which leaves the same bits in every lane).
constexpr int kSerialGroups = 32;

// Item i's sum (or maximum, mx) of src[g * stride] over the G workgroups, by
// this thread (serial mode) or by this wave (every lane returns it).
__device__ inline double group_item(GLB const double* src, size_t stride, int G, bool mx, bool wave_mode) {
  double acc = 0.0;
  if (!wave_mode) {
    for (int g = 0; g < G; ++g) {
      const double v = src[(size_t)g * stride];
      acc = mx ? fmax(acc, v) : acc + v;
    }
    return acc;
  }
  for (int g = (int)(threadIdx.x & 63); g < G; g += 64) {
    const double v = src[(size_t)g * stride];
    acc = mx ? fmax(acc, v) : acc + v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(acc, o, 64);
    acc = mx ? fmax(acc, w) : acc + w;
  }
  return acc;
}

// Runs f(item) for items 0..n-1: one thread per item, or one wave per item
// (then only lane 0's call stores).
template <class F>
__device__ inline void for_group_items(int n, bool wave_mode, F&& f) {
  if (!wave_mode) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) f(i);
  } else {
    const int nw = (int)(blockDim.x >> 6);
    for (int i = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); i < n; i += nw) f(i);
  }
}

__device__ void reduce_pass(const Drop& d, const Sched& sc, const Ctrl& c, Lds& s, int b, int G,
                            bool update, double delta_v) {
  const int M = d.M, K = d.K, tid = threadIdx.x, nth = blockDim.x;
  const int par = c.pass & 1;
  const bool wm = G > kSerialGroups;
  const bool store = !wm || (tid & 63) == 0;
  int changes = 0;
  double vq = 0.0, zr = 0.0;
  if (b == 0 && tid == 0) store_shared(&d.chg_count[par ^ 1], 0);  // next pass's counter
  // this workgroup's users k = b, b + G, ...: each sum of G partials, one
  // item per (user, quantity), into the accumulators (the workgroup's own
  // partials are in device memory already)
  const int nk = b < K ? (K - b + G - 1) / G : 0;
  const int nq = update ? M + 2 : 2;
  for_group_items(nk * nq, wm, [&](int i) {
    const int j = i / nq, f = i - j * nq, k = b + j * G;
    const int m = f - 2;
    GLB const double* src = f == 0 ? gl(d.r_part) + k : f == 1 ? gl(d.rh_part) + k : gl(d.S_part) + (size_t)m * K + k;
    const size_t gs = f < 2 ? (size_t)K : (size_t)M * K;
    const double acc = group_item(src, gs, G, false, wm);
    if (store) {
      if (f == 0) s.racc[k] = acc;
      else if (f == 1) s.rhacc[k] = acc;
      else s.Sacc[(size_t)m * K + k] = acc;
    }
  });
  if (tid == 0) {
    s.tmp[0] = 0.0;              // largest zeta' step (an integer maximum)
    *(LDS int*)(s.tmp + 1) = 0;  // association changes
  }
  __syncthreads();
  for (int j = tid; j < nk; j += nth) {
    const int k = b + j * G;
    const double r = s.racc[k], rh = s.rhacc[k];
    gl(d.user_rate)[k] = r;
    const bool el = gl(d.elastic)[k];
    if (!el) vq += qos_viol(r, gl(d.psi)[k]);
    if (update) {
      const int before = gl(d.A)[(size_t)c.rd * K + k];
      const int after = assoc_of(M, before, el, [&](int m) { return s.Sacc[(size_t)m * K + k]; });
      if (sc.tie_rel > 0.0 && assoc_near_tie(M, sc.tie_rel, [&](int m) { return s.Sacc[(size_t)m * K + k]; }))
        note_tie(d);
      gl(d.A)[(size_t)c.wr * K + k] = after;
      if (after != before)
        __hip_atomic_fetch_add((LDS int*)(s.tmp + 1), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (!el) {
        double res;
        gl(d.zeta)[k] = zeta_step(gl(d.zeta)[k], gl(d.psi)[k], rh, delta_v, sc.qos_down, &res);
        if (res == res)
          __hip_atomic_fetch_max((LDS unsigned long long*)s.tmp, (unsigned long long)__double_as_longlong(res),
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
  vq = block_sum(vq, s);  // in a fixed order; thread 0 holds the total
  if (tid == 0) {
    zr = s.tmp[0];
    changes = *(LDS int*)(s.tmp + 1);
  }
  __syncthreads();
  if (tid == 0) {
    if (changes > 0) __hip_atomic_fetch_add(&d.chg_count[par], changes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    gl(d.vq_part)[b] = vq;
    gl(d.zr_part)[b] = zr;
  }
  if (b == 0) {
    // per-RRH sums, xi' step, R, P, max delta, C12 and C14 violations
    for_group_items(2 * M + 3, wm, [&](int i) {
      GLB const double* src;
      int stride;
      LDS double* dst;
      if (i < M) {
        src = gl(d.psum_part) + i, stride = M, dst = s.psacc + i;
      } else if (i < 2 * M) {
        src = gl(d.pel_part) + (i - M), stride = M, dst = s.peacc + (i - M);
      } else {
        const int q = i - 2 * M;
        src = q == 0 ? gl(d.R_part) : q == 1 ? gl(d.d_part) : gl(d.sv_part), stride = 1, dst = s.tmp + q;
      }
      const double acc = group_item(src, stride, G, i == 2 * M + 1, wm);  // the largest power change
      if (store) *dst = acc;
    });
    __syncthreads();
    if (tid == 0) {
      double P = d.pstatic, Vp = 0.0, xr = 0.0;
      for (int m = 0; m < M; ++m) {
        const double ps = s.psacc[m], pmax = gl(d.pmax)[m];
        P += gl(d.eta)[m] * s.peacc[m];
        const double y = ps / pmax;
        if (y > 1.0 + kBudgetTol) Vp += y - (1.0 + kBudgetTol);
        if (update) {
          double res;
          gl(d.xi)[m] = xi_step(gl(d.xi)[m], ps, pmax, d.N, d.L, delta_v, &res);
          xr = fmax(xr, res);
        }
      }
      store_shared(&d.red[0], s.tmp[0]);
      store_shared(&d.red[1], P);
      store_shared(&d.red[2], s.tmp[1]);
      store_shared(&d.red[3], xr);
      store_shared(&d.red[4], Vp);
      store_shared(&d.red[5], s.tmp[2]);
    }
  }
}

// Makes subcarrier n of state buffer rd meet C14 (Sec. II-B, C8/C14: a
// co-scheduled pair is SIC-decodable only when its raw-gain and
// normalised-gain orders agree).  While a pair breaks it at the state's
// interference, the pair of largest margin (RRHs in increasing order, then
// pairs in decoding order, the first of equal margins) loses one user: the
// elastic one when exactly one is elastic, otherwise the one of lower rate on
// the subcarrier (the higher user index on equal rates); its slot is emptied
// with its C14 multipliers.  Every round removes a user, so the loop ends.
// One thread per subcarrier, on the state in device memory: it runs once, at
// the end of a solve, and only when the returned state breaks C14.
__device__ void repair_subcarrier(const Drop& d, int rd, int n) {
  const int M = d.M, N = d.N, K = d.K, L = d.L;
  const size_t nsl = (size_t)M * N * L;
  GLB int* sel = gl(d.sel) + rd * nsl;
  GLB double* p = gl(d.p) + rd * nsl;
  GLB double* al = gl(d.al) + rd * nsl;
  GLB double* be = gl(d.be) + rd * nsl;
  GLB double* zs = gl(d.zs) + rd * nsl * L;
  GLB const float* G = gl(d.G);
  const double sg = d.sigma;
  auto ici_of = [&](int m, int k) {  // sum over the other RRHs, in increasing order
    double acc = 0.0;
    for (int j = 0; j < M; ++j) {
      if (j == m) continue;
      double pj = 0.0;
      for (int q = 0; q < L; ++q)
        if (sel[((size_t)j * N + n) * L + q] >= 0) pj += p[((size_t)j * N + n) * L + q];
      acc += pj * (double)G[((size_t)j * N + n) * K + k];
    }
    return acc;
  };
  for (;;) {
    double best = kSicTol;
    int bm = -1, bq[2] = {0, 0};
    for (int m = 0; m < M; ++m) {
      // the selected users of (m,n) in decoding order: u ascending, ties to
      // the lower user
      int cnt = 0, uk[kMaxL], uq[kMaxL];
      double uu[kMaxL];
      for (int q = 0; q < L; ++q) {
        const int k = sel[((size_t)m * N + n) * L + q];
        if (k < 0) continue;
        const double u = (sg + ici_of(m, k)) / (double)G[((size_t)m * N + n) * K + k];
        int t = cnt++;
        while (t > 0 && (uu[t - 1] > u || (uu[t - 1] == u && uk[t - 1] > k))) {
          uu[t] = uu[t - 1];
          uk[t] = uk[t - 1];
          uq[t] = uq[t - 1];
          --t;
        }
        uu[t] = u;
        uk[t] = k;
        uq[t] = q;
      }
      for (int a = 0; a < cnt; ++a)
        for (int b = a + 1; b < cnt; ++b) {
          const float ga = G[((size_t)m * N + n) * K + uk[a]], gb = G[((size_t)m * N + n) * K + uk[b]];
          const bool a_strong = ga > gb || (ga == gb && uk[a] < uk[b]);
          const double us = a_strong ? uu[a] : uu[b], uw = a_strong ? uu[b] : uu[a];
          const double om = (us - uw) / (us + uw);
          if (om > best) {
            best = om;
            bm = m;
            bq[0] = uq[a];
            bq[1] = uq[b];
          }
        }
    }
    if (bm < 0) return;
    const size_t base = ((size_t)bm * N + n) * L;
    int ks[2];
    double r[2];
    for (int x = 0; x < 2; ++x) {
      const int k = sel[base + bq[x]];
      ks[x] = k;
      // rate on the subcarrier: interference of the users decoded before k
      const double g = (double)G[((size_t)bm * N + n) * K + k];
      const double ici = ici_of(bm, k), u = (sg + ici) / g;
      double pre = 0.0;
      for (int q = 0; q < L; ++q) {
        const int k2 = sel[base + q];
        if (k2 < 0 || k2 == k) continue;
        const double u2 = (sg + ici_of(bm, k2)) / (double)G[((size_t)bm * N + n) * K + k2];
        if (u2 < u || (u2 == u && k2 < k)) pre += p[base + q];
      }
      r[x] = log2_1p(p[base + bq[x]] * g / (sg + ici + g * pre));
    }
    const bool e0 = gl(d.elastic)[ks[0]], e1 = gl(d.elastic)[ks[1]];
    int drop;
    if (e0 != e1)
      drop = e0 ? 0 : 1;
    else if (r[0] != r[1])
      drop = r[0] < r[1] ? 0 : 1;
    else
      drop = ks[0] > ks[1] ? 0 : 1;
    const int q = bq[drop];
    sel[base + q] = -1;
    p[base + q] = 0.0;
    al[base + q] = 1.0;
    be[base + q] = 0.0;
    for (int b = 0; b < L; ++b) {
      zs[(base + q) * L + b] = 0.0;
      zs[(base + b) * L + q] = 0.0;
    }
  }
}

// Two violations a (new) and b (best): -1 when a is lower by more than
// kViolRel (relative), 1 when higher, 0 otherwise (zero equals only zero).
__device__ inline int cmp_viol(double a, double b) {
  if (a == 0.0 && b == 0.0) return 0;
  if (a == 0.0) return -1;
  if (b == 0.0) return 1;
  if (a < b * (1.0 - kViolRel)) return -1;
  if (a > b * (1.0 + kViolRel)) return 1;
  return 0;
}

// Loop control, identical in every workgroup: one step from the reduced
// values of the pass just done.  A sweep ranks the state it read against the
// step's best and rotates the state buffers; the dual loop ends at its cap,
// when the powers and every projected multiplier subgradient are below
// tol_dual (and no user moved), or after `stall` sweeps without a better
// state (a violation lower by more than kViolRel counts as better).  The evaluation that follows reads the
// best state; Dinkelbach's test (Sec. III) is the root condition
// |R - E P| <= tol R on a state that meets C12 and C13 (C14 is enforced
// through its multiplier and the selection and reported when still broken),
// otherwise E <- R/P and the next step starts from that state.  A warm start's first evaluation is of its
// p^0, feasible or not: E^1 = R/P (F is strictly decreasing in E with its
// root at the optimum, so the iteration converges from either side).
__device__ void advance(const Sched& sc, Ctrl& c, const Eval& e) {
  if (c.mode == kSweep) {
    c.v += 1;
    c.total += 1;
    c.reset = 0;
    const double V = e.Vq + e.Vp, V2 = e.Vs, f = e.R - c.E * e.P;
    bool replace = true, progress = true;
    if (c.have_best) {
      int r = cmp_viol(V, c.bV);
      if (r == 0) r = cmp_viol(V2, c.bV2);
      if (r != 0) {
        replace = progress = r < 0;
      } else {
        replace = f > c.bf;
        progress = f - c.bf > sc.tol_d * fabs(c.bR);
      }
    }
    const int rd = c.rd, wr = c.wr;
    if (replace) {
      c.wr = c.have_best ? c.best : 3 - rd - wr;
      c.best = rd;
      c.have_best = 1;
      c.bV = V;
      c.bV2 = V2;
      c.bf = f;
      c.bR = e.R;
    } else {
      c.wr = rd;
    }
    c.rd = wr;
    c.stall = progress ? 0 : c.stall + 1;
    const double delta = e.changes > 0 ? INFINITY : fmax(fmax(e.dm, e.xres), e.zres);
    bool end = c.v >= sc.sweeps;
    if (isnan(delta)) {
      c.flags |= ALLOC_NONFINITE;
      end = true;
    }
    if (!sc.fixed) {
      if (delta < sc.tol_dual) end = true;
      if (sc.stall > 0 && c.stall >= sc.stall) end = true;
    }
    if (end) {
      c.mode = kEval;
      if (c.have_best) c.rd = c.best;
      c.wr = c.rd == 2 ? 0 : c.rd + 1;
    }
  } else if (c.mode == kEval) {
    c.R = e.R;
    c.P = e.P;
    c.Vq = e.Vq;
    c.Vp = e.Vp;
    c.Vs = e.Vs;
    const bool feasible = e.Vq == 0.0 && e.Vp == 0.0;  // C14 is reported, not required
    const double F = e.R - c.E * e.P;
    c.i += 1;
    bool next = false;
    if (c.first_eval) {
      c.first_eval = 0;
      if (c.i >= sc.max_d) {
        c.flags |= ALLOC_NOT_CONVERGED;
        c.mode = kDone;
      } else {
        c.E = e.R / e.P;
        next = true;
      }
    } else if (c.flags & ALLOC_NONFINITE) {
      c.mode = kDone;
    } else if (feasible && fabs(F) <= sc.tol_d * e.R) {
      c.mode = kDone;
    } else if (c.i >= sc.max_d) {
      c.flags |= ALLOC_NOT_CONVERGED;
      c.mode = kDone;
    } else {
      c.E = e.R / e.P;
      next = true;
    }
    if (next) {
      c.v = 0;
      c.reset = 1;
      c.have_best = 0;
      c.stall = 0;
      c.mode = kSweep;
    }
    // the returned allocation meets C14: pairs that still break it are
    // dissolved and the allocation evaluated again
    if (c.mode == kDone && e.Vs > 0.0 && !(c.flags & ALLOC_NONFINITE)) c.mode = kRepair;
  } else if (c.mode == kFinal) {
    c.R = e.R;
    c.P = e.P;
    c.Vq = e.Vq;
    c.Vp = e.Vp;
    c.Vs = e.Vs;
    c.mode = kDone;
  }
  c.pass += 1;
}

// Loop control of the grid solver, identical in every workgroup: the reduced
// values are read with device-scope atomics after the grid barrier, the
// per-workgroup C13 violations and zeta' steps by fixed-order trees.  The
// workgroup's copy c sits in LDS; thread 0 advances it.
__device__ void control(const Drop& d, const Sched& sc, Ctrl& c, Lds& s, int G) {
  {  // the workgroups' C13 violations and largest zeta' steps
    const bool wm = G > kSerialGroups;
    for_group_items(2, wm, [&](int i) {
      const double acc = group_item(i == 0 ? gl(d.vq_part) : gl(d.zr_part), 1, G, i == 1, wm);
      if (!wm || (threadIdx.x & 63) == 0) s.tmp[i] = acc;
    });
    __syncthreads();
  }
  Eval e;
  e.R = load_shared(&d.red[0]);
  e.P = load_shared(&d.red[1]);
  e.dm = load_shared(&d.red[2]);
  e.xres = load_shared(&d.red[3]);
  e.Vp = load_shared(&d.red[4]);
  e.Vs = load_shared(&d.red[5]);
  e.Vq = s.tmp[0];
  e.zres = s.tmp[1];
  e.changes = c.mode == kSweep ? load_shared(&d.chg_count[c.pass & 1]) : 0;
  __syncthreads();
  if (threadIdx.x == 0) advance(sc, c, e);
  __syncthreads();
}

__device__ inline PassConst pass_const(const Sched& sc, const Ctrl& c) {
  const bool update = c.mode == kSweep;
  PassConst pc;
  pc.E = c.E;
  pc.delta_v = sc.step0 / sqrt(1.0 + (double)c.v);
  pc.refit = update && sc.refit_period > 0 && (c.v % sc.refit_period) == 0;
  pc.reset = update && c.reset;
  pc.update = update;
  pc.write_out = c.mode == kEval || c.mode == kFinal;
  pc.rd = c.rd;
  pc.wr = c.wr;
  return pc;
}

__global__ void __launch_bounds__(kGridBlock) solve_kernel(Drop d, Sched sc) {
  extern __shared__ __align__(16) char smem[];
  __shared__ Lds s_tab;
  __shared__ Ctrl c;
  if (threadIdx.x == 0) {
    carve_lds((LDS char*)smem, d.M, d.K, d.L, sc.tile, blockDim.x, &s_tab, kAllParts, sc.sdev);
    if (sc.sdev) s_tab.Sg = d.S_part + (size_t)blockIdx.x * d.M * d.K;
    c = *d.ctrl;
  }
  __syncthreads();
  Lds& s = s_tab;
  cg::grid_group grid = cg::this_grid();
  const int b = blockIdx.x, G = gridDim.x;
  while (c.mode != kDone) {
    if (c.mode == kRepair) {
      for (int n = b * blockDim.x + threadIdx.x; n < d.N; n += G * blockDim.x) repair_subcarrier(d, c.rd, n);
      grid.sync();
      if (threadIdx.x == 0) c.mode = kFinal;
      __syncthreads();
      continue;
    }
    const PassConst pc = pass_const(sc, c);
    begin_pass(d, s, c.rd);
    const int nb = (d.N - b + G - 1) / G;  // my subcarriers: b, b+G, ...
    for (int j = 0; j < nb; j += sc.tile) tile<false>(BlockTeam{(int)threadIdx.x, (int)blockDim.x}, d, sc, pc, s, b + j * G, G,
                                                   min(sc.tile, nb - j));
    write_partials(d, s, b);
    grid.sync();
    reduce_pass(d, sc, c, s, b, G, pc.update, pc.delta_v);
    grid.sync();
    control(d, sc, c, s, G);
    if (b == 0 && threadIdx.x == 0) *d.ctrl = c;
  }
}

// ---------------------------------------------------------- batched solver

// Initial state of one drop inside a workgroup, by the same rules as the
// single-drop initial-point kernels.  Cold (no p0): association by the
// summed log2(1 + Gamma pmask / sigma) over n in increasing n, the l
// strongest users of each (m,n), p = pmax/(N l).  Warm (initial powers p0):
// the RRH of largest positive sum over n of p0 (else the cold one), the l
// users of largest positive p0 at min(p0, pmask).  xi' = max(xi0, 0) (else
// 0); zeta' = max(zeta0, 0) (else 1) for streaming users, 0 for elastic.
__device__ void block_start(const Drop& d, Lds& s) {
  const int M = d.M, N = d.N, K = d.K, L = d.L, tid = threadIdx.x, nth = blockDim.x;
  GLB const double* p0 = gl(d.p0);
  GLB double* const Sg = gl(s.Sg);  // (Sacc is u's storage when Sg is set)
  for (int i = tid; i < M * K; i += nth) {
    const int m = i / K, k = i - m * K;
    double acc = 0.0, pacc = 0.0;
    for (int n = 0; n < N; ++n) {
      const size_t gi = ((size_t)m * N + n) * K + k;
      acc += log2_1p((double)gl(d.G)[gi] * gl(d.pmask)[m] / d.sigma);
      if (p0) pacc += p0[gi];
    }
    if (Sg) Sg[i] = acc;
    else s.Sacc[i] = acc;
    s.u[i] = pacc;  // the tile arrays are free before the first pass
  }
  __syncthreads();
  for (int k = tid; k < K; k += nth) {
    int best = 0;
    double bv = -1.0;
    for (int m = 0; m < M; ++m) {
      const double v = Sg ? Sg[m * K + k] : s.Sacc[m * K + k];
      if (v > bv) {
        bv = v;
        best = m;
      }
    }
    if (p0) {
      int wb = -1;
      double wv = 0.0;
      for (int m = 0; m < M; ++m)
        if (s.u[m * K + k] > wv) {
          wv = s.u[m * K + k];
          wb = m;
        }
      if (wb >= 0) best = wb;
    }
    gl(d.A)[k] = best;  // state buffer 0
    gl(d.zeta)[k] = gl(d.elastic)[k] ? 0.0 : (d.zeta0 ? fmax(gl(d.zeta0)[k], 0.0) : 1.0);
  }
  for (int m = tid; m < M; m += nth) gl(d.xi)[m] = d.xi0 ? fmax(gl(d.xi0)[m], 0.0) : 0.0;
  __syncthreads();
  for (int i = tid; i < M * N; i += nth) {
    const int m = i / N, n = i - m * N;
    int bk[kMaxL];
    double bv[kMaxL];
    int cnt = 0;
    for (int k = 0; k < K; ++k) {
      if (gl(d.A)[k] != m) continue;
      const size_t gi = ((size_t)m * N + n) * K + k;
      double v;
      if (p0) {
        v = p0[gi];
        if (!(v > 0.0)) continue;
      } else {
        v = gl(d.G)[gi];
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
    const size_t base = ((size_t)m * N + n) * L;
    for (int a = 0; a < L; ++a) {
      gl(d.sel)[base + a] = a < cnt ? bk[a] : -1;
      gl(d.p)[base + a] = a < cnt ? (p0 ? fmin(bv[a], gl(d.pmask)[m]) : gl(d.pmax)[m] / ((double)N * L)) : 0.0;
      gl(d.al)[base + a] = 1.0;
      gl(d.be)[base + a] = 0.0;
      for (int b = 0; b < L; ++b) gl(d.zs)[(base + a) * L + b] = 0.0;
    }
  }
  __syncthreads();
}


// Reductions and multiplier steps of one pass from the workgroup's own
// accumulators (it holds every subcarrier of the drop); the pass's reduced
// values go to thread 0's *e.
__device__ void block_reduce(const Drop& d, const Sched& sc, int wr, Lds& s, bool update,
                             double delta_v, int* changes, unsigned long long* zres, Eval* e) {
  const int M = d.M, K = d.K, tid = threadIdx.x, nth = blockDim.x;
  GLB const double* const Sg = gl(s.Sg);  // the tiles' sums, visible after their last barrier
  double vq = 0.0;
  for (int k = tid; k < K; k += nth) {
    gl(d.user_rate)[k] = s.racc[k];
    const bool el = gl(d.elastic)[k];
    if (!el) vq += qos_viol(s.racc[k], gl(d.psi)[k]);
    if (!update) continue;
    const int before = s.Al[k];
    const auto S = [&](int m) { return Sg ? Sg[m * K + k] : s.Sacc[m * K + k]; };
    const int after = assoc_of(M, before, el, S);
    if (sc.tie_rel > 0.0 && assoc_near_tie(M, sc.tie_rel, S)) note_tie(d);
    gl(d.A)[(size_t)wr * K + k] = after;
    if (after != before) atomicAdd(changes, 1);
    if (!el) {
      double res;
      gl(d.zeta)[k] = zeta_step(gl(d.zeta)[k], gl(d.psi)[k], s.rhacc[k], delta_v, sc.qos_down, &res);
      if (res == res)
        __hip_atomic_fetch_max((LDS unsigned long long*)zres, (unsigned long long)__double_as_longlong(res),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  vq = block_sum(vq, s);
  if (tid == 0) {
    double R = 0.0, P = d.pstatic, dm = 0.0, Vp = 0.0, Vs = 0.0, xr = 0.0;
    for (int m = 0; m < M; ++m) {
      const double ps = s.psacc[m], pmax = gl(d.pmax)[m];
      R += s.Racc[m];
      P += gl(d.eta)[m] * s.peacc[m];
      dm = fmax(dm, s.dmax[m]);
      Vs += s.svacc[m];
      const double y = ps / pmax;
      if (y > 1.0 + kBudgetTol) Vp += y - (1.0 + kBudgetTol);
      if (update) {
        double res;
        gl(d.xi)[m] = xi_step(gl(d.xi)[m], ps, pmax, d.N, d.L, delta_v, &res);
        xr = fmax(xr, res);
      }
    }
    e->R = R;
    e->P = P;
    e->dm = dm;
    e->Vq = vq;
    e->Vp = Vp;
    e->Vs = Vs;
    e->xres = xr;
    e->zres = __longlong_as_double((long long)*zres);
    e->changes = *changes;
  }
  __syncthreads();
}

// Barrier of the G workgroups that solve one drop together.  All of them
// are resident (the persistent grid never exceeds what the device holds at
// once), so every wait ends; as a safety net a wait longer than
// kGroupWaitTicks of the 100 MHz constant clock marks the drop broken
// (bar[2]) and every rank leaves.  Returns false once the drop is broken.
constexpr unsigned long long kGroupWaitTicks = 2000000000ull;  // 20 s

__device__ bool group_sync(unsigned* bar, int G) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == (unsigned)G - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > kGroupWaitTicks) {
          __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ok = 0;
    __threadfence();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Initial loop control: the initial state is in buffer 0; a warm start's
// allocation (start_eval) is evaluated first.
__host__ __device__ inline Ctrl initial_ctrl(double pstatic, int start_eval) {
  Ctrl c0;
  memset(&c0, 0, sizeof c0);
  c0.P = pstatic;
  c0.mode = start_eval ? kEval : kSweep;
  c0.reset = 1;
  c0.rd = 0;
  c0.wr = 1;
  c0.best = 2;
  c0.first_eval = start_eval;
  return c0;
}

// Wave tiles: wave w of W runs subcarriers w, w + W, ... into its own
// accumulators, which are then summed in wave order.
__device__ __attribute__((always_inline)) void wave_pass(const Drop& d, const Sched& sd, const PassConst& pc, Lds& s, Lds* sw) {
  const int M = d.M, K = d.K, W = blockDim.x >> 6;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const WaveTeam tm{(int)(threadIdx.x & 63)};
  Lds& v = sw[w];
  for (int i = tm.tid; i < M * K; i += tm.nth) v.Sacc[i] = 0.0;
  for (int k = tm.tid; k < K; k += tm.nth) {
    v.racc[k] = 0.0;
    v.rhacc[k] = 0.0;
  }
  for (int m = tm.tid; m < M; m += tm.nth) {
    v.psacc[m] = 0.0;
    v.peacc[m] = 0.0;
    v.Racc[m] = 0.0;
    v.dmax[m] = 0.0;
    v.svacc[m] = 0.0;
  }
  tm.sync();
  const int nb = (d.N - w + W - 1) / W;  // subcarriers of this wave
  for (int j = 0; j < nb; j += d.wave) tile<true>(tm, d, sd, pc, v, w + j * W, W, min(d.wave, nb - j));
  __syncthreads();
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int i = tid; i < M * K; i += nth) {
    double a = 0.0;
    for (int u = 0; u < W; ++u) a += sw[u].Sacc[i];
    s.Sacc[i] = a;
  }
  for (int k = tid; k < K; k += nth) {
    double r = 0.0, rh = 0.0;
    for (int u = 0; u < W; ++u) {
      r += sw[u].racc[k];
      rh += sw[u].rhacc[k];
    }
    s.racc[k] = r;
    s.rhacc[k] = rh;
  }
  for (int m = tid; m < M; m += nth) {
    double ps = 0.0, pe = 0.0, R = 0.0, dm = 0.0, sv = 0.0;
    for (int u = 0; u < W; ++u) {
      ps += sw[u].psacc[m];
      pe += sw[u].peacc[m];
      R += sw[u].Racc[m];
      dm = fmax(dm, sw[u].dmax[m]);
      sv += sw[u].svacc[m];
    }
    s.psacc[m] = ps;
    s.peacc[m] = pe;
    s.Racc[m] = R;
    s.dmax[m] = dm;
    s.svacc[m] = sv;
  }
  __syncthreads();
}

// A drop solved by one workgroup, every reduction inside it.
__device__ __attribute__((always_inline)) void solve_single(const Drop& d, const Sched& sd, Lds& s, Lds* sw, Ctrl& s_c, int& s_changes,
                                                            unsigned long long& s_zres, Eval& s_e, Ctrl* out) {
  block_start(d, s);
  if (threadIdx.x == 0) s_c = initial_ctrl(d.pstatic, d.start_eval);
  __syncthreads();
  while (s_c.mode != kDone) {
    if (s_c.mode == kRepair) {
      for (int n = threadIdx.x; n < d.N; n += blockDim.x) repair_subcarrier(d, s_c.rd, n);
      __syncthreads();
      if (threadIdx.x == 0) s_c.mode = kFinal;
      __syncthreads();
      continue;
    }
    const PassConst pc = pass_const(sd, s_c);
    if (threadIdx.x == 0) {
      s_changes = 0;
      s_zres = 0ull;
    }
    begin_pass(d, s, pc.rd);
    if (d.wave > 0)
      wave_pass(d, sd, pc, s, sw);
    else
      for (int n0 = 0; n0 < d.N; n0 += sd.tile)
        tile<true>(BlockTeam{(int)threadIdx.x, (int)blockDim.x}, d, sd, pc, s, n0, 1, min(sd.tile, d.N - n0));
    block_reduce(d, sd, pc.wr, s, pc.update, pc.delta_v, &s_changes, &s_zres, &s_e);
    if (threadIdx.x == 0) advance(sd, s_c, s_e);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s_c;
  __syncthreads();
}

// A drop solved by G workgroups together, this one of rank r: the grid
// solver's pass (subcarriers r, r+G, ..., partials, fixed-order reductions)
// with the group barrier in place of the grid barrier.
__device__ __attribute__((always_inline)) void solve_group(const Drop& d, const Sched& sd, Lds& s, int r, int G, Ctrl& c,
                                                           Ctrl* out) {
  if (r == 0) {
    if (threadIdx.x == 0) {
      store_shared(&d.chg_count[0], 0);
      store_shared(&d.chg_count[1], 0);
    }
    block_start(d, s);
  }
  if (threadIdx.x == 0) c = initial_ctrl(d.pstatic, d.start_eval);
  bool ok = group_sync(d.bar, G);
  while (ok && c.mode != kDone) {
    if (c.mode == kRepair) {
      for (int n = r * blockDim.x + threadIdx.x; n < d.N; n += G * blockDim.x) repair_subcarrier(d, c.rd, n);
      if (!(ok = group_sync(d.bar, G))) break;
      if (threadIdx.x == 0) c.mode = kFinal;
      __syncthreads();
      continue;
    }
    const PassConst pc = pass_const(sd, c);
    begin_pass(d, s, c.rd);
    const int nb = (d.N - r + G - 1) / G;
    for (int j = 0; j < nb; j += sd.tile) tile<false>(BlockTeam{(int)threadIdx.x, (int)blockDim.x}, d, sd, pc, s, r + j * G, G,
                                                   min(sd.tile, nb - j));
    write_partials(d, s, r);
    if (!(ok = group_sync(d.bar, G))) break;
    reduce_pass(d, sd, c, s, r, G, pc.update, pc.delta_v);
    if (!(ok = group_sync(d.bar, G))) break;
    control(d, sd, c, s, G);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!ok) {
      c.flags |= ALLOC_GROUP_TIMEOUT;
      c.mode = kDone;
    }
    if (r == 0 || !ok) *out = c;
  }
  __syncthreads();
}

// Persistent batched solver.  Workgroups take slots from an atomic queue in
// the host's order (largest work per slot first); a slot is (drop, rank).  A
// drop with one slot is solved inside one workgroup; a drop with G slots by
// the G workgroups that take them, which meet at the drop's group barrier.
// Slots go out in order and every workgroup is resident, so the earliest
// unfinished drop always has all its ranks running: no group waits forever.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
batch_kernel(const Drop* __restrict__ drops, const int2* __restrict__ slots, int S, Sched sc, int* queue, Ctrl* ctrls) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_idx, s_changes;
  __shared__ unsigned long long s_zres;
  __shared__ Eval s_e;
  __shared__ Ctrl s_c;
  __shared__ Lds s_tab;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(queue, 1);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(s_idx);
    __syncthreads();
    if (idx >= S) break;
    const int2 sl = slots[idx];
    const Drop& d = drops[sl.x];
    Sched sd = sc;
    sd.tile = d.tile;
    if (threadIdx.x == 0) {
      if (d.wave > 0)
        carve_waves((LDS char*)smem, d.M, d.K, d.L, d.wave, blockDim.x >> 6, &s_tab);
      else
        carve_lds((LDS char*)smem, d.M, d.K, d.L, sd.tile, blockDim.x, &s_tab, kAllParts, d.sdev);
      if (d.sdev) s_tab.Sg = d.S_part + (size_t)sl.y * d.M * d.K;
    }
    __syncthreads();
    if (d.group <= 1)
      solve_single(d, sd, s_tab, (Lds*)smem, s_c, s_changes, s_zres, s_e, ctrls + sl.x);  // wave tables at smem
    else
      solve_group(d, sd, s_tab, sl.y, d.group, s_c, ctrls + sl.x);
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
    acc += log2_1p((double)gl(d.G)[((size_t)m * d.N + n) * d.K + k] * gl(d.pmask)[m] / d.sigma);
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
  gl(d.A)[k] = best;  // state buffer 0
  gl(d.zeta)[k] = gl(d.elastic)[k] ? 0.0 : 1.0;
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
    if (gl(d.A)[k] != m) continue;
    double v;
    if (p0) {
      v = p0[((size_t)m * d.N + n) * d.K + k];
      if (!(v > 0.0)) continue;
    } else {
      v = gl(d.G)[((size_t)m * d.N + n) * d.K + k];
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
    gl(d.sel)[base + a] = a < cnt ? bk[a] : -1;
    double pa = 0.0;
    if (a < cnt) pa = p0 ? fmin(bv[a], gl(d.pmask)[m]) : gl(d.pmax)[m] / ((double)d.N * L);
    gl(d.p)[base + a] = pa;
    gl(d.al)[base + a] = 1.0;
    gl(d.be)[base + a] = 0.0;
    for (int b = 0; b < L; ++b) gl(d.zs)[(base + a) * L + b] = 0.0;
  }
}

__global__ void p0_sum_kernel(Drop d, const double* p0, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.M * d.K) return;
  const int m = i / d.K, k = i - m * d.K;
  double acc = 0.0;
  for (int n = 0; n < d.N; ++n) acc += p0[((size_t)m * d.N + n) * d.K + k];
  out[i] = acc;
}

// Initial multipliers: xi' = max(xi0, 0) (0 without xi0); zeta' = max(zeta0, 0)
// for streaming users (1 without zeta0), 0 for elastic users.
__global__ void init_mult_kernel(Drop d, const double* xi0, const double* zeta0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.M) gl(d.xi)[i] = xi0 ? fmax(xi0[i], 0.0) : 0.0;
  if (i < d.K) gl(d.zeta)[i] = gl(d.elastic)[i] ? 0.0 : (zeta0 ? fmax(zeta0[i], 0.0) : 1.0);
}

// Dense [M][N][K] powers from the decoding-order slots.
__global__ void dense_kernel(Drop d, float* out) {
  const size_t total = (size_t)d.M * d.N * d.K;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = 0.0f;
}

// The RRH that serves each user in the returned selection (-1 unserved):
// cleared, then written by the (m,n) whose slots hold the user (one RRH per
// user, since one sweep's selection follows one association).
__global__ void rrh_clear_kernel(int K, int* rrh) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) rrh[k] = -1;
}

__global__ void rrh_from_sel_kernel(Drop d, int* rrh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.M * d.N) return;
  const int m = i / d.N;
  for (int a = 0; a < d.L; ++a) {
    const int k = gl(d.out_sel)[(size_t)i * d.L + a];
    if (k >= 0) rrh[k] = m;
  }
}

__global__ void scatter_kernel(Drop d, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.M * d.N) return;
  const int m = i / d.N, n = i - m * d.N;
  for (int a = 0; a < d.L; ++a) {
    const int k = gl(d.out_sel)[(size_t)i * d.L + a];
    if (k >= 0) out[((size_t)m * d.N + n) * d.K + k] = (float)gl(d.out_p)[(size_t)i * d.L + a];
  }
}

}  // namespace

// ==================================================================== host

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
  if (prm->sweeps_per_dinkelbach < 1 || prm->max_dinkelbach < 1 || prm->max_groups < 0 || prm->tile < 0 ||
      prm->group_triples < 0 || !(prm->tie_rel >= 0.0) || !std::isfinite(prm->tie_rel) ||
      prm->warm_max_dinkelbach < 0 ||
      prm->lds_kb < 0 || !(prm->block == 0 || prm->block == 256 || prm->block == 512 || prm->block == 1024) || prm->wave < 0 ||
      prm->wave > 16)
    return ALLOC_EINVAL;
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

// Subcarriers per tile for a workgroup that owns nb of them: the fewest
// tiles that fit (at most cap subcarriers each when cap > 0), of equal size
// but the last.  A phase takes as long as its fullest tile's items need
// rounds of the workgroup's threads: four tiles of 16 subcarriers run faster
// than tiles of 18, 18, 18 and 10.
template <class Fits>
int balanced_tile(int nb, int cap, Fits fits) {
  int T = cap > 0 ? std::min(cap, nb) : nb;
  while (T > 1 && !fits(T)) --T;
  const int tiles = (nb + T - 1) / T;
  return (nb + tiles - 1) / tiles;
}

// Subcarriers per tile for a workgroup of nth threads holding nb
// subcarriers, and whether the tiles sum the association metric in device
// memory (sdev) instead of LDS: the M*K sums then leave LDS to the tile,
// taken when that means fewer tiles per pass (each tile pays its barriers
// and its per-slot phases once), or when without it not even one
// subcarrier fits.
struct TileChoice {
  int T;
  bool sdev;
};
TileChoice choose_tile(int M, int K, int L, int nb, int cap, int nth, size_t budget, bool allow_sdev) {
  auto fits = [&](bool sd) {
    return [=](int t) { return carve_lds(nullptr, M, K, L, t, nth, nullptr, kAllParts, sd) <= budget; };
  };
  const int T0 = balanced_tile(nb, cap, fits(false));
  if (!allow_sdev) return {T0, false};
  const int T1 = balanced_tile(nb, cap, fits(true));
  const bool lds_fits = fits(false)(1);
  if (!lds_fits || (nb + T1 - 1) / T1 < (nb + T0 - 1) / T0) return {T1, true};
  return {T0, false};
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
  p->stall_sweeps = 30;
  p->tol_dinkelbach = 1e-6;
  p->tol_dual = 1e-7;
  p->step0 = 0.1;
  p->qos_down = 0.2;
  p->flags = 0;
  p->max_groups = 0;
  p->tile = 0;
  p->lds_kb = 0;
  p->block = 0;
  p->wave = 0;
  p->group_triples = 0;
  p->tie_rel = 0.0;
  p->warm_max_dinkelbach = 0;
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
    case ALLOC_EFILE: return "file could not be read or written, or is not a saved network";
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
  c->refs = 0;
  c->closed = 0;
  c->scratch = nullptr;
  if (hipGetSymbolAddress((void**)&c->scratch, HIP_SYMBOL(scratch)) != hipSuccess || !c->scratch) {
    delete c;
    return ALLOC_EDEVICE;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    delete c;
    return ALLOC_EDEVICE;
  }
  if (hipFuncSetAttribute((const void*)solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)c->lds_max - 1024) != hipSuccess) {
    delete c;
    return ALLOC_EDEVICE;
  }
  *out = c;
  return ALLOC_OK;
}

void alloc_ctx_destroy(alloc_ctx* c) {
  if (!c || c->closed) return;
  if (c->refs > 0) {  // batches or networks still use it: freed with the last of them
    c->closed = 1;
    return;
  }
  (void)hipSetDevice(c->device);
  if (c->ws) (void)hipFree(c->ws);
  (void)hipEventDestroy(c->ev0);
  (void)hipEventDestroy(c->ev1);
  delete c;
}

}  // extern "C"

namespace alloc_internal {

void ctx_retain(alloc_ctx* c) { ++c->refs; }

void ctx_release(alloc_ctx* c) {
  if (--c->refs == 0 && c->closed) {
    c->closed = 0;
    alloc_ctx_destroy(c);
  }
}

}  // namespace alloc_internal

namespace alloc_internal {

// Scalars and flags of a result from the final loop control and rates.
void finish_result(const Ctrl& cf, const double* ur, int K, unsigned ties, alloc_result* res) {
  uint32_t flags = cf.flags;
  if (ties > 0) flags |= ALLOC_NEAR_TIE;
  res->near_ties = (int32_t)std::min<unsigned>(ties, 0x7fffffffu);
  if (cf.Vq > 0.0) flags |= ALLOC_QOS_INFEASIBLE;
  if (cf.Vp > 0.0) flags |= ALLOC_BUDGET_INFEASIBLE;
  if (cf.Vs > 0.0) flags |= ALLOC_SIC_INFEASIBLE;
  for (int k = 0; k < K; ++k)
    if (!std::isfinite(ur[k])) flags |= ALLOC_NONFINITE;
  res->ee = cf.P > 0.0 ? cf.R / cf.P : 0.0;
  res->rate_sum = cf.R;
  res->power_sum = cf.P;
  res->viol_qos = cf.Vq;
  res->viol_budget = cf.Vp;
  res->viol_sic = cf.Vs;
  res->dinkelbach_iters = cf.i;
  res->sweeps = cf.total;
  res->status_flags = flags;
}

// alloc_solve on the context's grow-only workspace, or on a fixed one
// (fixed != nullptr: fixed_bytes of device memory; a problem whose layout
// needs more is rejected with ALLOC_ETOOBIG and nothing is allocated).
int solve_one_ws(alloc_ctx* ctx, const alloc_problem* pb, const alloc_params* prm, const alloc_warm* warm,
                 const DevWarm* dev, alloc_result* res, char* fixed, size_t fixed_bytes) {
  if (!ctx || !res) return ALLOC_EINVAL;
  if (warm && dev) return ALLOC_EINVAL;
  int rc = validate(pb, prm);
  if (rc != ALLOC_OK) return rc;
  const int M = pb->M, N = pb->N, K = pb->K, L = pb->l, NP = L * (L - 1) / 2;
  const size_t budget = ctx->lds_max - 1024;  // the kernel's static LDS stays below 1 KB
  if (carve_lds(nullptr, M, K, L, 1, kGridBlock, nullptr, kAllParts, true) > budget) return ALLOC_ETOOBIG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ALLOC_EDEVICE;
  const bool gain_dev = prm->flags & ALLOC_GAIN_ON_DEVICE;
  const bool out_dev = prm->flags & ALLOC_OUT_ON_DEVICE;
  if (!gain_dev) {  // host gains are validated here; device gains by the caller's contract
    const size_t n3 = (size_t)M * N * K;
    for (size_t i = 0; i < n3; ++i)
      if (!(pb->gain[i] > 0.0f) || !std::isfinite(pb->gain[i])) return ALLOC_EINVAL;
  }

  // grid: up to one workgroup per CU (the LDS tile fills a CU), at most one
  // per subcarrier; the tile is as many of a workgroup's subcarriers as fit.
  // When two subcarriers' triples fit one round of a workgroup's threads, a
  // workgroup takes two: half the workgroups at the grid barriers and in the
  // reductions for a tile that is hardly longer (a 5 x 64 x 32 drop: 32.7 ->
  // 29.8 ms).
  int G = std::min(N, ctx->cus);
  if (2 * M * K <= kGridBlock && N >= 2) G = std::min(G, (N + 1) / 2);
  if (prm->max_groups > 0) G = std::min(G, prm->max_groups);
  const int nb = (N + G - 1) / G;
  const TileChoice tc = choose_tile(M, K, L, nb, prm->tile, kGridBlock, budget, true);
  const int T = tc.T;
  const size_t lds = carve_lds(nullptr, M, K, L, T, kGridBlock, nullptr, kAllParts, tc.sdev);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)solve_kernel, kGridBlock, lds) !=
      hipSuccess)
    return ALLOC_EDEVICE;
  if (per_cu < 1) return ALLOC_ETOOBIG;
  G = std::min(G, per_cu * ctx->cus);

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
  const size_t oA = lay.add(sizeof(int) * 3 * K);  // three state buffers
  const size_t oSel = lay.add(sizeof(int) * 3 * ns);
  const size_t oP = lay.add(sizeof(double) * 3 * ns);
  const size_t oAl = lay.add(sizeof(double) * 3 * ns);
  const size_t oBe = lay.add(sizeof(double) * 3 * ns);
  const size_t oZs = lay.add(sizeof(double) * 3 * ns * L);
  const size_t oXi = lay.add(sizeof(double) * M);
  const size_t oZeta = lay.add(sizeof(double) * K);
  const size_t oSvp = lay.add(sizeof(double) * G);
  const size_t oVqp = lay.add(sizeof(double) * G);
  const size_t oZrp = lay.add(sizeof(double) * G);
  const size_t oSp = lay.add(sizeof(double) * G * M * K);
  const size_t oRp = lay.add(sizeof(double) * G * K);
  const size_t oRhp = lay.add(sizeof(double) * G * K);
  const size_t oPsp = lay.add(sizeof(double) * G * M);
  const size_t oPep = lay.add(sizeof(double) * G * M);
  const size_t oRP = lay.add(sizeof(double) * G);
  const size_t oDp = lay.add(sizeof(double) * G);
  const size_t oChg = lay.add(sizeof(int) * 3);  // two change counters and the near-tie count
  const size_t oRed = lay.add(sizeof(double) * 8);
  const size_t oUr = lay.add(sizeof(double) * K);
  const size_t oRrh = lay.add(sizeof(int) * K);
  const size_t oOs = lay.add(sizeof(int) * ns);
  const size_t oOp = lay.add(sizeof(double) * ns);
  const size_t oOz = lay.add(sizeof(double) * (size_t)M * N * (NP > 0 ? NP : 1));
  const size_t oCtrl = lay.add(sizeof(Ctrl));
  const size_t oSnr = lay.add(sizeof(double) * M * K);
  const bool h_p0 = warm && warm->p0, h_xi = warm && warm->xi0, h_z = warm && warm->zeta0;
  const bool has_p0 = h_p0 || (dev && dev->p0);
  const size_t oP0 = lay.add(h_p0 ? sizeof(double) * n3 : 0);
  const size_t oP0s = lay.add(has_p0 ? sizeof(double) * M * K : 0);
  const size_t oXi0 = lay.add(h_xi ? sizeof(double) * M : 0);
  const size_t oZ0 = lay.add(h_z ? sizeof(double) * K : 0);
  const size_t oDense = lay.add(res->power && !out_dev ? sizeof(float) * n3 : 0);
  char* ws;
  if (fixed) {
    if (lay.total > fixed_bytes) return ALLOC_ETOOBIG;
    ws = fixed;
  } else {
    if (lay.total > ctx->ws_bytes) {
      if (ctx->ws) (void)hipFree(ctx->ws);
      ctx->ws = nullptr;
      ctx->ws_bytes = 0;
      if (hipMalloc((void**)&ctx->ws, lay.total) != hipSuccess) return ALLOC_ENOMEM;
      ctx->ws_bytes = lay.total;
    }
    ws = ctx->ws;
  }
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
  if (h_p0) ok = ok && h2d(oP0, warm->p0, sizeof(double) * n3);
  if (h_xi) ok = ok && h2d(oXi0, warm->xi0, sizeof(double) * M);
  if (h_z) ok = ok && h2d(oZ0, warm->zeta0, sizeof(double) * K);
  // a warm initial allocation is Dinkelbach's p^0: evaluate it first
  const Ctrl c0 = initial_ctrl(pstatic, has_p0);
  ok = ok && h2d(oCtrl, &c0, sizeof c0);
  static const int zeros3[3] = {0, 0, 0};
  ok = ok && h2d(oChg, zeros3, sizeof zeros3);
  if (!ok) return ALLOC_EDEVICE;

  Drop d;
  memset(&d, 0, sizeof d);
  d.M = M; d.N = N; d.K = K; d.L = L; d.NP = NP;
  d.dv = make_divs(M, K, L);
  d.G = gain_dev ? pb->gain : (const float*)(ws + oG);
  d.gvec4 = K % 4 == 0 && ((uintptr_t)d.G & 15) == 0;
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
  d.sv_part = (double*)(ws + oSvp);
  d.vq_part = (double*)(ws + oVqp);
  d.zr_part = (double*)(ws + oZrp);
  d.S_part = (double*)(ws + oSp);
  d.r_part = (double*)(ws + oRp);
  d.rh_part = (double*)(ws + oRhp);
  d.psum_part = (double*)(ws + oPsp);
  d.pel_part = (double*)(ws + oPep);
  d.R_part = (double*)(ws + oRP);
  d.d_part = (double*)(ws + oDp);
  d.chg_count = (int*)(ws + oChg);
  d.ties = (unsigned*)(ws + oChg) + 2;
  d.red = (double*)(ws + oRed);
  d.user_rate = (double*)(ws + oUr);
  d.out_sel = (int*)(ws + oOs);
  d.out_p = (double*)(ws + oOp);
  d.out_zs = (double*)(ws + oOz);
  d.ctrl = (Ctrl*)(ws + oCtrl);

  // initial point
  const double* p0 = h_p0 ? (const double*)(ws + oP0) : (dev ? dev->p0 : nullptr);
  const double* xi0 = h_xi ? (const double*)(ws + oXi0) : (dev ? dev->xi0 : nullptr);
  const double* zeta0 = h_z ? (const double*)(ws + oZ0) : (dev ? dev->zeta0 : nullptr);
  double* p0s = p0 ? (double*)(ws + oP0s) : nullptr;
  const int tb = 256;
  hipLaunchKernelGGL(cold_assoc_kernel, dim3((M * K + tb - 1) / tb), dim3(tb), 0, st, d,
                     (double*)(ws + oSnr));
  if (p0) hipLaunchKernelGGL(p0_sum_kernel, dim3((M * K + tb - 1) / tb), dim3(tb), 0, st, d, p0, p0s);
  hipLaunchKernelGGL(cold_pick_kernel, dim3((K + tb - 1) / tb), dim3(tb), 0, st, d,
                     (const double*)(ws + oSnr), (const double*)p0s);
  hipLaunchKernelGGL(cold_select_kernel, dim3((M * N + tb - 1) / tb), dim3(tb), 0, st, d, p0);
  hipLaunchKernelGGL(init_mult_kernel, dim3((std::max(M, K) + tb - 1) / tb), dim3(tb), 0, st, d, xi0,
                     zeta0);
  if (hipGetLastError() != hipSuccess) return ALLOC_EDEVICE;

  Sched sc;
  sc.max_d = prm->max_dinkelbach;
  sc.sweeps = prm->sweeps_per_dinkelbach;
  sc.refit_period = prm->refit_period;
  sc.fixed = prm->fixed_count;
  sc.stall = prm->stall_sweeps;
  sc.tol_d = prm->tol_dinkelbach;
  sc.tol_dual = prm->tol_dual;
  sc.step0 = prm->step0;
  sc.qos_down = prm->qos_down;
  sc.tie_rel = prm->tie_rel;
  sc.tile = T;
  sc.sdev = tc.sdev;
  void* args[] = {(void*)&d, (void*)&sc};
  if (ctx->timing && hipEventRecord(ctx->ev0, st) != hipSuccess) return ALLOC_EDEVICE;
  if (hipLaunchCooperativeKernel((const void*)solve_kernel, dim3(G), dim3(kGridBlock), args, lds, st) !=
      hipSuccess)
    return ALLOC_EDEVICE;
  if (ctx->timing && hipEventRecord(ctx->ev1, st) != hipSuccess) return ALLOC_EDEVICE;

  // outputs
  int* rrh = (int*)(ws + oRrh);
  hipLaunchKernelGGL(rrh_clear_kernel, dim3((K + tb - 1) / tb), dim3(tb), 0, st, K, rrh);
  hipLaunchKernelGGL(rrh_from_sel_kernel, dim3((M * N + tb - 1) / tb), dim3(tb), 0, st, d, rrh);
  if (hipGetLastError() != hipSuccess) return ALLOC_EDEVICE;
  const hipMemcpyKind kind = out_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  auto d2o = [&](void* dst, const void* src, size_t bytes) {
    return !dst || hipMemcpyAsync(dst, src, bytes, kind, st) == hipSuccess;
  };
  ok = d2o(res->sel, d.out_sel, sizeof(int) * ns) && d2o(res->slot_power, d.out_p, sizeof(double) * ns) &&
       d2o(res->rrh_of_user, rrh, sizeof(int) * K) && d2o(res->xi, d.xi, sizeof(double) * M) &&
       d2o(res->zeta, d.zeta, sizeof(double) * K) && d2o(res->user_rate, d.user_rate, sizeof(double) * K);
  if (NP > 0) ok = ok && d2o(res->zeta_sic, d.out_zs, sizeof(double) * M * N * NP);
  if (!ok) return ALLOC_EDEVICE;
  if (res->power) {  // dense powers: written in place on the device, or staged in the workspace
    float* dense = out_dev ? res->power : (float*)(ws + oDense);
    hipLaunchKernelGGL(dense_kernel, dim3(std::min<size_t>((n3 + tb - 1) / tb, 65535)), dim3(tb), 0, st, d,
                       dense);
    hipLaunchKernelGGL(scatter_kernel, dim3((M * N + tb - 1) / tb), dim3(tb), 0, st, d, dense);
    if (!out_dev &&
        hipMemcpyAsync(res->power, dense, sizeof(float) * n3, hipMemcpyDeviceToHost, st) != hipSuccess)
      return ALLOC_EDEVICE;
  }
  Ctrl cf;
  if (hipMemcpyAsync(&cf, d.ctrl, sizeof cf, hipMemcpyDeviceToHost, st) != hipSuccess) return ALLOC_EDEVICE;
  unsigned ties = 0;
  if (hipMemcpyAsync(&ties, d.ties, sizeof ties, hipMemcpyDeviceToHost, st) != hipSuccess) return ALLOC_EDEVICE;
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
  finish_result(cf, ur.data(), K, ties, res);
  return ALLOC_OK;
}

int solve_one(alloc_ctx* ctx, const alloc_problem* pb, const alloc_params* prm, const alloc_warm* warm,
              const DevWarm* dev, alloc_result* res) {
  return solve_one_ws(ctx, pb, prm, warm, dev, res, nullptr, 0);
}

// Host side of one batched solve: the packed device layout of every drop's
// inputs, state and outputs, the drop descriptors and the launch shape.
struct BatchOff {
  size_t G, psi, el, pmax, eta, pmask, w, A, sel, p, al, be, zs, xi, zeta, ur, os, op, oz;
  size_t Sp, rp, rhp, psp, pep, Rp, dp, svp, vqp, zrp, chg, red, bar;  // group drops (Sp also for sums in device memory)
  size_t ties;                                          // near-tie count (zeroed with the barriers)
  size_t wp0, wxi, wz;                                  // host warm starts, staged
};

struct BatchPlan {
  int B = 0;
  char* ws = nullptr;
  bool gain_dev = false;
  size_t oDrops = 0, oSlots = 0, oQueue = 0, oCtrls = 0, out_begin = 0, out_end = 0;
  size_t bar_begin = 0, bar_end = 0;
  std::vector<BatchOff> off;
  std::vector<Drop> drops;
  std::vector<int2> slots;  // (drop, rank), largest work per slot first
  std::vector<int> group;
  std::vector<TileChoice> tiles;  // per drop: subcarriers per tile, sums in device memory
  std::vector<int> waves;         // per drop: subcarriers per wave tile, 0 = workgroup tiles
  std::vector<std::vector<double>> psis;
  std::vector<std::vector<uint8_t>> els;
  std::vector<int> Ms, Ns, Ks, Ls;
  Sched sc;
  int grid = 0;
  int threads = kGridBlock;
  size_t lds = 0;
};

// Start of a batched solve: the work queue and every group barrier (arrival
// count, generation, broken flag) cleared by a kernel, so a captured graph
// holds no memset node and a replay after a timed-out group starts clean.
__global__ void reset_queue_kernel(int* q, unsigned* bars, int nbar) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *q = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nbar; i += gridDim.x * blockDim.x) bars[i] = 0u;
}

// Validates, lays out and uploads the drops' inputs into *buf (grown to fit,
// *bytes its size); host warm starts (hw, [B] or null) are staged per drop.
int batch_prepare(alloc_ctx* ctx, int B, const alloc_problem* probs, const alloc_params* prm,
                  const alloc_warm* hw, char** buf, size_t* bytes, BatchPlan& P) {
  if (!ctx || !probs || B < 1 || !prm) return ALLOC_EINVAL;
  if (prm->flags & ALLOC_OUT_ON_DEVICE) return ALLOC_EINVAL;
  const bool gain_dev = prm->flags & ALLOC_GAIN_ON_DEVICE;
  for (int b = 0; b < B; ++b) {
    const int rc = validate(&probs[b], prm);
    if (rc != ALLOC_OK) return rc;
    if (!gain_dev) {
      const alloc_problem& pb = probs[b];
      const size_t n3 = (size_t)pb.M * pb.N * pb.K;
      for (size_t i = 0; i < n3; ++i)
        if (!(pb.gain[i] > 0.0f) || !std::isfinite(pb.gain[i])) return ALLOC_EINVAL;
    }
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return ALLOC_EDEVICE;
  // LDS per workgroup (dynamic part; the kernel's static LDS on top): the
  // whole CU, or the requested share, raised to what the largest drop needs;
  // with wave tiles and no request, what the largest wave-tiled drop needs
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, (const void*)batch_kernel) != hipSuccess) return ALLOC_EDEVICE;
  const size_t stat = fa.sharedSizeBytes;
  const size_t full = ctx->lds_max - stat;
  const int nthreads = prm->block > 0 ? prm->block : 512;
  const int nwaves = nthreads / 64;
  size_t need = 0, need_wave = 0;
  for (int b = 0; b < B; ++b) {
    const alloc_problem& pb = probs[b];
    need = std::max(need, carve_lds(nullptr, pb.M, pb.K, pb.l, 1, nthreads, nullptr, kAllParts, true));
    if (prm->wave > 0) {
      const size_t w = carve_waves(nullptr, pb.M, pb.K, pb.l, prm->wave, nwaves, nullptr);
      if (w <= full) need_wave = std::max(need_wave, w);
    }
  }
  if (need > full) return ALLOC_ETOOBIG;
  size_t budget = full;
  if (prm->lds_kb > 0)
    budget = std::max(need, std::min(full, (size_t)prm->lds_kb * 1024 - std::min<size_t>(stat, (size_t)prm->lds_kb * 1024)));
  else if (need_wave > 0)
    budget = std::max(need, need_wave);

  P.threads = nthreads;
  int per_cu = 0;
  if (hipFuncSetAttribute((const void*)batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)full) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)batch_kernel, nthreads, budget) !=
          hipSuccess)
    return ALLOC_EDEVICE;
  if (per_cu < 1) return ALLOC_ETOOBIG;
  int cap = per_cu * ctx->cus;  // workgroups resident at once
  if (prm->max_groups > 0) cap = std::min(cap, prm->max_groups);

  // workgroups per drop: with group_triples, a drop of more triples is
  // split over about triples/group_triples of them; otherwise a drop with
  // more work than 1.5 times the average share of a resident workgroup is
  // split over about work/average of them.  At most one per subcarrier and
  // no more than are resident.
  P.group.assign(B, 1);
  double wsum = 0.0;
  for (int b = 0; b < B; ++b) wsum += (double)probs[b].M * probs[b].N * probs[b].K;
  const double avg = prm->group_triples > 0 ? (double)prm->group_triples : wsum / cap;
  const double above = prm->group_triples > 0 ? 1.0 : 1.5;
  for (int b = 0; b < B; ++b) {
    const double w = (double)probs[b].M * probs[b].N * probs[b].K;
    if (w > above * avg)
      P.group[b] = (int)std::min<double>({std::floor(w / avg + 0.5), (double)cap, (double)probs[b].N});
    P.group[b] = std::max(1, P.group[b]);
  }
  P.tiles.assign(B, TileChoice{1, false});
  P.waves.assign(B, 0);
  for (int b = 0; b < B; ++b) {
    const alloc_problem& pb = probs[b];
    const int g = P.group[b];
    P.waves[b] = (g == 1 && prm->wave > 0 &&
                  carve_waves(nullptr, pb.M, pb.K, pb.l, prm->wave, nwaves, nullptr) <= budget)
                     ? prm->wave
                     : 0;
    const int nb = (pb.N + g - 1) / g;  // subcarriers of one rank
    P.tiles[b] = choose_tile(pb.M, pb.K, pb.l, nb, prm->tile, nthreads, budget, P.waves[b] == 0);
  }

  P.B = B;
  P.gain_dev = gain_dev;
  P.off.assign(B, BatchOff{});
  size_t tot = 0;
  auto add = [&](size_t n) {
    const size_t o = tot;
    tot += (n + 255) & ~size_t(255);
    return o;
  };
  int S = 0;
  for (int b = 0; b < B; ++b) S += P.group[b];
  P.oDrops = add(sizeof(Drop) * B);
  P.oSlots = add(sizeof(int2) * S);
  P.oQueue = add(sizeof(int));
  P.oCtrls = add(sizeof(Ctrl) * B);
  const size_t small_begin = tot;
  for (int b = 0; b < B; ++b) {
    const alloc_problem& pb = probs[b];
    const size_t M = pb.M, K = pb.K;
    P.off[b].psi = add(sizeof(double) * K);
    P.off[b].el = add(K);
    P.off[b].pmax = add(sizeof(double) * M);
    P.off[b].eta = add(sizeof(double) * M);
    P.off[b].pmask = add(sizeof(double) * M);
    P.off[b].w = add(pb.weight ? sizeof(double) * M * K : 0);
  }
  const size_t small_end = tot;
  P.out_begin = tot;
  for (int b = 0; b < B; ++b) {
    const alloc_problem& pb = probs[b];
    const size_t M = pb.M, N = pb.N, K = pb.K, L = pb.l, NP = L * (L - 1) / 2;
    P.off[b].os = add(sizeof(int) * M * N * L);
    P.off[b].op = add(sizeof(double) * M * N * L);
    P.off[b].oz = add(sizeof(double) * M * N * (NP > 0 ? NP : 1));
    P.off[b].xi = add(sizeof(double) * M);
    P.off[b].zeta = add(sizeof(double) * K);
    P.off[b].ur = add(sizeof(double) * K);
  }
  P.out_end = tot;
  if (hw)
    for (int b = 0; b < B; ++b) {
      const alloc_problem& pb = probs[b];
      P.off[b].wp0 = add(hw[b].p0 ? sizeof(double) * pb.M * pb.N * pb.K : 0);
      P.off[b].wxi = add(hw[b].xi0 ? sizeof(double) * pb.M : 0);
      P.off[b].wz = add(hw[b].zeta0 ? sizeof(double) * pb.K : 0);
    }
  for (int b = 0; b < B; ++b) {
    const alloc_problem& pb = probs[b];
    const size_t M = pb.M, N = pb.N, K = pb.K, L = pb.l;
    P.off[b].A = add(sizeof(int) * 3 * K);  // three state buffers
    P.off[b].sel = add(sizeof(int) * 3 * M * N * L);
    P.off[b].p = add(sizeof(double) * 3 * M * N * L);
    P.off[b].al = add(sizeof(double) * 3 * M * N * L);
    P.off[b].be = add(sizeof(double) * 3 * M * N * L);
    P.off[b].zs = add(sizeof(double) * 3 * M * N * L * L);
    P.off[b].G = add(gain_dev ? 0 : sizeof(float) * M * N * K);
    const size_t g = P.group[b];
    if (g > 1 || P.tiles[b].sdev) P.off[b].Sp = add(sizeof(double) * g * M * K);
    if (g > 1) {
      P.off[b].rp = add(sizeof(double) * g * K);
      P.off[b].rhp = add(sizeof(double) * g * K);
      P.off[b].psp = add(sizeof(double) * g * M);
      P.off[b].pep = add(sizeof(double) * g * M);
      P.off[b].Rp = add(sizeof(double) * g);
      P.off[b].dp = add(sizeof(double) * g);
      P.off[b].svp = add(sizeof(double) * g);
      P.off[b].vqp = add(sizeof(double) * g);
      P.off[b].zrp = add(sizeof(double) * g);
      P.off[b].chg = add(sizeof(int) * 2);
      P.off[b].red = add(sizeof(double) * 8);
    }
  }
  P.bar_begin = tot;
  for (int b = 0; b < B; ++b) P.off[b].ties = add(sizeof(unsigned));
  for (int b = 0; b < B; ++b)
    if (P.group[b] > 1) P.off[b].bar = add(sizeof(unsigned) * 3);
  P.bar_end = tot;
  if (tot > *bytes) {
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *bytes = 0;
    if (hipMalloc((void**)buf, tot) != hipSuccess) return ALLOC_ENOMEM;
    *bytes = tot;
  }
  char* ws = *buf;
  P.ws = ws;
  hipStream_t st = ctx->stream;

  // host image of the small inputs and the drop descriptors
  std::vector<char> img(small_end - small_begin, 0);
  P.drops.assign(B, Drop{});
  P.psis.assign(B, {});
  P.els.assign(B, {});
  P.Ms.resize(B);
  P.Ns.resize(B);
  P.Ks.resize(B);
  P.Ls.resize(B);
  for (int b = 0; b < B; ++b) {
    const alloc_problem& pb = probs[b];
    const int M = pb.M, N = pb.N, K = pb.K, L = pb.l;
    const BatchOff& o = P.off[b];
    P.Ms[b] = M;
    P.Ns[b] = N;
    P.Ks[b] = K;
    P.Ls[b] = L;
    double* psi = (double*)(img.data() + o.psi - small_begin);
    uint8_t* el = (uint8_t*)(img.data() + o.el - small_begin);
    P.psis[b].assign(K, 0.0);
    P.els[b].assign(K, 0);
    for (int k = 0; k < K; ++k) {
      el[k] = pb.user_type[k] == 0;
      psi[k] = el[k] ? 0.0 : min_rate(pb.arrival_bps[k], pb.delay_s[k], pb.packet_bits, pb.bw_hz);
      P.psis[b][k] = psi[k];
      P.els[b][k] = el[k];
    }
    memcpy(img.data() + o.pmax - small_begin, pb.pmax_w, sizeof(double) * M);
    memcpy(img.data() + o.eta - small_begin, pb.eta, sizeof(double) * M);
    double* pm = (double*)(img.data() + o.pmask - small_begin);
    for (int m = 0; m < M; ++m) pm[m] = pb.pmask_w ? pb.pmask_w[m] : pb.pmax_w[m] / N;
    if (pb.weight) memcpy(img.data() + o.w - small_begin, pb.weight, sizeof(double) * M * K);
    Drop& d = P.drops[b];
    memset(&d, 0, sizeof d);
    d.M = M; d.N = N; d.K = K; d.L = L; d.NP = L * (L - 1) / 2;
    d.dv = make_divs(M, K, L);
    d.G = gain_dev ? pb.gain : (const float*)(ws + o.G);
    d.gvec4 = K % 4 == 0 && ((uintptr_t)d.G & 15) == 0;
    d.psi = (const double*)(ws + o.psi);
    d.elastic = (const uint8_t*)(ws + o.el);
    d.pmax = (const double*)(ws + o.pmax);
    d.eta = (const double*)(ws + o.eta);
    d.pmask = (const double*)(ws + o.pmask);
    d.w = pb.weight ? (const double*)(ws + o.w) : nullptr;
    d.sigma = pb.noise_w;
    d.pstatic = pb.p_fiber_hpn + (M - 1) * pb.p_fiber_lpn + (M - 1) * pb.p_circuit_lpn + pb.p_circuit_hpn;
    d.A = (int*)(ws + o.A);
    d.sel = (int*)(ws + o.sel);
    d.p = (double*)(ws + o.p);
    d.al = (double*)(ws + o.al);
    d.be = (double*)(ws + o.be);
    d.zs = (double*)(ws + o.zs);
    d.xi = (double*)(ws + o.xi);
    d.zeta = (double*)(ws + o.zeta);
    d.user_rate = (double*)(ws + o.ur);
    d.out_sel = (int*)(ws + o.os);
    d.out_p = (double*)(ws + o.op);
    d.out_zs = (double*)(ws + o.oz);
    d.ties = (unsigned*)(ws + o.ties);
    const int g = P.group[b];
    d.group = g;
    if (g > 1 || P.tiles[b].sdev) d.S_part = (double*)(ws + o.Sp);
    if (g > 1) {
      d.r_part = (double*)(ws + o.rp);
      d.rh_part = (double*)(ws + o.rhp);
      d.psum_part = (double*)(ws + o.psp);
      d.pel_part = (double*)(ws + o.pep);
      d.R_part = (double*)(ws + o.Rp);
      d.d_part = (double*)(ws + o.dp);
      d.sv_part = (double*)(ws + o.svp);
      d.vq_part = (double*)(ws + o.vqp);
      d.zr_part = (double*)(ws + o.zrp);
      d.chg_count = (int*)(ws + o.chg);
      d.red = (double*)(ws + o.red);
      d.bar = (unsigned*)(ws + o.bar);
    }
    d.tile = P.tiles[b].T;
    d.sdev = P.tiles[b].sdev;
    d.wave = P.waves[b];
  }
  // slots, largest work per slot first; a drop's slots are consecutive
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  auto per_slot = [&](int b) { return (double)probs[b].M * probs[b].N * probs[b].K / P.group[b]; };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return per_slot(x) > per_slot(y); });
  P.slots.clear();
  for (int b : order)
    for (int r = 0; r < P.group[b]; ++r) P.slots.push_back(make_int2(b, r));
  bool ok = hipMemcpyAsync(ws + small_begin, img.data(), img.size(), hipMemcpyHostToDevice, st) == hipSuccess;
  if (!gain_dev)
    for (int b = 0; b < B && ok; ++b)
      ok = hipMemcpyAsync(ws + P.off[b].G, probs[b].gain, sizeof(float) * probs[b].M * probs[b].N * probs[b].K,
                          hipMemcpyHostToDevice, st) == hipSuccess;
  if (!ok) return ALLOC_EDEVICE;

  Sched& sc = P.sc;
  sc.max_d = prm->max_dinkelbach;
  sc.sweeps = prm->sweeps_per_dinkelbach;
  sc.refit_period = prm->refit_period;
  sc.fixed = prm->fixed_count;
  sc.stall = prm->stall_sweeps;
  sc.tol_d = prm->tol_dinkelbach;
  sc.tol_dual = prm->tol_dual;
  sc.step0 = prm->step0;
  sc.qos_down = prm->qos_down;
  sc.tie_rel = prm->tie_rel;
  sc.tile = 1;
  sc.sdev = 0;
  P.lds = budget;
  P.grid = std::min(S, cap);
  return ALLOC_OK;
}

// Points warm-started drops at their initial powers and multipliers (the
// batched kernel builds the initial state from them); host arrays are copied
// into the drop's staging area first.
int batch_warm(alloc_ctx* ctx, const alloc_problem* probs, const alloc_warm* warms, const WarmFn* fn,
               BatchPlan& P) {
  hipStream_t st = ctx->stream;
  char* ws = P.ws;
  for (int b = 0; b < P.B; ++b) {
    DevWarm w{nullptr, nullptr, nullptr};
    if (fn) {
      const int rc = (*fn)(b, &w);
      if (rc != ALLOC_OK) return rc;
    } else {
      const alloc_problem& pb = probs[b];
      const BatchOff& o = P.off[b];
      auto up = [&](size_t off, const double* src, size_t n) {
        return hipMemcpyAsync(ws + off, src, sizeof(double) * n, hipMemcpyHostToDevice, st) == hipSuccess;
      };
      if (warms[b].p0) {
        if (!up(o.wp0, warms[b].p0, (size_t)pb.M * pb.N * pb.K)) return ALLOC_EDEVICE;
        w.p0 = (const double*)(ws + o.wp0);
      }
      if (warms[b].xi0) {
        if (!up(o.wxi, warms[b].xi0, pb.M)) return ALLOC_EDEVICE;
        w.xi0 = (const double*)(ws + o.wxi);
      }
      if (warms[b].zeta0) {
        if (!up(o.wz, warms[b].zeta0, pb.K)) return ALLOC_EDEVICE;
        w.zeta0 = (const double*)(ws + o.wz);
      }
    }
    Drop& d = P.drops[b];
    d.p0 = w.p0;
    d.xi0 = w.xi0;
    d.zeta0 = w.zeta0;
    d.start_eval = w.p0 != nullptr;
  }
  return ALLOC_OK;
}

int batch_upload(hipStream_t st, const BatchPlan& P) {
  const bool ok =
      hipMemcpyAsync(P.ws + P.oDrops, P.drops.data(), sizeof(Drop) * P.B, hipMemcpyHostToDevice, st) ==
          hipSuccess &&
      hipMemcpyAsync(P.ws + P.oSlots, P.slots.data(), sizeof(int2) * P.slots.size(), hipMemcpyHostToDevice, st) ==
          hipSuccess;
  return ok ? ALLOC_OK : ALLOC_EDEVICE;
}

// The batched solve proper: queue reset and the persistent kernel (no host
// copies or memsets, so the pair can be captured into a graph).
int batch_enqueue(hipStream_t st, const BatchPlan& P) {
  const int nbar = (int)((P.bar_end - P.bar_begin) / sizeof(unsigned));
  hipLaunchKernelGGL(reset_queue_kernel, dim3(std::max(1, std::min(1024, (nbar + 255) / 256))), dim3(256), 0, st,
                     (int*)(P.ws + P.oQueue), (unsigned*)(P.ws + P.bar_begin), nbar);
  hipLaunchKernelGGL(batch_kernel, dim3(P.grid), dim3(P.threads), P.lds, st, (const Drop*)(P.ws + P.oDrops),
                     (const int2*)(P.ws + P.oSlots), (int)P.slots.size(), P.sc, (int*)(P.ws + P.oQueue),
                     (Ctrl*)(P.ws + P.oCtrls));
  return hipGetLastError() == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

// Outputs: one copy of the packed region, scattered on the host.
int batch_collect(hipStream_t st, const BatchPlan& P, alloc_result* results) {
  std::vector<char> out(P.out_end - P.out_begin);
  std::vector<Ctrl> ctrls(P.B);
  std::vector<char> bars(P.bar_end - P.bar_begin);  // near-tie counts and barrier words
  if (hipMemcpyAsync(out.data(), P.ws + P.out_begin, out.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(ctrls.data(), P.ws + P.oCtrls, sizeof(Ctrl) * P.B, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(bars.data(), P.ws + P.bar_begin, bars.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return ALLOC_EDEVICE;
  for (int b = 0; b < P.B; ++b) {
    alloc_result& r = results[b];
    const size_t M = P.Ms[b], N = P.Ns[b], K = P.Ks[b], L = P.Ls[b], NP = L * (L - 1) / 2;
    const BatchOff& o = P.off[b];
    auto src = [&](size_t off) { return out.data() + (off - P.out_begin); };
    if (r.sel) memcpy(r.sel, src(o.os), sizeof(int) * M * N * L);
    if (r.slot_power) memcpy(r.slot_power, src(o.op), sizeof(double) * M * N * L);
    if (r.zeta_sic && NP > 0) memcpy(r.zeta_sic, src(o.oz), sizeof(double) * M * N * NP);
    if (r.rrh_of_user) {  // the RRH whose slots hold each user, -1 unserved
      const int* os = (const int*)src(o.os);
      for (size_t k = 0; k < K; ++k) r.rrh_of_user[k] = -1;
      for (size_t i = 0; i < M * N; ++i)
        for (size_t a = 0; a < L; ++a)
          if (os[i * L + a] >= 0) r.rrh_of_user[os[i * L + a]] = (int)(i / N);
    }
    if (r.xi) memcpy(r.xi, src(o.xi), sizeof(double) * M);
    if (r.zeta) memcpy(r.zeta, src(o.zeta), sizeof(double) * K);
    const double* ur = (const double*)src(o.ur);
    if (r.user_rate) memcpy(r.user_rate, ur, sizeof(double) * K);
    if (r.power) {
      memset(r.power, 0, sizeof(float) * M * N * K);
      const int* os = (const int*)src(o.os);
      const double* op = (const double*)src(o.op);
      for (size_t i = 0; i < M * N; ++i)
        for (size_t a = 0; a < L; ++a)
          if (os[i * L + a] >= 0) r.power[i * K + os[i * L + a]] = (float)op[i * L + a];
    }
    unsigned ties;
    memcpy(&ties, bars.data() + (o.ties - P.bar_begin), sizeof ties);
    finish_result(ctrls[b], ur, (int)K, ties, &r);
  }
  return ALLOC_OK;
}

int solve_batch(alloc_ctx* ctx, int B, const alloc_problem* probs, const alloc_params* prm,
                const alloc_warm* warms, const WarmFn* fn, alloc_result* results) {
  if (!ctx || !probs || !results || B < 1 || !prm) return ALLOC_EINVAL;
  if (warms && fn) return ALLOC_EINVAL;
  BatchPlan P;
  int rc = batch_prepare(ctx, B, probs, prm, warms, &ctx->ws, &ctx->ws_bytes, P);
  if (rc) return rc;
  if ((warms || fn) && (rc = batch_warm(ctx, probs, warms, fn, P))) return rc;
  hipStream_t st = ctx->stream;
  if ((rc = batch_upload(st, P))) return rc;
  if (ctx->timing && hipEventRecord(ctx->ev0, st) != hipSuccess) return ALLOC_EDEVICE;
  if ((rc = batch_enqueue(st, P))) return rc;
  if (ctx->timing && hipEventRecord(ctx->ev1, st) != hipSuccess) return ALLOC_EDEVICE;
  if ((rc = batch_collect(st, P, results))) return rc;
  ctx->last_ms = -1.0;
  if (ctx->timing) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) != hipSuccess) return ALLOC_EDEVICE;
    ctx->last_ms = ms;
  }
  return ALLOC_OK;
}

}  // namespace alloc_internal

extern "C" {

int alloc_solve(alloc_ctx* ctx, const alloc_problem* pb, const alloc_params* prm, const alloc_warm* warm,
                alloc_result* res) {
  if (!prm || (ctx && ctx->closed)) return ALLOC_EINVAL;
  if (warm && (prm->flags & ALLOC_WARM_ON_DEVICE)) {
    const alloc_internal::DevWarm dw{warm->p0, warm->xi0, warm->zeta0};
    return alloc_internal::solve_one(ctx, pb, prm, nullptr, &dw, res);
  }
  return alloc_internal::solve_one(ctx, pb, prm, warm, nullptr, res);
}

struct alloc_batch {
  alloc_ctx* ctx;
  char* buf;
  size_t bytes;
  alloc_internal::BatchPlan plan;
  hipStream_t cap;
  hipGraph_t graph;
  hipGraphExec_t exec;
  double last_ms;
};

void alloc_batch_destroy(alloc_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->buf) (void)hipFree(b->buf);
  alloc_internal::ctx_release(b->ctx);
  delete b;
}

int alloc_batch_create(alloc_ctx* ctx, int32_t B, const alloc_problem* probs, const alloc_params* prm,
                       alloc_batch** out) {
  if (!ctx || !out || ctx->closed) return ALLOC_EINVAL;
  alloc_batch* b = new alloc_batch();
  b->ctx = ctx;
  alloc_internal::ctx_retain(ctx);
  b->last_ms = -1.0;
  int rc = alloc_internal::batch_prepare(ctx, B, probs, prm, nullptr, &b->buf, &b->bytes, b->plan);
  if (rc == ALLOC_OK) rc = alloc_internal::batch_upload(ctx->stream, b->plan);
  if (rc == ALLOC_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = ALLOC_EDEVICE;
  // capture on a stream of our own (the context's may be the null stream)
  if (rc == ALLOC_OK && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) rc = ALLOC_EDEVICE;
  if (rc == ALLOC_OK && hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    rc = ALLOC_EDEVICE;
  if (rc == ALLOC_OK) {
    const int erc = alloc_internal::batch_enqueue(b->cap, b->plan);
    const bool end_ok = hipStreamEndCapture(b->cap, &b->graph) == hipSuccess;
    rc = erc ? erc : (end_ok ? ALLOC_OK : ALLOC_EDEVICE);
  }
  if (rc == ALLOC_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = ALLOC_EDEVICE;
  if (rc) {
    alloc_batch_destroy(b);
    return rc;
  }
  *out = b;
  return ALLOC_OK;
}

int alloc_batch_run(alloc_batch* b) {
  if (!b) return ALLOC_EINVAL;
  alloc_ctx* c = b->ctx;
  if (hipSetDevice(c->device) != hipSuccess) return ALLOC_EDEVICE;
  if (c->timing && hipEventRecord(c->ev0, c->stream) != hipSuccess) return ALLOC_EDEVICE;
  if (hipGraphLaunch(b->exec, c->stream) != hipSuccess) return ALLOC_EDEVICE;
  if (c->timing && hipEventRecord(c->ev1, c->stream) != hipSuccess) return ALLOC_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return ALLOC_EDEVICE;
  b->last_ms = -1.0;
  if (c->timing) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) return ALLOC_EDEVICE;
    b->last_ms = ms;
  }
  return ALLOC_OK;
}

int alloc_batch_results(alloc_batch* b, alloc_result* results) {
  if (!b || !results) return ALLOC_EINVAL;
  return alloc_internal::batch_collect(b->ctx->stream, b->plan, results);
}

double alloc_batch_last_ms(alloc_batch* b) { return b ? b->last_ms : -1.0; }

int alloc_solve_noalloc(alloc_ctx* ctx, const alloc_problem* pb, const alloc_params* prm, alloc_result* res) {
  if (!ctx || !prm || ctx->closed) return ALLOC_EINVAL;
  return alloc_internal::solve_one_ws(ctx, pb, prm, nullptr, nullptr, res, ctx->scratch, kScratchBytes);
}

size_t alloc_noalloc_max_bytes(void) { return kScratchBytes; }

int alloc_solve_batch(alloc_ctx* ctx, int32_t B, const alloc_problem* probs, const alloc_params* prm,
                      const alloc_warm* warms, alloc_result* results) {
  if (!prm || (ctx && ctx->closed)) return ALLOC_EINVAL;
  if (warms && (prm->flags & ALLOC_WARM_ON_DEVICE)) {
    const alloc_internal::WarmFn fn = [warms](int b, alloc_internal::DevWarm* w) {
      w->p0 = warms[b].p0;
      w->xi0 = warms[b].xi0;
      w->zeta0 = warms[b].zeta0;
      return ALLOC_OK;
    };
    return alloc_internal::solve_batch(ctx, B, probs, prm, nullptr, &fn, results);
  }
  return alloc_internal::solve_batch(ctx, B, probs, prm, warms, nullptr, results);
}

}  // extern "C"
