// hcao_kernels.hip -- gfx950 kernels of the HCAO DSMC collision step.
//
// A workgroup owns a run of consecutive reservoir cells for several steps
// (persistent): it keeps the tables and the cells' headers in LDS, forms NTC
// candidate pairs from a keyed permutation, tests them with the VHS
// acceptance, runs the reaction decision / Larsen-Borgnakke relaxation /
// isotropic scattering of each accepted pair in one lane, and places products
// and removes recombined particles with wavefront ballots. Cells never
// exchange particles, so a launch needs no inter-workgroup communication and
// the result does not depend on the launch shape.
//
// Arithmetic is IEEE fp64 without contraction (built with -ffp-contract=off);
// log/exp are the library's own fixed-sequence versions, so that every
// decision is reproducible bit for bit. The mixed form (MIX) keeps fp32
// velocities, kinematics and sampler arithmetic and fp64 energies.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hcao_tables.h"

namespace hcao {
namespace {

constexpr double kBoltz = 1.380649e-23;
constexpr uint8_t kDead = 255;  // species byte of a particle removed by recombination

// Instrumented builds (HCAO_PHASE_CLOCKS) let thread 0 of every step
// workgroup sum the shader clock spent between the barriers that end each
// phase; the default build compiles the marks away.
#ifdef HCAO_PHASE_CLOCKS
#define HCAO_PHASE_MARK(k)               \
  do {                                   \
    if (tid == 0) {                      \
      const uint64_t t_ = clock64();     \
      clk_acc[k] += t_ - clk_t;          \
      clk_t = t_;                        \
    }                                    \
  } while (0)
// per-wave marks inside the collision phase: every active lane reads the
// (wave-uniform) clock, the leading active lane of the wave keeps the sums
#define HCAO_WAVE_MARK(acc, k)           \
  do {                                   \
    const uint64_t t_ = clock64();       \
    (acc)[(k) - kPhaseCollideGather] += t_ - (acc##_t); \
    acc##_t = t_;                        \
  } while (0)
#else
#define HCAO_PHASE_MARK(k) \
  do {                     \
  } while (0)
#define HCAO_WAVE_MARK(acc, k) \
  do {                         \
  } while (0)
#endif

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon et al., SC'11)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t k0, uint32_t k1, uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                         uint32_t &x3) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * x0, p1 = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t y0 = hi1 ^ x1 ^ k0;
    const uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
}

// A stream (seed; pair, cell, step). The fp64 form takes one 64-bit draw
// (two words, low first) per uniform, (u >> 11) 2^-53; the mixed form takes
// one 32-bit word per uniform, (w >> 8) 2^-24 (exact in either type).
template <bool MIX>
struct RngT {
  uint32_t k0, k1, pair, cell, step, block;
  uint32_t w0, w1, w2, w3;
  uint32_t used;  // words consumed from the current block

  __device__ __forceinline__ void open(uint64_t seed, uint32_t p, uint32_t c, uint32_t s) {
    k0 = (uint32_t)seed;
    k1 = (uint32_t)(seed >> 32);
    pair = p;
    cell = c;
    step = s;
    block = 0;
    used = 4;
  }
  __device__ __forceinline__ void refill() {
    uint32_t x0 = block, x1 = pair, x2 = cell, x3 = step;
    philox10(k0, k1, x0, x1, x2, x3);
    w0 = x0;
    w1 = x1;
    w2 = x2;
    w3 = x3;
    block += 1;
    used = 0;
  }
  __device__ __forceinline__ uint64_t next64() {
    if (used >= 4) refill();
    uint64_t r = (used == 0) ? (((uint64_t)w1 << 32) | w0) : (((uint64_t)w3 << 32) | w2);
    used += 2;
    return r;
  }
  __device__ __forceinline__ uint32_t next32() {
    if (used >= 4) refill();
    const uint32_t r = used == 0 ? w0 : (used == 1 ? w1 : (used == 2 ? w2 : w3));
    used += 1;
    return r;
  }
  __device__ __forceinline__ double uniform() {
    if (MIX) return (double)((float)(next32() >> 8) * 0x1p-24f);
    return (double)(next64() >> 11) * 0x1p-53;
  }
  __device__ __forceinline__ float uniform_f() { return (float)(next32() >> 8) * 0x1p-24f; }
  // passes over the next n uniforms of this form without using them (blocks
  // wholly passed over are not computed)
  __device__ __forceinline__ void skip(uint32_t n) {
    if (n == 0) return;
    const uint32_t words = MIX ? n : 2 * n;
    // word index within the stream of the next word to be used
    const uint32_t at = (used >= 4 ? 4 * block : 4 * (block - 1) + used) + words;
    const uint32_t b = at / 4, w = at % 4;
    if (w == 0) {
      block = b;
      used = 4;  // the next draw computes block b
    } else if (b != block - 1 || used >= 4) {
      block = b;
      refill();  // computes block b, block = b + 1
      used = w;
    } else {
      used = w;
    }
  }
  // a 53-bit uniform in either form: the next two words (low first); the
  // fp64 form's uniform() takes the same two words
  __device__ __forceinline__ double uniform53() {
    if (!MIX) return uniform();
    const uint64_t lo = next32();
    const uint64_t hi = next32();
    return (double)(((hi << 32) | lo) >> 11) * 0x1p-53;
  }
};
using Rng = RngT<false>;

// Arithmetic type of the velocities, kinematics and sampler draws: fp64 in
// the fp64 form, fp32 in the mixed form.
template <bool MIX>
struct RealOf {
  using type = double;
};
template <>
struct RealOf<true> {
  using type = float;
};
template <bool MIX>
using Real = typename RealOf<MIX>::type;

template <bool MIX>
__device__ __forceinline__ Real<MIX> draw(RngT<MIX> &rng) {
  if constexpr (MIX)
    return rng.uniform_f();
  else
    return rng.uniform();
}

template <typename R>
struct V3 {
  R x, y, z;
};
using Vec3 = V3<double>;

// velocity of slot i in the state's own precision
#ifdef HCAO_CHECKED
// Bounds-checked builds: an index outside [0, n) raises kErrBounds and is
// replaced by 0, so that no access leaves its array (the call then reports
// HCAO_EBOUNDS and its results are void).
__device__ __forceinline__ uint64_t checked_index(uint64_t i, uint64_t n, uint32_t *err) {
  if (i < n) return i;
  atomicOr(err, kErrBounds);
  return 0;
}
#define HCAO_IDX(i, n, err) checked_index((i), (n), (err))
#else
#define HCAO_IDX(i, n, err) (i)
#endif

template <bool MIX>
__device__ __forceinline__ V3<Real<MIX>> ldv(const State &s, uint64_t i) {
  if constexpr (MIX)
    return V3<float>{s.fx[i], s.fy[i], s.fz[i]};
  else
    return V3<double>{s.vx[i], s.vy[i], s.vz[i]};
}
template <bool MIX>
__device__ __forceinline__ void stv(const State &s, uint64_t i, V3<Real<MIX>> v) {
  if constexpr (MIX) {
    s.fx[i] = v.x;
    s.fy[i] = v.y;
    s.fz[i] = v.z;
  } else {
    s.vx[i] = v.x;
    s.vy[i] = v.y;
    s.vz[i] = v.z;
  }
}
// the same for kernels that serve both forms (the set that is not null)
__device__ __forceinline__ Vec3 load_vel(const State &s, uint64_t i) {
  if (s.fx) return Vec3{(double)s.fx[i], (double)s.fy[i], (double)s.fz[i]};
  return Vec3{s.vx[i], s.vy[i], s.vz[i]};
}
__device__ __forceinline__ void store_vel(const State &s, uint64_t i, double x, double y, double z) {
  if (s.fx) {
    s.fx[i] = (float)x;
    s.fy[i] = (float)y;
    s.fz[i] = (float)z;
  } else {
    s.vx[i] = x;
    s.vy[i] = y;
    s.vz[i] = z;
  }
}

// ---------------------------------------------------------------------------
// Fixed-sequence exp / log / pow (Cody-Waite reduction + fixed series)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dexp(double x) {
  const double kLn2Hi = 0x1.62e42feep-1;
  const double kLn2Lo = 0x1.a39ef35793c76p-33;
  const double kInvLn2 = 0x1.71547652b82fep+0;
  if (x != x) return x;
  if (x > 708.0) return __longlong_as_double(0x7ff0000000000000LL);
  if (x < -707.0) return 0.0;
  const double kd = floor(x * kInvLn2 + 0.5);
  const double r = (x - kd * kLn2Hi) - kd * kLn2Lo;
  double p = 1.0 / 355687428096000.0;  // 1/17!
  p = p * r + 1.0 / 20922789888000.0;
  p = p * r + 1.0 / 1307674368000.0;
  p = p * r + 1.0 / 87178291200.0;
  p = p * r + 1.0 / 6227020800.0;
  p = p * r + 1.0 / 479001600.0;
  p = p * r + 1.0 / 39916800.0;
  p = p * r + 1.0 / 3628800.0;
  p = p * r + 1.0 / 362880.0;
  p = p * r + 1.0 / 40320.0;
  p = p * r + 1.0 / 5040.0;
  p = p * r + 1.0 / 720.0;
  p = p * r + 1.0 / 120.0;
  p = p * r + 1.0 / 24.0;
  p = p * r + 1.0 / 6.0;
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  const long long k = (long long)kd;
  return p * __longlong_as_double((k + 1023) << 52);
}

__device__ __forceinline__ double dlog(double x) {
  const double kLn2Hi = 0x1.62e42feep-1;
  const double kLn2Lo = 0x1.a39ef35793c76p-33;
  const double kSqrt2 = 0x1.6a09e667f3bcdp+0;
  if (x != x) return x;
  if (x < 0.0) return __longlong_as_double(0x7ff8000000000000LL);
  if (x == 0.0) return __longlong_as_double((long long)0xfff0000000000000ULL);
  if (x == __longlong_as_double(0x7ff0000000000000LL)) return x;
  int e = 0;
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  if ((b >> 52) == 0) {
    x = x * 0x1p54;
    b = (unsigned long long)__double_as_longlong(x);
    e = -54;
  }
  e += (int)((b >> 52) & 0x7ff) - 1023;
  double m = __longlong_as_double((long long)((b & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL));
  if (m > kSqrt2) {
    m = m * 0.5;
    e += 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double q = 1.0 / 23.0;
  q = q * z + 1.0 / 21.0;
  q = q * z + 1.0 / 19.0;
  q = q * z + 1.0 / 17.0;
  q = q * z + 1.0 / 15.0;
  q = q * z + 1.0 / 13.0;
  q = q * z + 1.0 / 11.0;
  q = q * z + 1.0 / 9.0;
  q = q * z + 1.0 / 7.0;
  q = q * z + 1.0 / 5.0;
  q = q * z + 1.0 / 3.0;
  q = q * z + 1.0;
  const double t = s * q;
  const double lm = t + t;
  const double ed = (double)e;
  return (ed * kLn2Lo + lm) + ed * kLn2Hi;
}

__device__ __forceinline__ double dpow(double x, double y) {
  if (x == 0.0) return (y > 0.0) ? 0.0 : ((y == 0.0) ? 1.0 : __longlong_as_double(0x7ff0000000000000LL));
  return dexp(y * dlog(x));
}

// Exact comparisons against a power through a single-precision filter.
// est = 2^(y log2 x) from the hardware log2/exp2 (v_log_f32, v_exp_f32) is
// within 5e-6 of x^y for x in [2^-53, 2^64] and y in (0, 1] (measured over
// 1.7e7 operands); a decision further than kFilter from est is the one the
// fp64 power gives, and only the band in between evaluates dpow. The
// result of every comparison is therefore that of the fp64 expression.
// Quantum numbers of slot i, a row of s.lrow uint16 read and written as
// dwords (two modes each). load_levels unpacks the first n modes to
// dst[m * ds]; store_levels packs src[m * ss] for m < n and zeros for
// n <= m < top (top >= n: modes only the old species had), in whole dwords
// (a mode past top in the last dword is 0 in the state and stays 0).
__device__ __forceinline__ void load_levels(const State &s, uint64_t i, uint32_t n, uint16_t *dst, uint32_t ds) {
  const uint32_t *row = reinterpret_cast<const uint32_t *>(s.lvl + i * s.lrow);
  for (uint32_t w = 0; 2 * w < n; ++w) {
    const uint32_t x = row[w];
    dst[2 * w * ds] = (uint16_t)(x & 0xFFFFu);
    if (2 * w + 1 < n) dst[(2 * w + 1) * ds] = (uint16_t)(x >> 16);
  }
}
__device__ __forceinline__ void store_levels(const State &s, uint64_t i, uint32_t n, uint32_t top, const uint16_t *src,
                                             uint32_t ss) {
  uint32_t *row = reinterpret_cast<uint32_t *>(s.lvl + i * s.lrow);
  for (uint32_t w = 0; 2 * w < top; ++w) {
    const uint32_t lo = 2 * w < n ? src[2 * w * ss] : 0u;
    const uint32_t hi = 2 * w + 1 < n ? src[(2 * w + 1) * ss] : 0u;
    row[w] = lo | (hi << 16);
  }
}
// the whole row of slot from to slot to (dwords)
__device__ __forceinline__ void copy_levels(const State &src, uint64_t from, const State &dst, uint64_t to) {
  const uint32_t *a = reinterpret_cast<const uint32_t *>(src.lvl + from * src.lrow);
  uint32_t *b = reinterpret_cast<uint32_t *>(dst.lvl + to * dst.lrow);
  for (uint32_t w = 0; w < src.lrow / 2; ++w) b[w] = a[w];
}

// The value lane + S holds, delivered to the lanes that a halving tree
// reads at level S (lane < S); other lanes receive arbitrary values. VALU
// cross-lane moves of gfx950 instead of LDS-routed shuffles: the 32- and
// 16-lane swaps for S = 32 and 16, DPP row shifts for S = 8 .. 1.
template <int S>
__device__ __forceinline__ uint32_t lane_down(uint32_t v) {
  if constexpr (S == 32)
    return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
  else if constexpr (S == 16)
    return __builtin_amdgcn_permlane16_swap(v, v, false, false)[1];
  else
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x100 + S, 0xF, 0xF, false);
}
template <int S>
__device__ __forceinline__ double tree_down(double v) {
  const uint32_t lo = lane_down<S>((uint32_t)__double2loint(v));
  const uint32_t hi = lane_down<S>((uint32_t)__double2hiint(v));
  return __hiloint2double((int)hi, (int)lo);
}
// Halving tree over the 64 lanes of a wave (lane t adds lane t + s, s = 32
// .. 1): lane 0 ends with the sum, in that order; every lane must be active.
template <int N>
__device__ __forceinline__ void tree_sum(double (&y)[N]) {
#pragma unroll
  for (int x = 0; x < N; ++x) y[x] = y[x] + tree_down<32>(y[x]);
#pragma unroll
  for (int x = 0; x < N; ++x) y[x] = y[x] + tree_down<16>(y[x]);
#pragma unroll
  for (int x = 0; x < N; ++x) y[x] = y[x] + tree_down<8>(y[x]);
#pragma unroll
  for (int x = 0; x < N; ++x) y[x] = y[x] + tree_down<4>(y[x]);
#pragma unroll
  for (int x = 0; x < N; ++x) y[x] = y[x] + tree_down<2>(y[x]);
#pragma unroll
  for (int x = 0; x < N; ++x) y[x] = y[x] + tree_down<1>(y[x]);
}

constexpr double kFilter = 1e-4;

__device__ __forceinline__ double pow_estimate(double x, double y) {
  return (double)__builtin_amdgcn_exp2f((float)y * __builtin_amdgcn_logf((float)x));
}

// u < x^y (as dpow computes it), for x in (0, 1] and y in (0, 1]
__device__ __forceinline__ bool below_pow(double u, double x, double y) {
  const double est = pow_estimate(x, y);
  if (u < est * (1.0 - kFilter)) return true;
  if (u > est * (1.0 + kFilter)) return false;
  return u < dpow(x, y);
}

// x^y in single precision (mixed form)
__device__ __forceinline__ float pow_f(float x, float y) {
  return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
}

// Larsen-Borgnakke acceptance u < (num / den)^q for num, den > 0: the fp64
// form divides in fp64 and decides as the fp64 power does; the mixed form
// takes the ratio and the power in fp32 (u is then an fp32 draw)
template <bool MIX>
__device__ __forceinline__ bool lb_accept(double u, double num, double den, double q) {
  if constexpr (MIX)
    return (float)u < pow_f((float)num / (float)den, (float)q);
  else
    return below_pow(u, num / den, q);
}

// ---------------------------------------------------------------------------
// keyed permutation of [0, n): Feistel network on Z_m x Z_m, m = ceil(sqrt n),
// with addition modulo m (generalised Feistel cipher, Black-Rogaway), 16
// rounds for m <= 8 and 10 above, cycle walking into [0, n) (m^2 / n < 1.2
// for n >= 25, so walks are short). The round function multiplies 24-bit
// factors (full-rate v_mul_u32_u24) and scales the hash to [0, m) by its
// high product with m.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t feistel_f(uint32_t r, uint32_t key, uint32_t m) {
  uint32_t h = __umul24(r ^ key, 0x9E3779u);
  h ^= h >> 15;
  h = __umul24(h, 0x85EBCBu);
  h ^= h >> 13;
  return __umulhi(h, m);
}

struct Perm {
  uint32_t n, m, pad, rounds;
  uint32_t k[16];
};

// the permutation evaluated with its keys in registers
struct PermReg {
  uint32_t n, m, rounds;
  uint32_t k[16];
  __device__ __forceinline__ void load(const Perm &P) {
    n = P.n;
    m = P.m;
    rounds = P.rounds;
#pragma unroll
    for (int i = 0; i < 16; ++i) k[i] = P.k[i];
  }
  template <int R>
  __device__ __forceinline__ void once_r(uint32_t &l, uint32_t &r) const {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      uint32_t s = l + feistel_f(r, k[i], m);
      s = s >= m ? s - m : s;
      l = r;
      r = s;
    }
  }
  __device__ __forceinline__ void once(uint32_t &l, uint32_t &r) const {
    if (rounds == 10)
      once_r<10>(l, r);
    else
      once_r<16>(l, r);
  }
  __device__ __forceinline__ uint32_t operator()(uint32_t i) const {
    uint32_t l = i / m, r = i - l * m;
    once(l, r);
    while (l * m + r >= n) once(l, r);
    return l * m + r;
  }
};

__device__ __forceinline__ void make_perm(Perm &P, uint32_t n, uint64_t seed, uint32_t cell, uint32_t step) {
  P.n = n;
  uint32_t m = (uint32_t)sqrtf((float)n);
  while (m * m < n) ++m;
  while (m > 1 && (m - 1) * (m - 1) >= n) --m;
  P.m = m;
  P.pad = 0;
  P.rounds = m <= 8 ? 16u : 10u;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (uint32_t blk = 0; blk < 4; ++blk) {
    uint32_t x0 = blk, x1 = 0xFFFFFFFFu, x2 = cell, x3 = step;
    philox10(k0, k1, x0, x1, x2, x3);
    P.k[4 * blk] = x0;
    P.k[4 * blk + 1] = x1;
    P.k[4 * blk + 2] = x2;
    P.k[4 * blk + 3] = x3;
  }
}

// ---------------------------------------------------------------------------
// tables in LDS
// ---------------------------------------------------------------------------
// species / pair / reaction tables and stretch levels, staged in LDS
struct Tab {
  const SpeciesTab *sp;
  const PairTab *pr;  // [a * ns + b]
  const ReactionTab *rx;
  const double *lev;
  const double *beta;  // exact sampler's beta tables (global memory)
  uint32_t ns, nr, mm, rec_nt;
  __device__ __forceinline__ const PairTab &pair(uint32_t a, uint32_t b) const { return pr[a * ns + b]; }
};

struct Ctx {
  Tab T;
  unsigned long long *ctr;  // LDS counters of the pair's cell
  uint16_t *scr;            // per-lane scratch, [2 * max_modes][block]
  uint32_t lane, block;
};

__device__ __forceinline__ double mode_energy(const SpeciesTab &S, const double *lev, uint32_t m, uint32_t i) {
  if (m < S.n_bend) return ((double)i + 0.5) * S.kt[m];
  return lev[S.lev_off[m] + i];
}

__device__ __forceinline__ double vib_energy(const SpeciesTab &S, const double *lev, const uint16_t *lv,
                                             uint32_t stride) {
  double e = 0.0;
  for (uint32_t m = 0; m < S.n_modes; ++m) e = e + mode_energy(S, lev, m, lv[m * stride]);
  return e;
}

// top quantum number a mode may be proposed at, given the energy e it may hold
__device__ __forceinline__ uint32_t mode_top(const SpeciesTab &S, const double *lev, uint32_t m, double e) {
  if (m < S.n_bend) {
    double fi = floor(e / S.kt[m] - 0.5);
    fi = fi < 0.0 ? 0.0 : fi;
    fi = fi > 65535.0 ? 65535.0 : fi;
    return (uint32_t)fi;
  }
  // highest level strictly below e (the table increases strictly), at least 0
  const double *L = lev + S.lev_off[m];
  uint32_t lo = 0, hi = S.idiss[m];
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (L[mid] < e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// uniform level on 0..top from one draw: min(floor(u (top + 1)), top)
template <bool MIX>
__device__ __forceinline__ uint32_t pick_level(uint32_t top, RngT<MIX> &rng) {
  uint32_t i;
  if constexpr (MIX)
    i = (uint32_t)(rng.uniform_f() * (float)(top + 1));
  else
    i = (uint32_t)floor(rng.uniform() * ((double)top + 1.0));
  return i > top ? top : i;
}

// u < exp(-a) for a >= 0, decided as the fp64 dexp decides (fp32 filter)
__device__ __forceinline__ bool below_exp_neg(double u, double a) {
  const double est = (double)__builtin_amdgcn_exp2f(-(float)a * 1.44269504f);
  if (u < est * (1.0 - kFilter)) return true;
  if (u > est * (1.0 + kFilter)) return false;
  return u < dexp(-a);
}

// Exact sampler, level proposal of one mode: the geometric level
// floor(-ln(1 - u) / c) with c = beta * slope. Returns false when it lies
// above top (the caller draws again). The fp64 form decides floor() as the
// fp64 expression -dlog(1 - u) / c does: an fp32 estimate far enough from
// an integer settles it, else the fp64 expression is evaluated.
template <bool MIX>
__device__ __forceinline__ bool geometric_level(RngT<MIX> &rng, double c, uint32_t top, uint32_t &i) {
  const float ftop1 = (float)top + 1.0f;
  if constexpr (MIX) {
    const float u = rng.uniform_f();
    const float x = -__builtin_amdgcn_logf(1.0f - u) * (0.69314718f / (float)c);
    if (!(x < ftop1)) return false;
    i = (uint32_t)floorf(x);
    return true;
  } else {
    const double u = rng.uniform();
    const double v = 1.0 - u;
    const float k = (float)(0.6931471805599453 / c);
    const float xe = -__builtin_amdgcn_logf((float)v) * k;
    const float band = 1e-5f * (xe + 1.0f) + 1e-6f * k;
    if (xe >= ftop1 + band) return false;
    const float fl = floorf(xe);
    if (xe - fl > band && (fl + 1.0f) - xe > band) {
      i = (uint32_t)fl;
      return true;
    }
    const double x = -dlog(v) / c;
    if (!(x < (double)top + 1.0)) return false;
    i = (uint32_t)floor(x);
    return true;
  }
}

// Exact sampler, slope of the geometric proposal of mode m on 0..top: the
// harmonic spacing of a bend; for a stretch the chord (E_top - E_0) / top,
// a lower bound of (E_i - E_0) / i when the spacings never grow, else the
// smallest (E_i - E_0) / i
__device__ __forceinline__ double exact_slope(const SpeciesTab &S, const double *lev, uint32_t m, uint32_t top) {
  if (m < S.n_bend) return S.kt[m];
  const double *L = lev + S.lev_off[m];
  if ((S.concave >> m) & 1u) return (L[top] - L[0]) / (double)top;
  double sl = L[1] - L[0];
  for (uint32_t i = 2; i <= top; ++i) {
    const double v = (L[i] - L[0]) / (double)i;
    if (v < sl) sl = v;
  }
  return sl;
}

// Larsen-Borgnakke relaxation of one molecule (levels at lv[m * stride]);
// e_tr is the pair's translational energy on entry and exit; btab is the
// molecule's beta table (exact sampler only). The exact sampler is compiled
// only into the instantiations with EX set, which run when some species
// uses it, so that it does not weigh on the register allocation of the
// others.
template <bool MIX, bool EX>
__device__ uint32_t relax(const Ctx &C, const SpeciesTab &S, uint16_t *lv, uint32_t stride, double &e_tr,
                          double q, const double *btab, RngT<MIX> &rng, bool &capped) {
  uint32_t trials = 0;
  capped = false;
  const uint32_t nm = S.n_modes;
  if (EX && S.sampler == HCAO_SAMPLER_EXACT) {
    // Independent draw from the joint target (E' - S)^q on S < E' (S: sum of
    // the modes' energies above their ground levels, E' = E_coll - ZPE) by
    // rejection from per-mode Boltzmann proposals at inverse temperature
    // beta: bends geometric, stretches geometric on the chord slope thinned
    // by exp(-beta (E_i - E_0 - slope i)); target / proposal over its
    // maximum is exp(q (ln y + 1 - y)), y = beta (E' - S) / q.
    const double e_coll = e_tr + vib_energy(S, C.T.lev, lv, stride);
    const double ep = e_coll - S.zpe;
    if (!(ep > 0.0)) return 0;
    uint32_t bin = (uint32_t)((unsigned long long)__double_as_longlong(ep) >> 48);
    bin = bin < kExactBinLo ? kExactBinLo : (bin > kExactBinHi ? kExactBinHi : bin);
    double beta = btab[bin - kExactBinLo];
    if (beta * ep < q) beta = q / ep;
    uint16_t *tops = C.scr + C.lane;
    uint16_t *cand = C.scr + (size_t)nm * C.block + C.lane;
    for (uint32_t m = 0; m < nm; ++m)
      tops[m * C.block] = (uint16_t)mode_top(S, C.T.lev, m, ep + mode_energy(S, C.T.lev, m, 0));
    for (;;) {
      double sum = 0.0;
      for (uint32_t m = 0; m < nm && !capped; ++m) {
        const uint32_t top = tops[m * C.block];
        uint32_t i = 0;
        if (top > 0) {
          const double sl = exact_slope(S, C.T.lev, m, top);
          const double c = beta * sl;
          for (;;) {
            ++trials;
            if (trials >= kMaxTrials) {
              capped = true;
              break;
            }
            if (!geometric_level<MIX>(rng, c, top, i)) continue;
            if (m >= S.n_bend && i > 0) {
              const double d = (mode_energy(S, C.T.lev, m, i) - mode_energy(S, C.T.lev, m, 0)) - sl * (double)i;
              if (d > 0.0) {
                bool keep;
                if constexpr (MIX)
                  keep = rng.uniform_f() < __builtin_amdgcn_exp2f(-(float)(beta * d) * 1.44269504f);
                else
                  keep = below_exp_neg(rng.uniform(), beta * d);
                if (!keep) continue;
              }
            }
            break;
          }
        }
        cand[m * C.block] = (uint16_t)i;
        sum = sum + (mode_energy(S, C.T.lev, m, i) - mode_energy(S, C.T.lev, m, 0));
      }
      if (capped) break;
      ++trials;
      if (sum < ep) {
        const double y = (beta * (ep - sum)) / q;
        bool ok;
        if constexpr (MIX) {
          const float yf = (float)y, qf = (float)q;
          const float ex = qf * ((__builtin_amdgcn_logf(yf) * 0.69314718f + 1.0f) - yf);
          ok = rng.uniform_f() < __builtin_amdgcn_exp2f(ex * 1.44269504f);
        } else {
          const double ua = rng.uniform();
          const float yf = (float)y, qf = (float)q;
          const float ex = qf * ((__builtin_amdgcn_logf(yf) * 0.69314718f + 1.0f) - yf);
          const double est = (double)__builtin_amdgcn_exp2f(ex * 1.44269504f);
          if (ua < est * (1.0 - kFilter))
            ok = true;
          else if (ua > est * (1.0 + kFilter))
            ok = false;
          else
            ok = ua < dexp(q * ((dlog(y) + 1.0) - y));
        }
        if (ok) {
          double ev = 0.0;
          for (uint32_t m = 0; m < nm; ++m) {
            const uint16_t l = cand[m * C.block];
            lv[m * stride] = l;
            ev = ev + mode_energy(S, C.T.lev, m, l);
          }
          e_tr = e_coll - ev;
          break;
        }
      }
      if (trials >= kMaxTrials) {
        capped = true;
        break;
      }
    }
    return trials;
  }
  if (S.sampler == HCAO_SAMPLER_JOINT) {
    const double e_coll = e_tr + vib_energy(S, C.T.lev, lv, stride);
    const double denom = e_coll - S.zpe;
    if (!(denom > 0.0)) return 0;
    uint16_t *tops = C.scr + C.lane;
    uint16_t *cand = C.scr + (size_t)nm * C.block + C.lane;
    for (uint32_t m = 0; m < nm; ++m) tops[m * C.block] = (uint16_t)mode_top(S, C.T.lev, m, e_coll);
    for (;;) {
      ++trials;
      double sum = 0.0;
      for (uint32_t m = 0; m < nm; ++m) {
        const uint32_t i = pick_level<MIX>(tops[m * C.block], rng);
        cand[m * C.block] = (uint16_t)i;
        sum = sum + mode_energy(S, C.T.lev, m, i);
      }
      const double ua = (double)draw<MIX>(rng);
      const bool ok = (sum < e_coll) && lb_accept<MIX>(ua, e_coll - sum, denom, q);
      if (ok) {
        for (uint32_t m = 0; m < nm; ++m) lv[m * stride] = cand[m * C.block];
        e_tr = e_coll - sum;
        break;
      }
      if (trials >= kMaxTrials) {
        capped = true;
        break;
      }
    }
    return trials;
  }
  // Gibbs sweep: the level of mode m is proposed from the linear envelope
  // w_i = 1 - c i of the target ((E_c - E_i) / (E_c - E_0))^q on 0..top
  // (valid for q <= 1 and levels whose spacings never grow; c = 0 gives the
  // uniform proposal) by inverting its discrete CDF, and accepted with
  // probability target / w_i.
  double et = e_tr;
  for (uint32_t m = 0; m < nm; ++m) {
    const double ec = et + mode_energy(S, C.T.lev, m, lv[m * stride]);
    const double e0 = mode_energy(S, C.T.lev, m, 0);
    const double den = ec - e0;
    if (!(den > 0.0)) continue;
    const uint32_t top = mode_top(S, C.T.lev, m, ec);
    double c = 0.0;
    if (top > 0 && ((S.concave >> m) & 1u))
      c = (q * (mode_energy(S, C.T.lev, m, top) - e0)) / ((double)top * den);
    const double z = ((double)top + 1.0) * (1.0 - (0.5 * c) * (double)top);
    const double h = 1.0 + 0.5 * c;
    const double hh = h * h, c2 = 2.0 * c;
    for (;;) {
      ++trials;
      uint32_t i;
      double w;
      if constexpr (MIX) {
        const float sv = rng.uniform_f() * (float)z;
        const float k = (2.0f * sv) / ((float)h + sqrtf((float)hh - (float)c2 * sv));
        const float fi = floorf(k);
        i = fi > (float)top ? top : (uint32_t)fi;
        w = (double)(1.0f - (float)c * (float)i);
      } else {
        const double sv = rng.uniform() * z;
        const double k = (2.0 * sv) / (h + sqrt(hh - c2 * sv));
        const double fi = floor(k);
        i = fi > (double)top ? top : (uint32_t)fi;
        w = 1.0 - c * (double)i;
      }
      const double ei = mode_energy(S, C.T.lev, m, i);
      const double ua = (double)draw<MIX>(rng);
      const bool ok = (ei < ec) && lb_accept<MIX>(MIX ? (double)((float)ua * (float)w) : ua * w, ec - ei, den, q);
      if (ok) {
        lv[m * stride] = (uint16_t)i;
        et = ec - ei;
        break;
      }
      if (trials >= kMaxTrials) {
        capped = true;
        break;
      }
    }
    if (capped) break;
  }
  e_tr = et;
  return trials;
}

// isotropic unit vector (Marsaglia 1972)
template <bool MIX>
__device__ __forceinline__ V3<Real<MIX>> unit_vector(RngT<MIX> &rng) {
  using R = Real<MIX>;
  R x, y, s;
  for (;;) {
    x = R(2) * draw<MIX>(rng) - R(1);
    y = R(2) * draw<MIX>(rng) - R(1);
    s = x * x + y * y;
    if (s < R(1)) break;
  }
  const R f = R(2) * sqrt(R(1) - s);
  return V3<R>{x * f, y * f, R(1) - R(2) * s};
}

// centre-of-mass velocity of a pair (the mixed form weighs with the mass
// fractions in fp32)
template <bool MIX>
__device__ __forceinline__ V3<Real<MIX>> com(const PairTab &P, V3<Real<MIX>> a, V3<Real<MIX>> b) {
  if constexpr (MIX) {
    const float fa = (float)P.wb, fb = (float)P.wa;  // m_a / M, m_b / M
    return V3<float>{fa * a.x + fb * b.x, fa * a.y + fb * b.y, fa * a.z + fb * b.z};
  } else {
    return Vec3{(P.m_a * a.x + P.m_b * b.x) / P.msum, (P.m_a * a.y + P.m_b * b.y) / P.msum,
                (P.m_a * a.z + P.m_b * b.z) / P.msum};
  }
}

// two bodies about the centre-of-mass velocity with relative energy e
template <bool MIX>
__device__ __forceinline__ void split(const PairTab &P, V3<Real<MIX>> vcm, double e, RngT<MIX> &rng,
                                      V3<Real<MIX>> &va, V3<Real<MIX>> &vb) {
  using R = Real<MIX>;
  R g;
  if constexpr (MIX)
    g = sqrtf((float)(2.0 * e) / (float)P.mr);
  else
    g = sqrt((2.0 * e) / P.mr);
  const V3<R> n = unit_vector<MIX>(rng);
  const R ga = (R)P.wa * g, gb = (R)P.wb * g;
  va = V3<R>{vcm.x + ga * n.x, vcm.y + ga * n.y, vcm.z + ga * n.z};
  vb = V3<R>{vcm.x - gb * n.x, vcm.y - gb * n.y, vcm.z - gb * n.z};
}

// kinetic energy 1/2 m |v|^2 in fp64
template <typename R>
__device__ __forceinline__ double kinetic(double m, V3<R> v) {
  const double x = v.x, y = v.y, z = v.z;
  return 0.5 * m * ((x * x + y * y) + z * z);
}

__device__ __forceinline__ void zero_levels(uint16_t *lv, uint32_t stride, uint32_t mm) {
  for (uint32_t m = 0; m < mm; ++m) lv[m * stride] = 0;
}

// One colliding pair held on chip: velocities and species in registers,
// quantum numbers in per-lane LDS slots (mode m of side x at lv_x[m * ls]).
// Rotational Larsen-Borgnakke share: the fraction f of E_tr + E_rot that the
// rotor keeps has density proportional to f^(zeta/2 - 1) (1 - f)^q:
// zeta = 2 by inversion, f = 1 - (1 - u)^(1/(q+1)); zeta = 3 by rejection
// from the uniform against the density over its value at the mode
// f* = 1/(1 + 2q).
template <bool MIX>
__device__ double rot_fraction(uint32_t zeta, double q, RngT<MIX> &rng) {
  if constexpr (MIX) {
    const float qf = (float)q;
    if (zeta == 2) return (double)(1.0f - pow_f(1.0f - rng.uniform_f(), 1.0f / (qf + 1.0f)));
    const float fs = 1.0f / (1.0f + 2.0f * qf);
    for (;;) {
      const float f = rng.uniform_f(), u2 = rng.uniform_f();
      if (u2 < pow_f(f / fs, 0.5f) * pow_f((1.0f - f) / (1.0f - fs), qf)) return (double)f;
    }
  } else {
    if (zeta == 2) return 1.0 - dpow(1.0 - rng.uniform(), 1.0 / (q + 1.0));
    const double fs = 1.0 / (1.0 + 2.0 * q);
    for (;;) {
      const double f = rng.uniform(), u2 = rng.uniform();
      if (u2 < dpow(f / fs, 0.5) * dpow((1.0 - f) / (1.0 - fs), q)) return f;
    }
  }
}

template <bool MIX>
struct PairLocal {
  using R = Real<MIX>;
  V3<R> v0, v1;
  uint32_t sp0, sp1;
  bool dead0, dead1;
  uint16_t *lv0, *lv1, *lvn;
  uint32_t ls;
  bool born;  // a dissociation product (species nb_sp, velocity nb_v, levels lvn)
  uint32_t nb_sp;
  V3<R> nb_v;
  bool has_m, m_moved;  // third body for recombination
  uint32_t sp_m;
  V3<R> v_m;
  double n_cell;
  double et_out;     // translational energy handed to the scattering (relative motions)
  double fold_used;  // mixed form: energy owed to the cell that joined this pair
  int32_t rec_i;  // recombination table node of the cell temperature (-1: below, -2: above)
  double rec_f;
  double r0, r1, rn;  // rotational energies of p, q and the product (rotors only)
  uint32_t nb_from;   // side (0: p, 1: q) whose position the product takes
#ifdef HCAO_PHASE_CLOCKS
  uint64_t wclk[5], wclk_t;  // collision sub-phase clocks of instrumented builds
#endif
};

__device__ __forceinline__ double vib_local(const Tab &T, uint32_t sp, const uint16_t *lv, uint32_t ls) {
  const SpeciesTab &S = T.sp[sp];
  double e = 0.0;
  for (uint32_t m = 0; m < S.n_modes; ++m) e = e + mode_energy(S, T.lev, m, lv[m * ls]);
  return e;
}

struct Channel {
  int32_t rx, side, mode;
};

// Channel enumeration of one pair (dissociation channels of p then q, then
// exchange channels of p then q, registration order). Pass 0 draws the
// steric numbers, counts the open channels and sums their excess energy;
// pass 1 repeats the same arithmetic to find the channel that holds target.
struct ChannelScan {
  uint32_t nch;
  double total;
  Channel first, last, pick;
  bool found;
};

template <bool MIX, bool EX>
__device__ __forceinline__ void scan_channels(const Tab &T, uint32_t sp0, uint32_t sp1, double ev0, double ev1,
                                              const uint16_t *lv0, const uint16_t *lv1, uint32_t ls, double e_tr,
                                              double rot0, double rot1, RngT<MIX> &rng, uint64_t &steric_ok,
                                              int pass, double target, ChannelScan &S) {
  double cum = 0.0;
  uint32_t seen = 0, ex_i = 0;
  for (uint32_t kind = 0; kind < 2; ++kind) {
    for (uint32_t side = 0; side < 2; ++side) {
      const uint32_t A = side ? sp1 : sp0, B = side ? sp0 : sp1;
      const double evA = side ? ev1 : ev0, evB = side ? ev0 : ev1;
      const uint16_t *lA = side ? lv1 : lv0;
      const SpeciesTab &SA = T.sp[A];
      for (uint32_t r = 0; r < T.nr; ++r) {
        const ReactionTab &R = T.rx[r];
        if (kind == 0) {
          if (R.kind != HCAO_RX_DISSOCIATION || (uint32_t)R.a != A) continue;
          const uint32_t nst = SA.n_modes - SA.n_bend;
          for (uint32_t j = 0; j < nst; ++j) {
            if (!((R.mask >> j) & 1ull)) continue;
            const uint32_t m = SA.n_bend + j;
            // Eq. Ecoll-diss: E_tr (+ gamma E_rot,A) + E_vib,A - sum ZPE(A, B, C) + E_A,j(0)
            const double etg = EX ? e_tr + R.gamma_rot * (side ? rot1 : rot0) : e_tr;
            const double ecoll = ((etg + evA) - R.zsum) + T.lev[SA.lev_off[m]];
            const double eex = ecoll - SA.de[m];
            const double pool = (etg + evA) - R.dh;
            const double left = (pool - T.sp[R.c].zpe) - T.sp[R.d].zpe;
            if (eex > 0.0 && left > 0.0 && seen < (uint32_t)kMaxChannels) {
              const Channel ch{(int32_t)r, (int32_t)side, (int32_t)m};
              ++seen;
              if (pass == 0) {
                if (seen == 1) S.first = ch;
                S.last = ch;
                S.total = S.total + eex;
              } else if (!S.found) {
                cum = cum + eex;
                if (target < cum) {
                  S.pick = ch;
                  S.found = true;
                }
              }
            }
          }
        } else {
          if (R.kind != HCAO_RX_EXCHANGE || (uint32_t)R.a != A || (uint32_t)R.b != B) continue;
          bool st_ok;
          if (pass == 0) {
            st_ok = (double)draw<MIX>(rng) < R.steric;
            if (st_ok && ex_i < 64) steric_ok |= (1ull << ex_i);
          } else {
            st_ok = ex_i < 64 ? ((steric_ok >> ex_i) & 1ull) != 0 : false;
          }
          ++ex_i;
          // Eq. Ecoll-exch: E_tr (+ gamma E_rot,A) + sum_j alpha_j E_vib,A,j
          const double etg = EX ? e_tr + R.gamma_rot * (side ? rot1 : rot0) : e_tr;
          double ecoll = etg;
          for (uint32_t m = 0; m < SA.n_modes; ++m)
            ecoll = ecoll + R.alpha[m] * mode_energy(SA, T.lev, m, lA[m * ls]);
          const double eex = ecoll - R.ea;
          const double pool = ((etg + evA) + evB) - R.dh;
          const double left = (pool - T.sp[R.c].zpe) - T.sp[R.d].zpe;
          if (st_ok && eex > 0.0 && left > 0.0 && seen < (uint32_t)kMaxChannels) {
            const Channel ch{(int32_t)r, (int32_t)side, -1};
            ++seen;
            if (pass == 0) {
              if (seen == 1) S.first = ch;
              S.last = ch;
              S.total = S.total + eex;
            } else if (!S.found) {
              cum = cum + eex;
              if (target < cum) {
                S.pick = ch;
                S.found = true;
              }
            }
          }
        }
      }
    }
  }
  if (pass == 0) S.nch = seen;
}

// Reaction decision and application, or relaxation of both molecules, then
// scattering, for one accepted pair held in P. Returns the reaction id or -1.
// The outcome is decided first; the molecules to relax are then queued (at
// most two, in draw order) and run through one sampler loop, and the
// velocities come from at most two isotropic splits. g2 is |v_p - v_q|^2 in
// fp64. In the mixed form, fold is energy owed to the cell's particles by
// earlier rounding; it joins this pair's translational energy when the sum
// stays positive.
template <bool MIX, bool EX>
__device__ int collide(const Ctx &C, PairLocal<MIX> &P, double g2, RngT<MIX> &rng, const double *rec,
                       double fold) {
  using Rl = Real<MIX>;
  const Tab &T = C.T;
  const uint32_t mm = T.mm;
  const uint32_t ls = P.ls;
  const uint32_t sp0 = P.sp0, sp1 = P.sp1;
  const PairTab &PP = T.pair(sp0, sp1);
  double e_tr0 = PP.hm * g2;
  if constexpr (MIX) {
    P.fold_used = 0.0;
    if (fold != 0.0 && e_tr0 + fold > 0.0) {
      e_tr0 = e_tr0 + fold;
      P.fold_used = fold;
    }
  }
  const double ev0 = vib_local(T, sp0, P.lv0, ls), ev1 = vib_local(T, sp1, P.lv1, ls);
  P.born = false;
  P.m_moved = false;

  // outcome: 0 none, 1 dissociation, 2 exchange, 3 recombination
  int kind = 0, rx = -1;
  uint32_t side = 0;  // reacting side: A of dissociation/exchange, B of recombination
  V3<Rl> vbc{Rl(0), Rl(0), Rl(0)};
  double et = e_tr0;

  // --- recombination first: B + C (+M) -> A (+M) ---
  // (pairs that no reaction lists skip the decision; it would draw nothing)
  for (uint32_t r = 0; PP.react && r < T.nr && kind == 0; ++r) {
    const ReactionTab &R = T.rx[r];
    if (R.kind != HCAO_RX_RECOMBINATION) continue;
    uint32_t sb;
    if (P.sp0 == (uint32_t)R.a && P.sp1 == (uint32_t)R.b)
      sb = 0;
    else if (P.sp1 == (uint32_t)R.a && P.sp0 == (uint32_t)R.b)
      sb = 1;
    else
      continue;
    // 53 bits in both forms: the per-collision probability can be far below
    // the 2^-24 steps of the mixed form's single-word uniforms
    const double u = rng.uniform53();
    if (!P.has_m) {
      atomicAdd(&C.ctr[HCAO_CTR_SUPPRESSED], 1ull);
      continue;
    }
    const double *tab = rec + R.rec_off + (size_t)P.sp_m * T.rec_nt;
    double prob;
    if (P.rec_i == -1)
      prob = tab[0];
    else if (P.rec_i == -2)
      prob = tab[T.rec_nt - 1];
    else
      prob = tab[P.rec_i] + P.rec_f * (tab[P.rec_i + 1] - tab[P.rec_i]);
    prob = prob * P.n_cell;
    if (prob > 1.0) prob = 1.0;
    if (!(u < prob)) continue;
    const V3<Rl> vb = sb ? P.v1 : P.v0, vc = sb ? P.v0 : P.v1;
    const V3<Rl> c3 = com<MIX>(T.pair(R.a, R.b), vb, vc);
    const double gx = (double)c3.x - (double)P.v_m.x, gy = (double)c3.y - (double)P.v_m.y,
                 gz = (double)c3.z - (double)P.v_m.z;
    const double e_am = T.pair(R.c, P.sp_m).hm * ((gx * gx + gy * gy) + gz * gz);
    double pool = (((e_am + e_tr0) + (sb ? ev1 : ev0)) + (sb ? ev0 : ev1)) - R.dh;
    double rsum = 0.0;
    if constexpr (EX) {
      // B's and C's rotation: kept by A's rotor, else pooled
      rsum = (sb ? P.r1 : P.r0) + (sb ? P.r0 : P.r1);
      if (T.sp[R.c].zeta_rot == 0) pool = pool + rsum;
    }
    const double e_left = pool - T.sp[R.c].zpe;
    if (!(e_left > 0.0)) {
      atomicAdd(&C.ctr[HCAO_CTR_SUPPRESSED], 1ull);
      continue;
    }
    kind = 3;
    rx = (int)r;
    side = sb;
    vbc = c3;
    et = e_left;
    if constexpr (EX) {
      const double ra = T.sp[R.c].zeta_rot > 0 ? rsum : 0.0;
      P.r0 = sb ? 0.0 : ra;
      P.r1 = sb ? ra : 0.0;
    }
  }

  // --- dissociation and exchange channels, competition by excess energy ---
  // A pair none of whose channels can open skips the scan (its steric draws
  // are passed over): the bounds are tested with a margin far above the
  // rounding of the scan's own sums, so only pairs that certainly stay shut
  // skip it and the result is the scan's.
  bool may_open = false;
  if (kind == 0 && PP.react) {
    const PairBound &B = PP.bound;
    for (uint32_t sd = 0; sd < 2; ++sd) {
      const double ev = sd ? ev1 : ev0;
      const double et = EX ? e_tr0 + (sd ? P.r1 : P.r0) : e_tr0;
      const double scale = 1e-9 * ((fabs(et) + ev) + fabs(B.dis_c[sd] < 0.0 ? 0.0 : B.dis_c[sd]) + 1e-30);
      if ((et + ev) + B.dis_c[sd] > -scale - 1e-9 * fabs(B.dis_c[sd])) may_open = true;
      if (B.ex_a[sd] >= 0.0 && (et + B.ex_a[sd] * ev) - B.ex_e[sd] > -scale - 1e-9 * B.ex_e[sd]) may_open = true;
    }
    if (!may_open) rng.skip(B.n_steric);
  }
  if (kind == 0 && PP.react && may_open) {
    uint64_t steric_ok = 0;
    ChannelScan S;
    S.nch = 0;
    S.total = 0.0;
    S.found = false;
    S.first = S.last = S.pick = Channel{-1, 0, 0};
    scan_channels<MIX, EX>(T, sp0, sp1, ev0, ev1, P.lv0, P.lv1, ls, e_tr0, P.r0, P.r1, rng, steric_ok, 0, 0.0, S);
    if (S.nch > 0) {
      Channel pick = S.first;
      if (S.nch > 1) {
        const double target = (double)draw<MIX>(rng) * S.total;
        scan_channels<MIX, EX>(T, sp0, sp1, ev0, ev1, P.lv0, P.lv1, ls, e_tr0, P.r0, P.r1, rng, steric_ok, 1, target,
                               S);
        pick = S.found ? S.pick : S.last;
      }
      const ReactionTab &R = T.rx[pick.rx];
      rx = pick.rx;
      side = (uint32_t)pick.side;
      const double eva = side ? ev1 : ev0, evb = side ? ev0 : ev1;
      const double ra = side ? P.r1 : P.r0, rb = side ? P.r0 : P.r1;
      const double grot = EX ? R.gamma_rot * ra : 0.0;
      const double etg = EX ? e_tr0 + grot : e_tr0;
      if (R.kind == HCAO_RX_DISSOCIATION) {
        kind = 1;
        et = (((etg + eva) - R.dh) - T.sp[R.c].zpe) - T.sp[R.d].zpe;
        if constexpr (EX) {
          // the uncoupled rotation stays with B's rotor, else is pooled
          double keep = ra - grot;
          if (T.sp[R.c].zeta_rot == 0) {
            et = et + keep;
            keep = 0.0;
          }
          if (side)
            P.r1 = keep;
          else
            P.r0 = keep;
          P.rn = 0.0;
        }
      } else {
        kind = 2;
        et = ((((etg + eva) + evb) - R.dh) - T.sp[R.c].zpe) - T.sp[R.d].zpe;
        if constexpr (EX) {
          // A's uncoupled rotation goes to C's rotor, B's to D's; else pooled
          double keep_c = ra - grot, keep_d = rb;
          if (T.sp[R.c].zeta_rot == 0) {
            et = et + keep_c;
            keep_c = 0.0;
          }
          if (T.sp[R.d].zeta_rot == 0) {
            et = et + keep_d;
            keep_d = 0.0;
          }
          P.r0 = side ? keep_d : keep_c;
          P.r1 = side ? keep_c : keep_d;
        }
      }
    }
  }

  HCAO_WAVE_MARK(P.wclk, kPhaseCollideDecide);
  // --- queue the relaxations (at most two, in draw order) ---
  uint16_t *lvj0 = nullptr, *lvj1 = nullptr;
  uint32_t spj0 = 0, spj1 = 0;
  double qj0 = 0.0, qj1 = 0.0;
  uint32_t bj0 = 0, bj1 = 0;  // beta table offsets (exact sampler)
  bool pv = false;
  uint32_t njob = 0;
  const ReactionTab &RX = T.rx[rx < 0 ? 0 : rx];
  uint16_t *la = side ? P.lv1 : P.lv0;
  uint16_t *lb = side ? P.lv0 : P.lv1;
  uint32_t ja_sp = 0, jb_sp = 0;  // candidate jobs a and b
  uint16_t *ja_lv = nullptr, *jb_lv = nullptr;
  double ja_q = 0.0, jb_q = 0.0;
  uint32_t ja_b = 0, jb_b = 0;
  if (kind == 0) {
    pv = true;
    ja_sp = sp0;
    ja_lv = P.lv0;
    ja_q = PP.q;
    ja_b = PP.beta_off;
    jb_sp = sp1;
    jb_lv = P.lv1;
    jb_q = PP.q;
    jb_b = T.pair(sp1, sp0).beta_off;
  } else if (kind == 1) {
    // A + M -> B + C + M: B takes A's slot, C is new, both from the ground state
    const uint32_t spM = side ? sp0 : sp1;
    zero_levels(la, ls, mm);
    zero_levels(P.lvn, ls, mm);
    ja_sp = (uint32_t)RX.c;
    ja_lv = la;
    ja_q = T.pair(RX.c, spM).q;
    ja_b = T.pair(RX.c, spM).beta_off;
    jb_sp = (uint32_t)RX.d;
    jb_lv = P.lvn;
    jb_q = T.pair(RX.d, spM).q;
    jb_b = T.pair(RX.d, spM).beta_off;
  } else if (kind == 2) {
    // A + B -> C + D: C takes A's slot, D takes B's
    zero_levels(la, ls, mm);
    zero_levels(lb, ls, mm);
    const double qcd = T.pair(RX.c, RX.d).q;
    ja_sp = (uint32_t)RX.c;
    ja_lv = la;
    ja_q = qcd;
    ja_b = T.pair(RX.c, RX.d).beta_off;
    jb_sp = (uint32_t)RX.d;
    jb_lv = lb;
    jb_q = qcd;
    jb_b = T.pair(RX.d, RX.c).beta_off;
  } else {
    // B + C (+M) -> A (+M): A takes B's slot
    zero_levels(la, ls, mm);
    ja_sp = (uint32_t)RX.c;
    ja_lv = la;
    ja_q = T.pair(RX.c, P.sp_m).q;
    ja_b = T.pair(RX.c, P.sp_m).beta_off;
  }
  if (T.sp[ja_sp].n_modes > 0) {
    lvj0 = ja_lv;
    spj0 = ja_sp;
    qj0 = ja_q;
    bj0 = ja_b;
    ++njob;
  }
  if (kind != 3 && T.sp[jb_sp].n_modes > 0) {
    if (njob == 0) {
      lvj0 = jb_lv;
      spj0 = jb_sp;
      qj0 = jb_q;
      bj0 = jb_b;
    } else {
      lvj1 = jb_lv;
      spj1 = jb_sp;
      qj1 = jb_q;
      bj1 = jb_b;
    }
    ++njob;
  }
  uint64_t tr = 0;
  uint32_t nrel = 0, ncap = 0;
  for (uint32_t j = 0; j < njob; ++j) {
    const SpeciesTab &S = T.sp[j ? spj1 : spj0];
    if (pv) {
      const double u = (double)draw<MIX>(rng);
      if (!(u < S.p_vib)) continue;
      ++nrel;
    }
    bool capped = false;
    const uint32_t bo = j ? bj1 : bj0;
    tr += relax<MIX, EX>(C, S, j ? lvj1 : lvj0, ls, et, j ? qj1 : qj0, C.T.beta + (bo == 0xFFFFFFFFu ? 0u : bo), rng, capped);
    ncap += capped ? 1u : 0u;
  }
  if (tr) atomicAdd(&C.ctr[HCAO_CTR_TRIALS], (unsigned long long)tr);
  if (nrel) atomicAdd(&C.ctr[HCAO_CTR_RELAX], (unsigned long long)nrel);
  if (ncap) atomicAdd(&C.ctr[HCAO_CTR_CAPPED], (unsigned long long)ncap);

  HCAO_WAVE_MARK(P.wclk, kPhaseCollideRelax);
  // --- rotational relaxation of each rotor in turn (non-reactive collisions) ---
  if constexpr (EX) {
    if (kind == 0) {
      for (uint32_t x = 0; x < 2; ++x) {
        const SpeciesTab &S = T.sp[x ? sp1 : sp0];
        if (S.zeta_rot == 0) continue;
        const double u = (double)draw<MIX>(rng);
        if (!(u < S.p_rot)) continue;
        const double ec = et + (x ? P.r1 : P.r0);
        const double er = rot_fraction<MIX>(S.zeta_rot, PP.q, rng) * ec;
        if (x)
          P.r1 = er;
        else
          P.r0 = er;
        et = ec - er;
      }
    }
  }

  // --- scattering ---
  const V3<Rl> va0 = side ? P.v1 : P.v0, vb0 = side ? P.v0 : P.v1;
  double e1 = et, e2 = 0.0;
  if (kind == 1) {
    // share of the translational energy in the B-C motion: density
    // proportional to sqrt(beta (1 - beta)), by rejection
    Rl beta;
    for (;;) {
      const Rl u1 = draw<MIX>(rng), u2 = draw<MIX>(rng);
      if (u2 * Rl(0.5) < sqrt(u1 * (Rl(1) - u1))) {
        beta = u1;
        break;
      }
    }
    e2 = (double)beta * et;
    e1 = et - e2;
  }
  const uint32_t spA = side ? sp1 : sp0, spB = side ? sp0 : sp1;
  const PairTab *t1;
  V3<Rl> cm;
  if (kind == 0) {
    t1 = &PP;
    cm = com<MIX>(PP, P.v0, P.v1);
  } else if (kind == 1) {
    t1 = &T.pair(spA, spB);
    cm = com<MIX>(*t1, va0, vb0);
  } else if (kind == 2) {
    t1 = &T.pair(RX.c, RX.d);
    cm = com<MIX>(T.pair(spA, spB), va0, vb0);
  } else {
    t1 = &T.pair(RX.c, P.sp_m);
    cm = com<MIX>(*t1, vbc, P.v_m);
  }
  V3<Rl> x1, y1;
  P.et_out = et;
  split<MIX>(*t1, cm, e1, rng, x1, y1);
  if (kind == 0) {
    P.v0 = x1;
    P.v1 = y1;
    return -1;
  }
  if (kind == 1) {
    V3<Rl> x2, y2;
    split<MIX>(T.pair(RX.c, RX.d), x1, e2, rng, x2, y2);
    x1 = x2;
    P.born = true;
    P.nb_sp = (uint32_t)RX.d;
    P.nb_v = y2;
    P.nb_from = side;
    atomicAdd(&C.ctr[HCAO_CTR_BIRTHS], 1ull);
  }
  if (kind == 3) {
    P.v_m = y1;
    P.m_moved = true;
    atomicAdd(&C.ctr[HCAO_CTR_DEATHS], 1ull);
  }
  const uint32_t new_a = (uint32_t)RX.c;
  const uint32_t new_b = kind == 2 ? (uint32_t)RX.d : spB;
  if (side) {
    P.v1 = x1;
    P.sp1 = new_a;
    if (kind == 3)
      P.dead0 = true;
    else {
      P.v0 = y1;
      P.sp0 = new_b;
    }
  } else {
    P.v0 = x1;
    P.sp0 = new_a;
    if (kind == 3)
      P.dead1 = true;
    else {
      P.v1 = y1;
      P.sp1 = new_b;
    }
  }
  atomicAdd(&C.ctr[HCAO_CTR_REACTION0 + rx], 1ull);
  return rx;
}

// Sums of m, m v_x, m v_y, m v_z and m |v|^2 over a cell's particles by one
// wave: lane t sums particles t, t + 64, t + 128, ... in slot order (loads
// of four blocks issued together), then a halving tree (lane t takes lane
// t + s for s = 32, ..., 1) combines the 64 partial sums; lane 0 returns
// them (every lane of the wave takes part). The running sums of the cell
// temperature start from these.
template <bool MIX>
__device__ void cell_sums(const State &st, const SpeciesTab *spt, uint64_t base, uint32_t n, uint32_t lane,
                          double out[5]) {
  constexpr int U = 4;
  double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0, x4 = 0.0;
  for (uint32_t b0 = 0; b0 < n; b0 += 64 * U) {
    double m[U], vx[U], vy[U], vz[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = b0 + 64 * u + lane;
      m[u] = 0.0;
      vx[u] = vy[u] = vz[u] = 0.0;
      if (i < n) {
        const uint64_t g = base + i;
        m[u] = spt[st.sp[g]].mass;
        const V3<Real<MIX>> v = ldv<MIX>(st, g);
        vx[u] = v.x;
        vy[u] = v.y;
        vz[u] = v.z;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (b0 + 64 * u + lane < n) {
        x0 = x0 + m[u];
        x1 = x1 + m[u] * vx[u];
        x2 = x2 + m[u] * vy[u];
        x3 = x3 + m[u] * vz[u];
        x4 = x4 + m[u] * ((vx[u] * vx[u] + vy[u] * vy[u]) + vz[u] * vz[u]);
      }
    }
  }
  double x[5] = {x0, x1, x2, x3, x4};
  tree_sum(x);
  for (int q = 0; q < 5; ++q) out[q] = x[q];
}

// adds one particle's terms m, m v, m |v|^2 to acc (in that order)
template <typename R>
__device__ __forceinline__ void add_terms(double acc[5], double m, V3<R> v) {
  const double x = v.x, y = v.y, z = v.z;
  acc[0] = acc[0] + m;
  acc[1] = acc[1] + m * x;
  acc[2] = acc[2] + m * y;
  acc[3] = acc[3] + m * z;
  acc[4] = acc[4] + m * ((x * x + y * y) + z * z);
}

// ---------------------------------------------------------------------------
// the collision step: one workgroup per group of consecutive cells
// ---------------------------------------------------------------------------
// Per-cell state kept in LDS across the steps of a launch (base .. weight)
// and per-step quantities (ncand .. perm).
struct CellHdr {
  uint64_t base;
  uint32_t cell, n, cap, ncand, cstart, pad;
  double sgmax, rem, volume, weight;
  double rem_new, n_cell, rec_f;
  double defect;  // mixed form: energy the cell's particles lack
  double tsum[5];  // recombination: running sums m, m v, m |v|^2 of the cell's particles
  int32_t rec_i, pad2;
  unsigned long long sgbits, excess;
  Perm perm;
};

// the cell of flattened candidate j: the last cell whose range starts at or before j
__device__ __forceinline__ uint32_t group_cell(const CellHdr *hdr, uint32_t ncell, uint32_t j) {
  uint32_t lo = 0, hi = ncell;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (hdr[mid].cstart <= j)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Phase 0 stages the tables in LDS and computes each cell's NTC candidate
// count and permutation keys (and, with recombination, the cell
// temperature). Phase A tests every candidate pair of the group (lane per
// candidate) and appends the accepted ones to a work list. Phase B gives
// every lane one accepted pair: the pair's state is gathered once into
// registers and per-lane LDS, the reaction / relaxation / scattering runs
// on chip, and the result is written back. Phase C removes recombined
// particles, places the products of each cell in pair order and writes the
// per-cell state. Pairs are disjoint and every draw is keyed by (cell,
// pair), so the order in which lanes take work does not change the result.
//
// The mixed form (MIX) keeps fp32 velocities, tests VHS acceptance and
// samples levels in fp32, and keeps energies, thresholds and accumulators in
// fp64. Each pair records the fp64 energy its fp32 velocities lost or gained
// (the audit of its particles before and after); the cell's sum, reduced in
// pair order, is owed to the cell and joins the translational energy of the
// cell's pair 0 in the next step in which that pair collides.
template <int BLOCK, bool MIX, int EX>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3))) void k_step(StepArgs A) {
  using R = Real<MIX>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ uint32_t s_nwork, s_total, s_next;
  __shared__ uint32_t s_bin[256];
  const uint32_t tid = threadIdx.x;
  // the wave index is the same on every lane of a wave: held in a scalar
  // register, so that per-wave loops (one wave per cell) and what they
  // address stay scalar
  const uint32_t lane = tid & 63u, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const unsigned long long lt = lane ? ((1ull << lane) - 1ull) : 0ull;
  const Tables *GT = A.tab;
  const uint32_t ns = GT->n_species, nr = GT->n_reactions, mm = GT->max_modes, nl = GT->n_levels;
  const uint32_t nctr = 8 + nr;
  const uint32_t c0 = A.grp[2 * blockIdx.x], c1 = A.grp[2 * blockIdx.x + 1];
  const uint32_t ncell = c1 - c0;
  const uint64_t wbase = A.grp_work[2 * blockIdx.x];
#ifdef HCAO_PHASE_CLOCKS
  uint64_t clk_acc[kPhases] = {};
  uint64_t clk_t = clock64();
#endif

  // ---- LDS carve-up ----
  unsigned char *q = smem;
  SpeciesTab *l_sp = reinterpret_cast<SpeciesTab *>(q);
  q += sizeof(SpeciesTab) * ns;
  PairTab *l_pr = reinterpret_cast<PairTab *>(q);
  q += sizeof(PairTab) * ns * ns;
  ReactionTab *l_rx = reinterpret_cast<ReactionTab *>(q);
  q += sizeof(ReactionTab) * nr;
  double *l_lev = reinterpret_cast<double *>(q);
  q += sizeof(double) * nl;
  CellHdr *hdr = reinterpret_cast<CellHdr *>(q);
  q += sizeof(CellHdr) * ncell;
  unsigned long long *l_ctr = reinterpret_cast<unsigned long long *>(q);
  q += sizeof(unsigned long long) * nctr * ncell * 2;  // per-step counters, then totals
  uint16_t *scr = reinterpret_cast<uint16_t *>(q);  // [2 mm][BLOCK] sampler scratch
  uint16_t *plv = scr + (size_t)2 * mm * BLOCK;      // [3 mm][BLOCK] pair levels

  unsigned long long *l_tot = l_ctr + (size_t)nctr * ncell;  // counters summed over the launch's steps

  // ---- once per launch: tables and the persistent cell state ----
  {
    const uint64_t *src = reinterpret_cast<const uint64_t *>(GT->sp);
    uint64_t *dst = reinterpret_cast<uint64_t *>(l_sp);
    for (uint32_t i = tid; i < ns * sizeof(SpeciesTab) / 8; i += BLOCK) dst[i] = src[i];
    for (uint32_t i = tid; i < ns * ns; i += BLOCK) l_pr[i] = GT->pr[i / ns][i % ns];
    src = reinterpret_cast<const uint64_t *>(GT->rx);
    dst = reinterpret_cast<uint64_t *>(l_rx);
    for (uint32_t i = tid; i < nr * sizeof(ReactionTab) / 8; i += BLOCK) dst[i] = src[i];
    for (uint32_t i = tid; i < nl; i += BLOCK) l_lev[i] = A.lev[i];
    for (uint32_t i = tid; i < nctr * ncell; i += BLOCK) l_tot[i] = 0ull;
  }
  for (uint32_t g = tid; g < ncell; g += BLOCK) {
    CellHdr &H = hdr[g];
    const uint32_t c = c0 + g;
    H.base = A.cells.off[c];
    H.cell = c;
    H.n = A.cells.cnt[c];
    H.cap = A.cells.cap[c];
    H.sgmax = A.cells.sgmax[c];
    H.rem = A.cells.rem[c];
    H.volume = A.cells.volume[c];
    H.weight = A.cells.weight[c];
    H.defect = MIX ? A.cells.defect[c] : 0.0;
    if (A.cells.tsum)
      for (int q = 0; q < 5; ++q) H.tsum[q] = A.cells.tsum[(size_t)q * A.cells.n_cells + c];
  }
  if constexpr (EX >= 1) {
    // spatial mode: the particles were re-binned since the last step, so the
    // running sums start afresh from them (one wave per cell; masses from
    // the species table in LDS)
    if (A.cells.tsum && A.st.px) {
      __syncthreads();
      for (uint32_t g = wave; g < ncell; g += BLOCK / 64) {
        double sums[5];
        cell_sums<MIX>(A.st, l_sp, hdr[g].base, hdr[g].n, lane, sums);
        if (lane == 0)
          for (int q = 0; q < 5; ++q) hdr[g].tsum[q] = sums[q];
      }
    }
  }
  const Tab T{l_sp, l_pr, l_rx, l_lev, A.beta, ns, nr, mm, GT->rec_nt};
  const uint32_t wcap = (uint32_t)(A.grp_work[2 * blockIdx.x + 1] - wbase);
  uint32_t *work_in = A.work + (size_t)kWorkWords * wbase;  // accepted pairs as found
  uint32_t *work = work_in + (size_t)kWorkFound * wcap;       // their indices sorted by key
  uint8_t *bflag = A.bflag + wbase;
  double *wdef = MIX ? A.wdef + wbase : nullptr;
  __syncthreads();
  HCAO_PHASE_MARK(kPhaseLoad);

  const uint32_t step0 = A.step_dev ? *A.step_dev + A.step : A.step;
  for (uint32_t si = 0; si < A.n_steps; ++si) {
  const uint32_t step = step0 + si;

  // ---- phase 0: candidate counts and permutation keys of the step ----
  for (uint32_t i = tid; i < nctr * ncell; i += BLOCK) l_ctr[i] = 0ull;
  for (uint32_t i = tid; i < 256; i += BLOCK) s_bin[i] = 0;  // the work-list sort's bins, counted in phase A
  for (uint32_t g = tid; g < ncell; g += BLOCK) {
    CellHdr &H = hdr[g];
    const uint32_t n = H.n;
    // NTC candidate count: floor(1/2 N (N-1) F_N (sigma g)_max dt / V + remainder)
    const double x = 0.5 * (double)n * (double)(n - (n > 0 ? 1u : 0u)) * H.weight * H.sgmax * A.dt / H.volume + H.rem;
    const double fl = floor(x);
    uint64_t ncand = (uint64_t)fl;
    uint64_t excess = 0;
    if (ncand > n / 2) {
      excess = ncand - n / 2;
      ncand = n / 2;
    }
    H.ncand = (uint32_t)ncand;
    H.rem_new = x - fl;
    H.n_cell = (double)n * H.weight / H.volume;
    H.rec_i = -1;
    H.rec_f = 0.0;
    H.sgbits = 0ull;
    H.excess = excess;
    if (ncand > 0) make_perm(H.perm, n, A.seed, H.cell, step);
    if (GT->has_recomb && n >= 2) {
      // cell temperature from the running sums and its recombination-table coordinate
      const double p2 = (H.tsum[1] * H.tsum[1] + H.tsum[2] * H.tsum[2]) + H.tsum[3] * H.tsum[3];
      const double t = (H.tsum[4] - p2 / H.tsum[0]) / (3.0 * kBoltz * (double)n);
      if (t > 0.0) {
        const double u = (dlog(t) - GT->rec_l0) * GT->rec_inv_step;
        if (!(u > 0.0)) {
          H.rec_i = -1;
        } else if (!(u < (double)(GT->rec_nt - 1))) {
          H.rec_i = -2;
        } else {
          const double fi = floor(u);
          H.rec_i = (int32_t)fi;
          H.rec_f = u - fi;
        }
      }
    }
  }
  __syncthreads();
  HCAO_PHASE_MARK(kPhaseNtc);
  if (tid == 0) {
    uint32_t acc = 0;
    for (uint32_t g = 0; g < ncell; ++g) {
      hdr[g].cstart = acc;
      acc += hdr[g].ncand;
    }
    s_total = acc;
    s_nwork = 0;
    s_next = 0;
  }
  __syncthreads();
  HCAO_PHASE_MARK(kPhaseTemperature);
  const uint32_t total = s_total;

  // ---- phase A: candidate pairs, VHS acceptance ----
  // Accepted pairs are appended to a work list (one LDS atomic per wave)
  // with a key that orders them by the sampler work they carry: the mode
  // counts of p and of q. A counting sort by that key (largest first) then
  // gives each wave of phase B pairs whose relaxations have the same shape.
  for (uint32_t j0 = 0; j0 < total; j0 += BLOCK) {
    const uint32_t j = j0 + tid;
    bool acc = false;
    uint32_t pj = 0, qj = 0, key = 0, rw1 = 0, rw2 = 0, rw3 = 0, g_acc = 0;
    if (j < total) {
      const uint32_t g = group_cell(hdr, ncell, j);
      g_acc = g;
      const CellHdr &H = hdr[g];
      const uint32_t k = j - H.cstart;
      PermReg perm;
      perm.load(H.perm);
      const uint32_t p = perm(2 * k), qq = perm(2 * k + 1);
      pj = p;
      qj = qq;
      const uint64_t gp = HCAO_IDX(H.base + p, A.st.n_slots, A.err), gq = HCAO_IDX(H.base + qq, A.st.n_slots, A.err);
      const V3<R> vp = ldv<MIX>(A.st, gp), vq = ldv<MIX>(A.st, gq);
      const R dx = vp.x - vq.x, dy = vp.y - vq.y, dz = vp.z - vq.z;
      const R g2 = (dx * dx + dy * dy) + dz * dz;
      const uint32_t a = A.st.sp[gp], b = A.st.sp[gq];
      const PairTab &PP = T.pair(a, b);
      RngT<MIX> rng;
      rng.open(A.seed, k, H.cell, step);
      const R ua = draw<MIX>(rng);
      // the rest of the pair stream's first block, handed to the collision pass
      rw1 = rng.w1;
      rw2 = rng.w2;
      rw3 = rng.w3;
      bflag[HCAO_IDX(j, wcap, A.err)] = 0;
      // VHS acceptance ua < sigma g / (sigma g)_max with sigma g = C (g^2)^(1-w).
      if constexpr (MIX) {
        const float sg = (g2 > 0.0f) ? (float)PP.csg * pow_f(g2, (float)PP.esg) : 0.0f;
        const unsigned long long sb = (unsigned long long)__double_as_longlong((double)sg);
        if ((double)sg > H.sgmax && sb > hdr[g].sgbits) atomicMax(&hdr[g].sgbits, sb);
        acc = ua < sg / (float)H.sgmax;
      } else {
        // The exact sigma g is needed for the decision only near the filter
        // band, and for the (sigma g)_max update only when it may exceed the
        // cell's current value (the update keeps the larger of the two).
        const double est = (g2 > 0.0) ? PP.csg * pow_estimate(g2, PP.esg) : 0.0;
        const double ratio = est / H.sgmax;
        const bool need_max = est >= H.sgmax * (1.0 - 2.0 * kFilter);
        if (ua < ratio * (1.0 - kFilter) && !need_max) {
          acc = true;
        } else if (ua > ratio * (1.0 + kFilter) && !need_max) {
          acc = false;
        } else {
          const double sg = (g2 > 0.0) ? PP.csg * dpow(g2, PP.esg) : 0.0;
          const unsigned long long sb = (unsigned long long)__double_as_longlong(sg);
          if (sb > hdr[g].sgbits) atomicMax(&hdr[g].sgbits, sb);
          acc = ua < sg / H.sgmax;
        }
      }
      const uint32_t na = T.sp[a].n_modes < 15 ? T.sp[a].n_modes : 15;
      const uint32_t nb = T.sp[b].n_modes < 15 ? T.sp[b].n_modes : 15;
      key = 255u - (na * 16u + nb);
      if (acc) atomicAdd(&s_bin[key], 1u);
    }
    const unsigned long long ma = __ballot(acc);
    uint32_t wb = 0;
    if (lane == 0 && ma) wb = atomicAdd(&s_nwork, (uint32_t)__popcll(ma));
    wb = __builtin_amdgcn_readfirstlane(wb);  // every lane is active here: lane 0's value
    if (acc) {
      uint32_t *w = work_in + (size_t)kWorkFound * HCAO_IDX(wb + (uint32_t)__popcll(ma & lt), wcap, A.err);
      w[0] = j;
      w[1] = pj;
      w[2] = qj;
      w[3] = key | (g_acc << 8);
      w[4] = rw1;
      w[5] = rw2;
      w[6] = rw3;
    }
  }
  __syncthreads();
  HCAO_PHASE_MARK(kPhaseAccept);

  // ---- counting sort of the work list by key ----
  // (the bins were counted as phase A appended the pairs)
  const uint32_t nwork = s_nwork;
  if (tid < 64) {
    // exclusive scan of the 256 bins, four per lane
    const uint32_t b0 = s_bin[4 * lane], b1 = s_bin[4 * lane + 1], b2 = s_bin[4 * lane + 2], b3 = s_bin[4 * lane + 3];
    const uint32_t sum = ((b0 + b1) + b2) + b3;
    uint32_t inc = sum;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = __shfl_up(inc, d);
      if ((int)lane >= d) inc += o;
    }
    const uint32_t ex = inc - sum;
    s_bin[4 * lane] = ex;
    s_bin[4 * lane + 1] = ex + b0;
    s_bin[4 * lane + 2] = ex + b0 + b1;
    s_bin[4 * lane + 3] = ex + b0 + b1 + b2;
  }
  __syncthreads();
  for (uint32_t i = tid; i < nwork; i += BLOCK) {
    const uint32_t *f = work_in + (size_t)kWorkFound * i;
    work[HCAO_IDX(atomicAdd(&s_bin[f[3] & 0xFFu], 1u), wcap, A.err)] = i;  // the entry itself stays where it was found
  }
  __syncthreads();
  HCAO_PHASE_MARK(kPhaseSort);

  // ---- phase B: one accepted pair per lane ----
  // Waves take 64 consecutive pairs of the sorted list at a time from a
  // shared counter, so that a wave that drew light pairs takes the next
  // block instead of waiting at the barrier for one that drew heavy ones.
  for (;;) {
    uint32_t c0 = 0;
    if (lane == 0) c0 = atomicAdd(&s_next, 64u);
    c0 = __builtin_amdgcn_readfirstlane(c0);  // every lane is active here: lane 0's value
    if (c0 >= nwork) break;
    const uint32_t i = c0 + lane;
    if (i < nwork) {
#ifdef HCAO_PHASE_CLOCKS
    PairLocal<MIX> P;
    for (int x = 0; x < 5; ++x) P.wclk[x] = 0;
    P.wclk_t = clock64();
    const bool lead = lane == (uint32_t)(__ffsll((long long)__ballot(1)) - 1);
#else
    PairLocal<MIX> P;
#endif
    const uint32_t *wi = work_in + (size_t)kWorkFound * work[i];
    const uint32_t j = wi[0], p = wi[1], qq = wi[2];
    const uint32_t g = wi[3] >> 8;
    const CellHdr &H = hdr[g];
    const uint32_t k = j - H.cstart;
    const uint64_t gp = HCAO_IDX(H.base + p, A.st.n_slots, A.err), gq = HCAO_IDX(H.base + qq, A.st.n_slots, A.err);
    P.v0 = ldv<MIX>(A.st, gp);
    P.v1 = ldv<MIX>(A.st, gq);
    P.sp0 = A.st.sp[gp];
    P.sp1 = A.st.sp[gq];
    P.dead0 = P.dead1 = false;
    P.ls = BLOCK;
    P.lv0 = plv + tid;
    P.lv1 = plv + (size_t)mm * BLOCK + tid;
    P.lvn = plv + (size_t)2 * mm * BLOCK + tid;
    // quantum numbers of the species' own modes (the others are 0 in the state
    // and nothing reads them here)
    const uint32_t nm0 = T.sp[P.sp0].n_modes, nm1 = T.sp[P.sp1].n_modes;
    load_levels(A.st, gp, nm0, P.lv0, BLOCK);
    load_levels(A.st, gq, nm1, P.lv1, BLOCK);
    P.r0 = P.r1 = P.rn = 0.0;
    if constexpr (EX >= 2) {
      if (A.st.rot) {
        P.r0 = A.st.rot[gp];
        P.r1 = A.st.rot[gq];
      }
    }
    P.has_m = false;
    uint64_t gm = 0;
    if ((T.pair(P.sp0, P.sp1).react & kReactRecomb) && 2 * H.ncand + k < H.n) {
      // third body of pair k: the particle at permutation index 2 N_cand + k
      PermReg perm;
      perm.load(H.perm);
      gm = HCAO_IDX(H.base + perm(2 * H.ncand + k), A.st.n_slots, A.err);
      P.has_m = true;
      P.sp_m = A.st.sp[gm];
      P.v_m = ldv<MIX>(A.st, gm);
    }
    P.n_cell = H.n_cell;
    P.rec_i = H.rec_i;
    P.rec_f = H.rec_f;
    // |v_p - v_q|^2 in fp64 (exact differences of fp32 velocities in the mixed form)
    const double dx = (double)P.v0.x - (double)P.v1.x, dy = (double)P.v0.y - (double)P.v1.y,
                 dz = (double)P.v0.z - (double)P.v1.z;
    const double g2 = (dx * dx + dy * dy) + dz * dz;
    RngT<MIX> rng;
    rng.open(A.seed, k, H.cell, step);
    // resume after the acceptance draw of phase A: its block's other words
    rng.block = 1;
    rng.w1 = wi[4];
    rng.w2 = wi[5];
    rng.w3 = wi[6];
    rng.used = MIX ? 1u : 2u;
    unsigned long long *ctr = l_ctr + (size_t)g * nctr;
    atomicAdd(&ctr[HCAO_CTR_COLLISIONS], 1ull);
    Ctx C{T, ctr, scr, tid, BLOCK};
    // mixed form: momentum of the pair (and of the third body) before the
    // collision, in fp64 from the stored fp32 velocities
    double mt = 0.0, px = 0.0, py = 0.0, pz = 0.0, mm3 = 0.0;
    if constexpr (MIX) {
      const double m0 = T.sp[P.sp0].mass, m1 = T.sp[P.sp1].mass;
      mt = m0 + m1;
      px = m0 * (double)P.v0.x + m1 * (double)P.v1.x;
      py = m0 * (double)P.v0.y + m1 * (double)P.v1.y;
      pz = m0 * (double)P.v0.z + m1 * (double)P.v1.z;
      if (P.has_m) mm3 = T.sp[P.sp_m].mass;  // joins the sums only if the third body takes part
    }
    const Vec3 vm_in = P.has_m ? Vec3{(double)P.v_m.x, (double)P.v_m.y, (double)P.v_m.z} : Vec3{0.0, 0.0, 0.0};
    // recombination: the pair's terms of its cell's running sums before the collision
    const uint32_t sp_in0 = P.sp0, sp_in1 = P.sp1;
    const V3<R> v_in0 = P.v0, v_in1 = P.v1;
    HCAO_WAVE_MARK(P.wclk, kPhaseCollideGather);
    collide<MIX, (EX >= 2)>(C, P, g2, rng, A.rec, (MIX && k == 0) ? H.defect : 0.0);
    HCAO_WAVE_MARK(P.wclk, kPhaseCollideScatter);
    if constexpr (MIX) {
      // Energy audit of the fp32 kinematics: the scattering intends the
      // kinetic energy of the total centre-of-mass motion plus the
      // translational energy handed to it (vibrational and formation energy
      // are bookkept in fp64 and cancel); the defect is the intended minus
      // the stored fp32 kinetic energy, less energy owed that joined here.
      if (P.m_moved) {
        mt = mt + mm3;
        px = px + mm3 * vm_in.x;
        py = py + mm3 * vm_in.y;
        pz = pz + mm3 * vm_in.z;
      }
      const double ke_int = (0.5 * ((px * px + py * py) + pz * pz)) / mt + P.et_out;
      double ke_out = 0.0;
      if (!P.dead0) ke_out = ke_out + kinetic(T.sp[P.sp0].mass, P.v0);
      if (!P.dead1) ke_out = ke_out + kinetic(T.sp[P.sp1].mass, P.v1);
      if (P.born) ke_out = ke_out + kinetic(T.sp[P.nb_sp].mass, P.nb_v);
      if (P.m_moved) ke_out = ke_out + kinetic(T.sp[P.sp_m].mass, P.v_m);
      wdef[HCAO_IDX(j, wcap, A.err)] = (ke_int - ke_out) - P.fold_used;
    }
    if (A.tdelta) {
      // the pair's change of its cell's running sums: its particles after
      // (p, q, the recoiling third body, the product) minus before (p, q,
      // the third body if it took part)
      double before[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, after[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      add_terms(before, T.sp[sp_in0].mass, v_in0);
      add_terms(before, T.sp[sp_in1].mass, v_in1);
      if (P.m_moved) add_terms(before, T.sp[P.sp_m].mass, vm_in);
      if (!P.dead0) add_terms(after, T.sp[P.sp0].mass, P.v0);
      if (!P.dead1) add_terms(after, T.sp[P.sp1].mass, P.v1);
      if (P.m_moved) add_terms(after, T.sp[P.sp_m].mass, P.v_m);
      if (P.born) add_terms(after, T.sp[P.nb_sp].mass, P.nb_v);
      const uint64_t e = HCAO_IDX(wbase + j, A.tdelta_stride, A.err);
      for (int x = 0; x < 5; ++x) A.tdelta[(size_t)x * A.tdelta_stride + e] = after[x] - before[x];
    }
    stv<MIX>(A.st, gp, P.v0);
    stv<MIX>(A.st, gq, P.v1);
    A.st.sp[gp] = P.dead0 ? (uint8_t)kDead : (uint8_t)P.sp0;
    A.st.sp[gq] = P.dead1 ? (uint8_t)kDead : (uint8_t)P.sp1;
    // the new species' modes, and zeros over the modes only the old species had
    // (a removed particle's levels are not kept)
    if (!P.dead0) {
      const uint32_t nn = T.sp[P.sp0].n_modes;
      store_levels(A.st, gp, nn, nn > nm0 ? nn : nm0, P.lv0, BLOCK);
    }
    if (!P.dead1) {
      const uint32_t nn = T.sp[P.sp1].n_modes;
      store_levels(A.st, gq, nn, nn > nm1 ? nn : nm1, P.lv1, BLOCK);
    }
    if constexpr (EX >= 2) {
      if (A.st.rot) {
        A.st.rot[gp] = P.dead0 ? 0.0 : P.r0;
        A.st.rot[gq] = P.dead1 ? 0.0 : P.r1;
      }
    }
    if (P.m_moved) stv<MIX>(A.st, gm, P.v_m);
    if (P.born) {
      const uint64_t gb = HCAO_IDX(wbase + j, A.born.n_slots, A.err);
      stv<MIX>(A.born, gb, P.nb_v);
      A.born.sp[gb] = (uint8_t)P.nb_sp;
      store_levels(A.born, gb, mm, A.born.lrow, P.lvn, BLOCK);
      if constexpr (EX >= 1) {
        if (A.born.rot) A.born.rot[gb] = P.rn;
        if (A.st.px) {
          const uint64_t gs = P.nb_from ? gq : gp;
          A.born.px[gb] = A.st.px[gs];
          A.born.py[gb] = A.st.py[gs];
          A.born.pz[gb] = A.st.pz[gs];
        }
      }
    }
    bflag[HCAO_IDX(j, wcap, A.err)] = (uint8_t)((P.born ? kFlagBorn : 0) | kFlagCollided);
    HCAO_WAVE_MARK(P.wclk, kPhaseCollideWrite);
#ifdef HCAO_PHASE_CLOCKS
    if (lead && A.clk)
      for (int x = 0; x < 5; ++x) atomicAdd(&A.clk[kPhaseCollideGather + x], (unsigned long long)P.wclk[x]);
#endif
    }
  }
  __syncthreads();
  HCAO_PHASE_MARK(kPhaseCollide);

  // ---- phase C: deaths, products in pair order, per-cell state ----
  // one wave per cell: ballots give each survivor its new slot and each
  // product its rank in pair order. In the mixed form the per-pair records
  // of a cell's first 64 candidates are loaded while the wave still works
  // on its previous cell, so that their latency overlaps it (the fp64 form
  // has no registers to spare for it).
  const bool records = MIX || A.tdelta != nullptr;
  constexpr bool kPrefetch = MIX;
  auto chunk_load = [&](uint32_t g, uint32_t k0, double (&y)[6], uint8_t &fl) {
    const CellHdr &H = hdr[g];
    const uint32_t k = k0 + lane;
    const bool in = k < H.ncand;
    const uint64_t e = wbase + H.cstart + k;
    for (int x = 0; x < 6; ++x) y[x] = 0.0;
    fl = 0;
    const uint32_t r = (uint32_t)HCAO_IDX(H.cstart + k, in ? wcap : ~0ull, A.err);
    if (MIX && in) fl = bflag[r];  // the mixed form's defect records need it too
    if (A.tdelta && in) {
      if (!MIX) fl = bflag[r];
      for (int x = 0; x < 5; ++x) y[x] = A.tdelta[(size_t)x * A.tdelta_stride + e];
    }
    if (MIX && in) y[5] = wdef[r];
  };
  double ny[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  uint8_t nfl = 0;
  if (kPrefetch && records && wave < ncell) chunk_load(wave, 0, ny, nfl);
  for (uint32_t g = wave; g < ncell; g += BLOCK / 64) {
    const CellHdr &H = hdr[g];
    const unsigned long long *in = l_ctr + (size_t)g * nctr;
    double cy[6];
    for (int x = 0; x < 6; ++x) cy[x] = ny[x];
    const uint8_t cfl = nfl;
    if (kPrefetch && records && g + BLOCK / 64 < ncell) chunk_load(g + BLOCK / 64, 0, ny, nfl);
    uint32_t alive = H.n;
    if (in[HCAO_CTR_DEATHS] != 0ull) {
      // stable in-place compaction: a chunk's survivors move to lower slots
      // after the whole chunk has been read
      uint32_t kept = 0;
      for (uint32_t i0 = 0; i0 < H.n; i0 += 64) {
        const uint32_t i = i0 + lane;
        const uint64_t src = HCAO_IDX(H.base + i, A.st.n_slots, A.err);
        const bool live = i < H.n && A.st.sp[src] != kDead;
        const unsigned long long m = __ballot(live);
        const uint64_t dst = HCAO_IDX(H.base + kept + (uint32_t)__popcll(m & lt), A.st.n_slots, A.err);
        V3<R> v{R(0), R(0), R(0)};
        uint8_t spv = 0;
        if (live) {
          v = ldv<MIX>(A.st, src);
          spv = A.st.sp[src];
        }
        if (live) {
          stv<MIX>(A.st, dst, v);
          A.st.sp[dst] = spv;
        }
        if (live) copy_levels(A.st, src, A.st, dst);
        if constexpr (EX >= 1) {
          if (A.st.rot) {
            double rv = 0.0;
            if (live) rv = A.st.rot[src];
            if (live) A.st.rot[dst] = rv;
          }
          if (A.st.px) {
            double x = 0.0, y = 0.0, z = 0.0;
            if (live) {
              x = A.st.px[src];
              y = A.st.py[src];
              z = A.st.pz[src];
            }
            if (live) {
              A.st.px[dst] = x;
              A.st.py[dst] = y;
              A.st.pz[dst] = z;
            }
          }
        }
        kept += (uint32_t)__popcll(m);
      }
      alive = kept;
    }
    const uint32_t births = (uint32_t)in[HCAO_CTR_BIRTHS];
    const bool overflow = alive + births > H.cap;
    if (births && !overflow) {
      uint32_t done = 0;
      for (uint32_t k0 = 0; k0 < H.ncand; k0 += 64) {
        const uint32_t k = k0 + lane;
        const bool f = k < H.ncand && (bflag[H.cstart + k] & kFlagBorn) != 0;
        const unsigned long long m = __ballot(f);
        if (f) {
          const uint64_t from = HCAO_IDX(wbase + H.cstart + k, A.born.n_slots, A.err),
                         to = HCAO_IDX(H.base + alive + done + (uint32_t)__popcll(m & lt), A.st.n_slots, A.err);
          stv<MIX>(A.st, to, ldv<MIX>(A.born, from));
          A.st.sp[to] = A.born.sp[from];
          copy_levels(A.born, from, A.st, to);
          if constexpr (EX >= 1) {
            if (A.st.rot) A.st.rot[to] = A.born.rot[from];
            if (A.st.px) {
              A.st.px[to] = A.born.px[from];
              A.st.py[to] = A.born.py[from];
              A.st.pz[to] = A.born.pz[from];
            }
          }
        }
        done += (uint32_t)__popcll(m);
      }
    }
    // Per-pair records of the cell, over chunks of 64 consecutive candidates
    // (left to right), each chunk reduced by a halving tree: the mixed
    // form's energy defects, and the changes of the running sums (a
    // candidate that did not collide contributes 0). A chunk's loads are all
    // issued before any is used.
    double dsum = 0.0, d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (records) {
      for (uint32_t k0 = 0; k0 < H.ncand; k0 += 64) {
        double y[6];
        uint8_t fl;
        if (kPrefetch && k0 == 0) {
          for (int x = 0; x < 6; ++x) y[x] = cy[x];
          fl = cfl;
        } else {
          chunk_load(g, k0, y, fl);
        }
        // (a record that phase B did not write is ignored)
        if (!(fl & kFlagCollided))
          for (int x = 0; x < (MIX ? 6 : 5); ++x) y[x] = 0.0;
        tree_sum(y);  // only lane 0's sums are used below
        for (int x = 0; x < 5; ++x) d[x] = d[x] + y[x];
        dsum = dsum + y[5];
      }
      if (A.tdelta && lane == 0)
        for (int x = 0; x < 5; ++x) hdr[g].tsum[x] = H.tsum[x] + d[x];
    }
    unsigned long long *tot = l_tot + (size_t)g * nctr;
    for (uint32_t i = lane; i < nctr; i += 64) {
      unsigned long long v = in[i];
      if (i == HCAO_CTR_CANDIDATES) v = H.ncand;
      if (i == HCAO_CTR_SUPPRESSED) v += H.excess;
      tot[i] += v;
    }
    if (lane == 0) {
      if (overflow) atomicOr(A.err, kErrCapacity);
      CellHdr &Hm = hdr[g];
      Hm.n = overflow ? alive : alive + births;
      const double seen = __longlong_as_double((long long)H.sgbits);
      Hm.sgmax = seen > H.sgmax ? seen : H.sgmax;
      Hm.rem = H.rem_new;
      if (MIX) Hm.defect = H.defect + dsum;
    }
  }
  __syncthreads();
  HCAO_PHASE_MARK(kPhasePlace);
  }  // steps

  // ---- persistent cell state back to HBM ----
  for (uint32_t g = wave; g < ncell; g += BLOCK / 64) {
    const CellHdr &H = hdr[g];
    const uint32_t c = H.cell;
    unsigned long long *out = A.cells.ctr + (size_t)c * kNumCtr;
    const unsigned long long *tot = l_tot + (size_t)g * nctr;
    for (uint32_t i = lane; i < nctr; i += 64)
      if (tot[i]) atomicAdd(&out[i], tot[i]);  // no return value: the wave does not wait
    if (lane == 0) {
      A.cells.cnt[c] = H.n;
      A.cells.sgmax[c] = H.sgmax;
      A.cells.rem[c] = H.rem;
      if (MIX) A.cells.defect[c] = H.defect;
      if (A.cells.tsum)
        for (int q = 0; q < 5; ++q) A.cells.tsum[(size_t)q * A.cells.n_cells + c] = H.tsum[q];
    }
  }
#ifdef HCAO_PHASE_CLOCKS
  HCAO_PHASE_MARK(kPhaseStore);
  if (tid == 0 && A.clk)
    for (int k = 0; k < kPhases; ++k) atomicAdd(&A.clk[k], (unsigned long long)clk_acc[k]);
#endif
}

// ---------------------------------------------------------------------------
// thermal initial state
// ---------------------------------------------------------------------------
__device__ __forceinline__ void polar_normals(Rng &rng, double &n1, double &n2) {
  double x, y, s;
  for (;;) {
    x = 2.0 * rng.uniform() - 1.0;
    y = 2.0 * rng.uniform() - 1.0;
    s = x * x + y * y;
    if (s < 1.0 && s > 0.0) break;
  }
  const double f = sqrt((-2.0 * dlog(s)) / s);
  n1 = x * f;
  n2 = y * f;
}

// Internal state of a new molecule at T_vib (levels) and T_rot (rotational
// energy): bends by the floor form, stretches by the uniform proposal with
// the Boltzmann acceptance, then (rotors only) Gamma(zeta/2, k T_rot):
// -ln(1 - u) plus, for zeta = 3, half the square of one polar normal. Writes
// the level row and the rotational energy of
// slot g. The thermal initial state and admission through open faces draw
// the same way.
__device__ __forceinline__ void sample_internal(const SpeciesTab &S, const double *lev, Rng &rng, double tv,
                                                double trot, const State &st, uint64_t g, uint32_t mm) {
  for (uint32_t m = 0; m < mm; ++m) {
    uint32_t l = 0;
    if (m < S.n_modes) {
      if (m < S.n_bend) {
        const double r = 1.0 - rng.uniform();
        const double lg = -dlog(r);
        double fi = floor(lg * (tv / S.theta[m]));
        fi = fi > 65535.0 ? 65535.0 : fi;
        l = (uint32_t)fi;
      } else {
        const uint32_t top = S.idiss[m];
        const double *L = lev + S.lev_off[m];
        const double kt = kBoltz * tv;
        for (;;) {
          const double u = rng.uniform();
          uint32_t j = (uint32_t)floor(u * (double)(top + 1));
          j = j > top ? top : j;
          const double u2 = rng.uniform();
          const double xx = (L[j] - L[0]) / kt;
          if (u2 < dexp(-xx)) {
            l = j;
            break;
          }
        }
      }
    }
    st.lvl[g * st.lrow + m] = (uint16_t)l;
  }
  for (uint32_t m = mm; m < st.lrow; ++m) st.lvl[g * st.lrow + m] = 0;
  if (st.rot) {
    double e = 0.0;
    if (S.zeta_rot > 0) {
      double gm = -dlog(1.0 - rng.uniform());
      if (S.zeta_rot == 3) {
        double z1, z2;
        polar_normals(rng, z1, z2);
        gm = gm + 0.5 * (z1 * z1);
      }
      e = (kBoltz * trot) * gm;
    }
    st.rot[g] = e;
  }
}

struct InitArgs {
  const Tables *tab;
  const double *lev;
  State st;
  const uint64_t *off;
  const uint32_t *counts;  // [n_cells][n_species]
  const double *t_trans, *t_vib;
  uint64_t seed;
  uint32_t n_cells;
  uint32_t nx, ny, nz;  // spatial mode grid (positions drawn when st.px is set)
  double len[3];
};

__global__ __launch_bounds__(256) void k_init(InitArgs A) {
  const uint32_t c = blockIdx.x;
  const Tables &T = *A.tab;
  const uint32_t ns = T.n_species, mm = T.max_modes;
  const uint32_t *cnt = A.counts + (size_t)c * ns;
  uint32_t n = 0;
  for (uint32_t s = 0; s < ns; ++s) n += cnt[s];
  const double tt = A.t_trans[c], tv = A.t_vib[c];
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    uint32_t s = 0, acc = cnt[0];
    while (i >= acc) acc += cnt[++s];
    const SpeciesTab &S = T.sp[s];
    Rng rng;
    rng.open(A.seed, i, c, 0xFFFFFFFEu);
    double n1, n2, n3, n4;
    polar_normals(rng, n1, n2);
    polar_normals(rng, n3, n4);
    const double sigma = sqrt((kBoltz * tt) / S.mass);
    const uint64_t g = A.off[c] + i;
    store_vel(A.st, g, sigma * n1, sigma * n2, sigma * n3);
    A.st.sp[g] = (uint8_t)s;
    sample_internal(S, A.lev, rng, tv, tt, A.st, g, mm);
    if (A.st.px) {
      // spatial mode: uniform in the cell, one draw per axis
      const uint32_t ix = c % A.nx, iy = (c / A.nx) % A.ny, iz = c / (A.nx * A.ny);
      A.st.px[g] = ((double)ix + rng.uniform()) * (A.len[0] / (double)A.nx);
      A.st.py[g] = ((double)iy + rng.uniform()) * (A.len[1] / (double)A.ny);
      A.st.pz[g] = ((double)iz + rng.uniform()) * (A.len[2] / (double)A.nz);
    }
  }
}

// ---------------------------------------------------------------------------
// initial (sigma g)_max bound per cell: max over present species pairs of
// C (4 max|v|^2)^(1-w); remainder reset
// ---------------------------------------------------------------------------
struct CellInitArgs {
  const Tables *tab;
  State st;
  CellArrays cells;
};

__global__ __launch_bounds__(256) void k_cell_init(CellInitArgs A) {
  __shared__ unsigned long long s_v;
  __shared__ uint32_t s_mask;
  const uint32_t c = blockIdx.x;
  const uint64_t base = A.cells.off[c];
  const uint32_t n = A.cells.cnt[c];
  if (threadIdx.x == 0) {
    s_v = 0ull;
    s_mask = 0u;
  }
  __syncthreads();
  double vmax2 = 0.0;
  uint32_t mask = 0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const Vec3 v = load_vel(A.st, base + i);
    const double v2 = (v.x * v.x + v.y * v.y) + v.z * v.z;
    vmax2 = v2 > vmax2 ? v2 : vmax2;
    mask |= 1u << A.st.sp[base + i];
  }
  atomicMax(&s_v, (unsigned long long)__double_as_longlong(vmax2));
  atomicOr(&s_mask, mask);
  if (A.cells.tsum && threadIdx.x < 64) {
    // the running sums of the cell temperature start from the particles
    double sums[5];
    if (A.st.fx)
      cell_sums<true>(A.st, A.tab->sp, base, n, threadIdx.x, sums);
    else
      cell_sums<false>(A.st, A.tab->sp, base, n, threadIdx.x, sums);
    if (threadIdx.x == 0)
      for (int q = 0; q < 5; ++q) A.cells.tsum[(size_t)q * A.cells.n_cells + c] = sums[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const Tables &T = *A.tab;
    const double g2 = 4.0 * __longlong_as_double((long long)s_v);
    double best = 0.0;
    if (g2 > 0.0) {
      for (uint32_t a = 0; a < T.n_species; ++a) {
        if (!((s_mask >> a) & 1u)) continue;
        for (uint32_t b = 0; b < T.n_species; ++b) {
          if (!((s_mask >> b) & 1u)) continue;
          const double sg = T.pr[a][b].csg * dpow(g2, T.pr[a][b].esg);
          best = sg > best ? sg : best;
        }
      }
    }
    A.cells.sgmax[c] = best;
    A.cells.rem[c] = 0.0;
    unsigned long long *ctr = A.cells.ctr + (size_t)c * kNumCtr;
    for (int i = 0; i < kNumCtr; ++i) ctr[i] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// moments per cell: [0..2] sum m v, [3] sum m |v|^2, [4] sum m, [5] sum h_s,
// [6 + s] count_s, [6 + S + s] sum (E_vib - ZPE)_s. Thread partials are
// combined by a fixed halving tree.
// ---------------------------------------------------------------------------
struct MomentArgs {
  const Tables *tab;
  const double *lev;
  State st;
  const uint64_t *off;
  const uint32_t *cnt;
  double *out;  // [n_cells][6 + 3 S]: sums, counts, E_vib above ZPE, E_rot per species
};

__global__ __launch_bounds__(256) void k_moments(MomentArgs A) {
  constexpr int kB = 256;
  constexpr int kW = 6 + 3 * kMaxSpecies;
  __shared__ double s_red[kB];
  const uint32_t c = blockIdx.x;
  const Tables &T = *A.tab;
  const uint32_t ns = T.n_species;
  const uint64_t base = A.off[c];
  const uint32_t n = A.cnt[c];
  double acc[kW];
#pragma unroll
  for (int j = 0; j < kW; ++j) acc[j] = 0.0;
  for (uint32_t i = threadIdx.x; i < n; i += kB) {
    const uint64_t g = base + i;
    const uint32_t s = A.st.sp[g];
    const SpeciesTab &S = T.sp[s];
    const double m = S.mass;
    const Vec3 v = load_vel(A.st, g);
    const double vx = v.x, vy = v.y, vz = v.z;
    acc[0] += m * vx;
    acc[1] += m * vy;
    acc[2] += m * vz;
    acc[3] += m * ((vx * vx + vy * vy) + vz * vz);
    acc[4] += m;
    acc[5] += S.formation;
    double ev = 0.0;
    for (uint32_t q = 0; q < S.n_modes; ++q) ev = ev + mode_energy(S, A.lev, q, A.st.lvl[g * A.st.lrow + q]);
    const double er = A.st.rot ? A.st.rot[g] : 0.0;
#pragma unroll
    for (int j = 0; j < kMaxSpecies; ++j) {
      if ((uint32_t)j == s) {
        acc[6 + j] += 1.0;
        acc[6 + kMaxSpecies + j] += ev - S.zpe;
        acc[6 + 2 * kMaxSpecies + j] += er;
      }
    }
  }
  double *out = A.out + (size_t)c * (6 + 3 * ns);
#pragma unroll
  for (int j = 0; j < kW; ++j) {
    const int blk = j < 6 ? -1 : (j - 6) / kMaxSpecies, sj = j < 6 ? 0 : (j - 6) % kMaxSpecies;
    const bool used = j < 6 || sj < (int)ns;
    if (!used) continue;
    s_red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) s_red[threadIdx.x] += s_red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int dst = j < 6 ? j : 6 + blk * (int)ns + sj;
      out[dst] = s_red[0];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// stable counting sort of particles by cell (LSD radix, 8-bit digits):
// per-tile digit histograms, one exclusive scan in digit-major order, and a
// stable scatter that ranks equal digits inside a wavefront with ballots.
// ---------------------------------------------------------------------------
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr uint32_t kSortMaxBits = 9;  // digit width of a pass: up to 9 bits (512 bins)
constexpr uint32_t kSortMaxBins = 1u << kSortMaxBits;

__global__ __launch_bounds__(kSortBlock) void k_sort_hist(const uint32_t *keys, uint64_t n, uint32_t shift,
                                                          uint32_t bits, uint32_t *hist, uint32_t n_tiles) {
  __shared__ uint32_t s_h[kSortMaxBins];
  const uint32_t bins = 1u << bits, mask = bins - 1u;
  for (uint32_t b = threadIdx.x; b < bins; b += kSortBlock) s_h[b] = 0;
  __syncthreads();
  const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const uint64_t i = t0 + (uint64_t)it * kSortBlock + threadIdx.x;
    if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < bins; b += kSortBlock) hist[(uint64_t)b * n_tiles + blockIdx.x] = s_h[b];
}

// Multi-block exclusive scan of u32 into u64: each 1024-thread block scans
// a chunk of kScanChunk entries (16 per thread) and leaves its total in
// bsum; one block then scans the totals; a third pass adds each chunk's
// offset. Integer sums, so the result does not depend on the split.
constexpr int kScanPer = 16;
constexpr uint64_t kScanChunk = 1024 * kScanPer;

__global__ __launch_bounds__(1024) void k_scan_chunk(const uint32_t *in, uint64_t *out, uint64_t n, uint64_t *bsum) {
  __shared__ uint64_t s_part[1024];
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint64_t sum = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (b0 + k < n) sum += in[b0 + k];
  s_part[threadIdx.x] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t v = (int)threadIdx.x >= d ? s_part[threadIdx.x - d] : 0;
    __syncthreads();
    s_part[threadIdx.x] += v;
    __syncthreads();
  }
  uint64_t acc = s_part[threadIdx.x] - sum;
  for (int k = 0; k < kScanPer; ++k)
    if (b0 + k < n) {
      out[b0 + k] = acc;
      acc += in[b0 + k];
    }
  if (threadIdx.x == 1023) bsum[blockIdx.x] = s_part[1023];
}

__global__ __launch_bounds__(1024) void k_scan_top(uint64_t *bsum, uint64_t nb) {
  __shared__ uint64_t s_part[1024];
  const uint64_t b0 = (uint64_t)threadIdx.x * kScanPer;
  uint64_t sum = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (b0 + k < nb) sum += bsum[b0 + k];
  s_part[threadIdx.x] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t v = (int)threadIdx.x >= d ? s_part[threadIdx.x - d] : 0;
    __syncthreads();
    s_part[threadIdx.x] += v;
    __syncthreads();
  }
  uint64_t acc = s_part[threadIdx.x] - sum;
  for (int k = 0; k < kScanPer; ++k)
    if (b0 + k < nb) {
      const uint64_t v = bsum[b0 + k];
      bsum[b0 + k] = acc;
      acc += v;
    }
}

__global__ __launch_bounds__(256) void k_scan_add(uint64_t *out, uint64_t n, const uint64_t *bsum) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / kScanChunk];
}

__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(const uint32_t *keys_in, const uint32_t *idx_in,
                                                             uint32_t *keys_out, uint32_t *idx_out, uint64_t n,
                                                             uint32_t shift, uint32_t bits, const uint64_t *offs,
                                                             uint32_t n_tiles) {
  constexpr int kWaves = kSortBlock / 64;
  __shared__ uint32_t s_run[kSortMaxBins];
  __shared__ uint32_t s_wave[kWaves][kSortMaxBins];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t bins = 1u << bits, mask = bins - 1u;
  for (uint32_t b = tid; b < bins; b += kSortBlock) s_run[b] = 0;
  __syncthreads();
  const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
  const unsigned long long lt = lane ? ((1ull << lane) - 1ull) : 0ull;
  // the tile's keys and indices are loaded at once, before the ranking
  // rounds (whose barriers would otherwise wait on each round's loads)
  uint32_t kr[kSortItems], ir[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const uint64_t i = t0 + (uint64_t)it * kSortBlock + tid;
    kr[it] = i < n ? keys_in[i] : 0u;
    ir[it] = i < n ? idx_in[i] : 0u;
  }
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    for (int w = 0; w < kWaves; ++w)
      for (uint32_t b = tid; b < bins; b += kSortBlock) s_wave[w][b] = 0;
    __syncthreads();
    const uint64_t i = t0 + (uint64_t)it * kSortBlock + tid;
    const bool valid = i < n;
    const uint32_t key = kr[it];
    const uint32_t d = (key >> shift) & mask;
    unsigned long long same = __ballot(valid);
#pragma unroll
    for (uint32_t bit = 0; bit < kSortMaxBits; ++bit) {
      if (bit < bits) {  // the same on every lane
        const unsigned long long bb = __ballot(((d >> bit) & 1u) != 0u);
        same &= ((d >> bit) & 1u) ? bb : ~bb;
      }
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt);
    if (valid && rank == 0) s_wave[wave][d] = (uint32_t)__popcll(same);
    __syncthreads();
    uint32_t before = s_run[d];
    for (uint32_t w = 0; w < wave; ++w) before += s_wave[w][d];
    if (valid) {
      const uint64_t pos = offs[(uint64_t)d * n_tiles + blockIdx.x] + before + rank;
      keys_out[pos] = key;
      idx_out[pos] = ir[it];
    }
    __syncthreads();
    for (uint32_t b = tid; b < bins; b += kSortBlock) {
      uint32_t add = 0;
      for (int w = 0; w < kWaves; ++w) add += s_wave[w][b];
      s_run[b] += add;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// load: validate host particles, count per cell, place in sorted order
// ---------------------------------------------------------------------------
struct LoadArgs {
  const Tables *tab;
  const uint32_t *cell;
  const uint8_t *sp;
  const double *vel;   // 3n
  const uint16_t *lvl; // n x mm
  uint64_t n;
  uint32_t n_cells;
  uint32_t *count;     // [n_cells]
  uint32_t *err;
};

__global__ __launch_bounds__(256) void k_load_check(LoadArgs A) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const Tables &T = *A.tab;
  const uint32_t mm = T.max_modes;
  uint32_t err = 0;
  const uint32_t c = A.cell[i], s = A.sp[i];
  if (c >= A.n_cells || s >= T.n_species) {
    err |= kErrInvalid;
  } else {
    const double vx = A.vel[3 * i], vy = A.vel[3 * i + 1], vz = A.vel[3 * i + 2];
    if (!isfinite(vx) || !isfinite(vy) || !isfinite(vz)) err |= kErrNonFinite;
    const SpeciesTab &S = T.sp[s];
    for (uint32_t m = 0; m < mm; ++m) {
      const uint32_t l = A.lvl[i * mm + m];
      if (m >= S.n_modes) {
        if (l != 0) err |= kErrLevel;
      } else if (m >= S.n_bend && l > S.idiss[m]) {
        err |= kErrLevel;
      }
    }
    atomicAdd(&A.count[c], 1u);
  }
  if (err) atomicOr(A.err, err);
}

struct PlaceArgs {
  const Tables *tab;
  const uint32_t *sorted_cell, *sorted_idx;
  const uint64_t *packed_start;  // exclusive scan of counts
  const uint64_t *off;           // slot offsets
  const uint8_t *sp;
  const double *vel;
  const uint16_t *lvl;
  const double *rot;  // may be null
  const double *pos;  // 3n, spatial mode
  State st;
  uint64_t n;
};

__global__ __launch_bounds__(256) void k_load_place(PlaceArgs A) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.n) return;
  const uint32_t c = A.sorted_cell[j];
  const uint64_t src = A.sorted_idx[j];
  const uint64_t g = A.off[c] + (j - A.packed_start[c]);
  const uint32_t mm = A.tab->max_modes;
  store_vel(A.st, g, A.vel[3 * src], A.vel[3 * src + 1], A.vel[3 * src + 2]);
  A.st.sp[g] = A.sp[src];
  for (uint32_t m = 0; m < A.st.lrow; ++m) A.st.lvl[g * A.st.lrow + m] = m < mm ? A.lvl[src * mm + m] : (uint16_t)0;
  if (A.st.rot) A.st.rot[g] = A.rot ? A.rot[src] : 0.0;
  if (A.st.px) {
    A.st.px[g] = A.pos[3 * src];
    A.st.py[g] = A.pos[3 * src + 1];
    A.st.pz[g] = A.pos[3 * src + 2];
  }
}

// advances the device step index after the launches of a graph replay
__global__ void k_advance(uint32_t *step, uint32_t n) {
  if (threadIdx.x == 0) step[0] = step[0] + n;
}

__global__ void k_iota(uint32_t *x, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (uint32_t)i;
}


// ---------------------------------------------------------------------------
// Eq. recomb-correct: forward probability summed over every combination of
// vibrational levels (set-up work, not part of the step)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double level_above_ground(const SpeciesTab &S, const double *lev, uint32_t m, uint32_t j) {
  return mode_energy(S, lev, m, j) - mode_energy(S, lev, m, 0);
}

template <bool WRITE>
__global__ __launch_bounds__(256) void k_rec_enum(RecEnumArgs A) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= A.n_prefix) return;
  const SpeciesTab &S = A.tab->sp[A.species];
  const uint32_t nm = S.n_modes, np = A.n_prefix_modes;
  uint32_t j[kMaxModes];
  double st[kMaxModes + 1];
  uint64_t x = tid;
  for (uint32_t m = 0; m < np; ++m) {
    j[m] = (uint32_t)(x % A.box[m]);
    x /= A.box[m];
  }
  uint32_t n = 0;
  const uint64_t o = WRITE ? A.offset[tid] : 0;
  auto emit = [&](double e, uint32_t code) {
    if (WRITE) {
      A.rec_e[o + n] = e;
      A.rec_code[o + n] = code;
    }
    ++n;
  };
  // the prefix: valid while below de; a crossing inside it is emitted once,
  // by the prefix whose crossing level is the first one and whose later
  // digits are 0
  double s = 0.0;
  bool walk = true;
  for (uint32_t m = 0; m < np && walk; ++m) {
    if (m >= S.n_bend && j[m] > S.idiss[m]) {
      walk = false;
      break;
    }
    const double s2 = s + level_above_ground(S, A.lev, m, j[m]);
    if (!(s2 < A.de)) {
      bool first = j[m] == 0 || s + level_above_ground(S, A.lev, m, j[m] - 1) < A.de;
      for (uint32_t k = m + 1; k < np; ++k) first = first && j[k] == 0;
      if (first) emit(s2, m | (j[m] << 8));
      walk = false;
      break;
    }
    s = s2;
  }
  if (walk) {
    if (np == nm) {
      emit(s, kRecLeaf);
    } else {
      uint32_t m = np;
      j[m] = 0;
      st[m] = s;
      for (;;) {
        bool back = false;
        if (m >= S.n_bend && j[m] > S.idiss[m]) {
          back = true;
        } else {
          const double s2 = st[m] + level_above_ground(S, A.lev, m, j[m]);
          if (!(s2 < A.de)) {
            emit(s2, m | (j[m] << 8));
            back = true;
          } else if (m + 1 == nm) {
            emit(s2, kRecLeaf);
            ++j[m];
          } else {
            st[m + 1] = s2;
            j[m + 1] = 0;
            ++m;
          }
        }
        if (back) {
          if (m == np) break;
          --m;
          ++j[m];
        }
      }
    }
  }
  if (!WRITE) A.count[tid] = n;
}

// Regularized upper incomplete gamma Q(a, x) times exp(-y), x > 0 (series
// for the lower function below x = a + 1, Lentz's continued fraction above;
// Press et al., Numerical Recipes 6.2); the prefactor joins exp(-y) in one
// exponent so that small terms do not underflow early.
__device__ double gamma_q_scaled(double a, double x, double lga, double y) {
  const double lpre = (a * log(x) - x) - lga;
  if (x < a + 1.0) {
    double ap = a, del = 1.0 / a, sum = del;
    for (int i = 1; i <= 1000; ++i) {
      ap += 1.0;
      del *= x / ap;
      sum += del;
      if (fabs(del) < fabs(sum) * 1e-17) break;
    }
    return (1.0 - sum * exp(lpre)) * exp(-y);
  }
  const double tiny = 1e-300;
  double b = (x + 1.0) - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i <= 1000; ++i) {
    const double an = -(double)i * ((double)i - a);
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (fabs(del - 1.0) < 1e-17) break;
  }
  return exp(lpre - y) * h;
}

__global__ __launch_bounds__(256) void k_rec_sum(RecSumArgs A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  double *tail = reinterpret_cast<double *>(smem);  // stretch levels: sum_{k >= j} exp(-beta (e_k - e_j))
  __shared__ double s_z[kMaxModes + 1], s_bend[kMaxModes], s_red[256];
  const SpeciesTab &S = A.tab->sp[A.species];
  const uint32_t nm = S.n_modes, tid = threadIdx.x;
  const double beta = 1.0 / (kBoltz * A.t[blockIdx.x]);
  if (tid < nm) {
    const uint32_t m = tid;
    if (m < S.n_bend) {
      const double z = 1.0 / (1.0 - exp(-(beta * S.kt[m])));
      s_bend[m] = z;
      s_z[m] = z;
    } else {
      // tail sums from the top level down; the partition sum is tail[0]
      const uint32_t base = S.lev_off[m] - S.lev_off[S.n_bend];
      const uint32_t top = S.idiss[m];
      tail[base + top] = 1.0;
      for (uint32_t k = top; k-- > 0;) {
        const double step = level_above_ground(S, A.lev, m, k + 1) - level_above_ground(S, A.lev, m, k);
        tail[base + k] = 1.0 + exp(-(beta * step)) * tail[base + k + 1];
      }
      s_z[m] = tail[base];
    }
  }
  __syncthreads();
  if (tid == 0) {
    // s_z[m] becomes the product of the partition sums of modes m..nm-1
    double z = 1.0;
    s_z[nm] = 1.0;
    for (uint32_t m = nm; m-- > 0;) {
      z = z * s_z[m];
      s_z[m] = z;
    }
  }
  __syncthreads();
  double acc = 0.0;
  for (uint64_t i = tid; i < A.n_rec; i += 256) {
    const double e = A.rec_e[i];
    const uint32_t code = A.rec_code[i];
    if (code == kRecLeaf) {
      acc += gamma_q_scaled(A.a, beta * (A.de - e), A.lgamma_a, beta * e);
    } else {
      const uint32_t m = code & 0xFFu, jj = code >> 8;
      const double rel = m < S.n_bend ? s_bend[m] : tail[(S.lev_off[m] - S.lev_off[S.n_bend]) + jj];
      acc += (exp(-(beta * e)) * rel) * s_z[m + 1];
    }
  }
  s_red[tid] = acc;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
    if (tid < w) s_red[tid] = s_red[tid] + s_red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    A.num[blockIdx.x] = s_red[0];
    A.den[blockIdx.x] = s_z[0];
  }
}


// ---------------------------------------------------------------------------
// spatial mode: ballistic move with periodic or specular walls, then a
// stable re-bin by (new cell, old slot) that sorts only the particles that
// left their cell
// ---------------------------------------------------------------------------
// one coordinate over dt: periodic axes wrap into [0, L); a specular face
// reflects (x < 0: -x, x > L: 2L - x, velocity reversed; flip set) until
// inside [0, L]; crossing an open face sets left and ends the move
__device__ __forceinline__ double move_axis(double x, double &v, double dt, double len, bool periodic, bool open_lo,
                                           bool open_hi, bool &left, bool &flip) {
  double y = x + v * dt;
  if (periodic) {
    while (y < 0.0) y = y + len;
    while (y >= len) y = y - len;
  } else {
    for (;;) {
      if (y < 0.0) {
        if (open_lo) {
          left = true;
          break;
        }
        y = -y;
        v = -v;
        flip = true;
      } else if (y > len) {
        if (open_hi) {
          left = true;
          break;
        }
        y = (len + len) - y;
        v = -v;
        flip = true;
      } else {
        break;
      }
    }
  }
  return y;
}

// a particle over dt on x, then y, then z; true if it leaves through an open
// face (its coordinates are then of no use); flip tells whether a specular
// face reversed a velocity component
__device__ __forceinline__ bool move_particle(double &x, double &y, double &z, double &vx, double &vy, double &vz,
                                              double dt, const double len[3], uint32_t periodic, uint32_t open,
                                              bool &flip) {
  bool left = false;
  x = move_axis(x, vx, dt, len[0], (periodic & 1u) != 0, (open & 1u) != 0, (open & 2u) != 0, left, flip);
  if (left) return true;
  y = move_axis(y, vy, dt, len[1], (periodic & 2u) != 0, (open & 4u) != 0, (open & 8u) != 0, left, flip);
  if (left) return true;
  z = move_axis(z, vz, dt, len[2], (periodic & 4u) != 0, (open & 16u) != 0, (open & 32u) != 0, left, flip);
  return left;
}

__device__ __forceinline__ uint32_t axis_index(double x, double len, uint32_t n) {
  const double f = floor(x / (len / (double)n));
  if (!(f >= 0.0)) return 0;
  if (f >= (double)n) return n - 1;
  return (uint32_t)f;
}

// one workgroup of four waves per cell; ranks in slot order come from
// ballots within a wave and the per-wave totals in LDS
__global__ __launch_bounds__(256) void k_move(MoveArgs A) {
  __shared__ uint32_t s_wave[2][4];
  const uint32_t c = blockIdx.x, tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  const uint64_t base = A.off[c];
  const uint32_t n = A.cnt[c], top = A.cap[c] - 1u;
  const uint64_t below_lane = (1ull << lane) - 1ull;
  uint32_t run_s = 0, run_m = 0;
  for (uint32_t i0 = 0; i0 < n; i0 += 256) {
    const uint32_t i = i0 + tid;
    const uint64_t g = base + i;
    bool mover = false, stayer = false;
    uint32_t key = 0;
    if (i < n) {
      const Vec3 v = load_vel(A.st, g);
      double vx = v.x, vy = v.y, vz = v.z;
      double x = A.st.px[g], y = A.st.py[g], z = A.st.pz[g];
      bool flip = false;
      // the moved state is not stored: the place pass moves the particle
      // again as it copies it (the same arithmetic, so the same bits)
      if (!move_particle(x, y, z, vx, vy, vz, A.dt, A.len, A.periodic, A.open, flip)) {
        key = axis_index(x, A.len[0], A.nx) +
              A.nx * (axis_index(y, A.len[1], A.ny) + A.ny * axis_index(z, A.len[2], A.nz));
        mover = key != c;
        stayer = !mover;
      }
    }
    const uint64_t bm = __ballot(mover), bs = __ballot(stayer);
    if (lane == 0) {
      s_wave[0][wv] = (uint32_t)__popcll(bs);
      s_wave[1][wv] = (uint32_t)__popcll(bm);
    }
    __syncthreads();
    uint32_t pre_s = run_s, pre_m = run_m;
    for (uint32_t w = 0; w < 4; ++w) {
      const uint32_t ns = s_wave[0][w], nm = s_wave[1][w];
      if (w < wv) {
        pre_s += ns;
        pre_m += nm;
      }
      run_s += ns;
      run_m += nm;
    }
    // stayer ranks count up from the first slot, mover ranks down from the
    // last: together they never pass n <= cap entries
    if (mover) {
      const uint64_t at = base + top - (pre_m + (uint32_t)__popcll(bm & below_lane));
      A.list[at] = i;
      A.key[at] = key;
    }
    if (stayer) A.list[base + pre_s + (uint32_t)__popcll(bs & below_lane)] = i;
    __syncthreads();
  }
  if (tid == 0) {
    A.n_stay[c] = run_s;
    A.n_move[c] = run_m;
    const uint32_t gone = n - run_s - run_m;
    if (gone && A.flux) atomicAdd(&A.flux[1], (unsigned long long)gone);
  }
}

// geometry of face cell t / n_species: face f, its axis k and side, the two
// tangential axes a < b, the face cell's indices and the cell behind it
struct FaceCell {
  uint32_t f, k, side, a, b, ia, ib, cell;
  double da, db;
};
__device__ __forceinline__ FaceCell face_cell(const InflowArgs &A, uint32_t gfc) {
  FaceCell F;
  F.f = 0;
  while (gfc >= A.face_base[F.f + 1]) ++F.f;
  F.k = F.f >> 1;
  F.side = F.f & 1u;
  F.a = F.k == 0 ? 1u : 0u;
  F.b = F.k == 2 ? 1u : 2u;
  const uint32_t n3[3] = {A.nx, A.ny, A.nz};
  const uint32_t na = n3[F.a], nb = n3[F.b];
  const uint32_t j = gfc - A.face_base[F.f];
  F.ia = j % na;
  F.ib = j / na;
  uint32_t idx[3];
  idx[F.k] = F.side ? n3[F.k] - 1u : 0u;
  idx[F.a] = F.ia;
  idx[F.b] = F.ib;
  F.cell = idx[0] + A.nx * (idx[1] + A.ny * idx[2]);
  F.da = A.len[F.a] / (double)na;
  F.db = A.len[F.b] / (double)nb;
  return F;
}

__global__ __launch_bounds__(256) void k_inflow_count(InflowArgs A) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t ns = A.n_species;
  if (t >= (uint64_t)A.face_base[6] * ns) return;
  const uint32_t gfc = (uint32_t)(t / ns), s = (uint32_t)(t % ns);
  const FaceCell F = face_cell(A, gfc);
  uint32_t cnt = 0;
  if ((A.open >> F.f) & 1u) {
    const double area = F.da * F.db;
    const double x = ((A.flux_s[s] * area) * A.dt) / A.weight[F.cell] + A.rem[t];
    const double fl = floor(x);
    if (fl < 16777216.0) {
      cnt = (uint32_t)fl;
      A.rem[t] = x - fl;
    } else {
      atomicOr(A.err, kErrCapacity);
    }
  }
  A.count[t] = cnt;
}

// admission j of the step: its (face cell, species) t is the last with
// ibase[t] <= j (entries without admissions share the next one's base), i =
// j - ibase[t]. Normal speed from the flux-weighted Maxwellian, sigma
// sqrt(-2 ln(1 - u)); tangential speeds, a polar normal pair times sigma;
// the flight fraction tau; the place on the face cell, uniform per
// tangential axis; levels and rotation as the thermal initial state draws
// them; then a move over tau dt
__global__ __launch_bounds__(256) void k_inflow_make(InflowArgs A) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.n_ins) return;
  if (j >= A.cap_ins) {
    atomicOr(A.err, kErrCapacity);
    return;
  }
  const uint32_t ns = A.n_species;
  uint64_t lo = 0, hi = (uint64_t)A.face_base[6] * ns - 1;
  while (lo < hi) {
    const uint64_t mid = (lo + hi + 1) >> 1;
    if (A.ibase[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  const uint64_t t = lo;
  const uint32_t i = (uint32_t)(j - A.ibase[t]);
  const uint32_t gfc = (uint32_t)(t / ns), s = (uint32_t)(t % ns);
  const FaceCell F = face_cell(A, gfc);
  const SpeciesTab &S = A.tab->sp[s];
  const uint32_t mm = A.tab->max_modes;
  const double sigma = sqrt((kBoltz * A.t_trans) / S.mass);
  Rng rng;
  rng.open(A.seed, (s << 24) | i, A.n_cells + gfc, A.step);
  const double vn = sigma * sqrt(-2.0 * dlog(1.0 - rng.uniform()));
  double n1, n2;
  polar_normals(rng, n1, n2);
  const double tau = rng.uniform();
  const double ua = rng.uniform();
  const double ub = rng.uniform();
  double p[3], v[3];
  p[F.k] = F.side ? A.len[F.k] : 0.0;
  v[F.k] = F.side ? -vn : vn;
  p[F.a] = ((double)F.ia + ua) * F.da;
  p[F.b] = ((double)F.ib + ub) * F.db;
  v[F.a] = sigma * n1;
  v[F.b] = sigma * n2;
  A.ins.sp[j] = (uint8_t)s;
  sample_internal(S, A.lev, rng, A.t_vib, A.t_trans, A.ins, j, mm);
  bool flip = false;
  const bool left =
      move_particle(p[0], p[1], p[2], v[0], v[1], v[2], tau * A.dt, A.len, A.periodic, A.open, flip);
  store_vel(A.ins, j, v[0], v[1], v[2]);
  A.ins.px[j] = p[0];
  A.ins.py[j] = p[1];
  A.ins.pz[j] = p[2];
  const uint64_t m_real = A.mbase[A.n_cells];
  A.mkey[m_real + j] = left ? A.n_cells
                            : axis_index(p[0], A.len[0], A.nx) +
                                  A.nx * (axis_index(p[1], A.len[1], A.ny) + A.ny * axis_index(p[2], A.len[2], A.nz));
  A.mslot[m_real + j] = (uint32_t)(A.tot + j);
  if (i == 0) atomicAdd(&A.flux[0], (unsigned long long)A.count[t]);
  if (left) atomicAdd(&A.flux[1], 1ull);
}

// movers of cell c into the list, in slot order
// (one wave per cell, four cells per workgroup)
__global__ __launch_bounds__(256) void k_list_movers(RebinArgs A) {
  const uint32_t c = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (c >= A.n_cells) return;
  const uint32_t nm = A.n_move[c];
  const uint64_t base = A.off[c], mb = A.mbase[c];
  const uint64_t top = base + A.cap[c] - 1u;
  for (uint32_t r = threadIdx.x & 63u; r < nm; r += 64u) {
    A.mkey[mb + r] = A.key[top - r];
    A.mslot[mb + r] = (uint32_t)(base + A.list[top - r]);
  }
}

// start of every key's run in the sorted keys: packed[c] = first j with
// key[j] >= c, for c = 0..n_cells (packed[n_cells] = n); each run boundary
// fills the starts of the keys it skips
__global__ __launch_bounds__(256) void k_run_starts(const uint32_t *key, uint64_t n, uint32_t n_cells,
                                                    uint64_t *packed) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t k = key[j] < n_cells ? key[j] : n_cells;
  const uint32_t prev = j ? (key[j - 1] < n_cells ? key[j - 1] : n_cells) : 0u;
  const uint32_t from = j ? prev + 1 : 0u;
  if (j == 0 || k != prev)
    for (uint32_t c = from; c <= k; ++c) packed[c] = j;
  if (j == n - 1)
    for (uint32_t c = k + 1; c <= n_cells; ++c) packed[c] = n;
}

__device__ __forceinline__ void copy_particle(const State &s, const State &d, uint64_t from, uint64_t to, uint32_t mm) {
  if (s.fx) {
    d.fx[to] = s.fx[from];
    d.fy[to] = s.fy[from];
    d.fz[to] = s.fz[from];
  } else {
    d.vx[to] = s.vx[from];
    d.vy[to] = s.vy[from];
    d.vz[to] = s.vz[from];
  }
  d.sp[to] = s.sp[from];
  copy_levels(s, from, d, to);
  if (s.rot) d.rot[to] = s.rot[from];
  d.px[to] = s.px[from];
  d.py[to] = s.py[from];
  d.pz[to] = s.pz[from];
}

// per new cell k: the split of its run of sorted list entries at the first
// entry from a slot above off[k] (by bisection: the run is in slot order),
// its count (capped at its capacity, which raises the capacity error; the
// place pass stores it) and where its particles go (RebinDest). One thread
// per cell.
__global__ __launch_bounds__(256) void k_rebin_cells(RebinArgs A) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= A.n_cells) return;
  const uint64_t base = A.off[k];
  uint64_t lo = 0, hi = 0;
  if (A.m) {
    lo = A.packed[k];
    hi = A.packed[k + 1];
  }
  uint64_t a = lo, b = hi;
  while (a < b) {
    const uint64_t mid = (a + b) >> 1;
    if (A.mslot[A.sidx[mid]] < base)
      a = mid + 1;
    else
      b = mid;
  }
  const uint32_t ns = A.n_stay[k], cap = A.cap[k];
  const uint64_t want = (hi - lo) + ns;
  const uint32_t total = (uint32_t)(want > cap ? cap : want);
  if (want > cap) atomicOr(A.err, kErrCapacity);
  RebinDest d;
  d.first = base - lo;
  d.split = a;
  d.end = base + total;
  d.below = (uint32_t)(a - lo);
  d.ns = ns;
  A.dest[k] = d;
}

// Cells of up to kStageSlots old slots are staged through LDS by the place
// pass; an output entry of kNoSlot is dropped (capacity overflow).
constexpr uint32_t kStageSlots = 384;
constexpr uint64_t kNoSlot = ~0ull;

// New slot of every list entry (by its sorted position j: its new cell's
// destination record gives it), ~0u when the entry is dropped (an
// admission that left again, or a slot past its new cell's capacity).
// Slots of the spatial mode fit 32 bits below ~0u. One thread per sorted
// entry; the writes scatter by list index, so that the place pass reads
// its movers' slots in list order.
constexpr uint32_t kNoSlot32 = 0xFFFFFFFFu;
__global__ __launch_bounds__(256) void k_rebin_slots(RebinArgs A) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.m) return;
  const uint32_t k = A.skey[j];
  uint32_t slot = kNoSlot32;
  if (k < A.n_cells) {
    const RebinDest d = A.dest[k];
    const uint64_t to = d.first + j + (j >= d.split ? d.ns : 0u);
    if (to < d.end) slot = (uint32_t)to;
  }
  A.slot[HCAO_IDX(A.sidx[j], A.m, A.err)] = slot;
}

__device__ __forceinline__ uint64_t entry_slot(const RebinArgs &A, uint64_t m) {
  const uint32_t v = A.slot[m];
  return v == kNoSlot32 ? kNoSlot : (uint64_t)v;
}

// one particle to its new slot with the step's move applied (the same
// arithmetic as the move pass)
__device__ __forceinline__ void copy_moved(const RebinArgs &A, uint64_t from, uint64_t to) {
  const State &s = A.src, &d = A.dst;
  const Vec3 v = load_vel(s, from);
  double vx = v.x, vy = v.y, vz = v.z;
  double x = s.px[from], y = s.py[from], z = s.pz[from];
  bool flip = false;
  move_particle(x, y, z, vx, vy, vz, A.dt, A.len, A.periodic, A.open, flip);
  store_vel(d, to, vx, vy, vz);
  d.sp[to] = s.sp[from];
  copy_levels(s, from, d, to);
  if (s.rot) d.rot[to] = s.rot[from];
  d.px[to] = x;
  d.py[to] = y;
  d.pz[to] = z;
}

// The place pass, pushed from the old cells: one workgroup per old cell j
// writes each of its particles, moved over the step, to its slot in the
// new cell. The order in
// every new cell is that of a stable sort of all particles by new cell:
// movers from slots below off[k], k's stayers, the other movers, the
// admissions (k_rebin_admit). The movers from j into one new cell hold
// consecutive sorted positions, hence consecutive new slots; the workgroup
// ranks its movers by new slot, so that its writes form runs. A cell of up
// to kStageSlots old slots is read whole, in slot order, into registers
// (issued first, so that the loads overlap the ranking) and then LDS, and
// written from there in output order; its level rows (4 to 32 bytes each)
// follow as one run of dwords, read in order and written dword by dword in
// output order. Larger cells copy each particle directly. The old count is read before the new one is written (only this
// workgroup touches cnt[j]). Workgroups go to the eight XCDs in turn, so
// the grid (a multiple of 8) gives each XCD one contiguous range of cells:
// movers go to neighbouring cells, whose lines are then in the same L2.
__global__ __launch_bounds__(256) void k_rebin_push(RebinArgs A) {
  constexpr uint32_t kPer = (kStageSlots + 255u) / 256u;  // staged slots per thread
  constexpr uint32_t kPerL = (kStageSlots * (kMaxModes / 2) + 255u) / 256u;  // staged level dwords per thread
  // positions (rows 0-2) and velocities (rows 3-5: bits of a double, or of
  // a float); mover new slots while ranking, level rows after the fields
  __shared__ uint64_t s_pv[6][kStageSlots];
  static_assert(kStageSlots * (kMaxModes / 2) * 4 <= sizeof(s_pv), "level rows must fit the staging rows");
  uint64_t(*s_pos)[kStageSlots] = s_pv;
  uint64_t(*s_vel)[kStageSlots] = s_pv + 3;
  __shared__ uint64_t s_rot[kStageSlots];
  __shared__ uint64_t s_to[kStageSlots];
  __shared__ uint16_t s_src[kStageSlots], s_msrc[kStageSlots];
  __shared__ uint8_t s_sp[kStageSlots];
  const uint32_t per_xcd = gridDim.x >> 3;
  const uint32_t j = (blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
  if (j >= A.n_cells) return;
  const uint32_t tid = threadIdx.x;
  const uint64_t base = A.off[j], mb = A.mbase[j];
  const uint32_t ns = A.n_stay[j], nm = (uint32_t)(A.mbase[j + 1] - mb), n_old = A.cnt[j];
  const RebinDest own = A.dest[j];
  const uint32_t n_out = ns + nm;
  const State &S = A.src, &D = A.dst;
  if (n_old > kStageSlots) {
    for (uint32_t t = tid; t < n_out; t += blockDim.x) {
      uint64_t from, to;
      if (t < ns) {
        from = base + A.list[base + t];
        to = base + own.below + t;
        if (to >= own.end) continue;
      } else {
        const uint64_t m = HCAO_IDX(mb + (t - ns), A.m, A.err);
        from = A.mslot[m];
        to = entry_slot(A, m);
        if (to == kNoSlot) continue;
      }
      copy_moved(A, HCAO_IDX(from, S.n_slots, A.err), HCAO_IDX(to, D.n_slots, A.err));
    }
  } else {
    const bool f32 = S.fx != nullptr, rot = S.rot != nullptr;
    uint64_t rp[kPer][3], rv[kPer][3], rr[kPer];
    uint8_t rs[kPer];
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint32_t i = tid + 256u * q;
      if (i < n_old) {
        const uint64_t g = base + i;
        rp[q][0] = reinterpret_cast<const uint64_t *>(S.px)[g];
        rp[q][1] = reinterpret_cast<const uint64_t *>(S.py)[g];
        rp[q][2] = reinterpret_cast<const uint64_t *>(S.pz)[g];
        if (f32) {
          rv[q][0] = reinterpret_cast<const uint32_t *>(S.fx)[g];
          rv[q][1] = reinterpret_cast<const uint32_t *>(S.fy)[g];
          rv[q][2] = reinterpret_cast<const uint32_t *>(S.fz)[g];
        } else {
          rv[q][0] = reinterpret_cast<const uint64_t *>(S.vx)[g];
          rv[q][1] = reinterpret_cast<const uint64_t *>(S.vy)[g];
          rv[q][2] = reinterpret_cast<const uint64_t *>(S.vz)[g];
        }
        rr[q] = rot ? reinterpret_cast<const uint64_t *>(S.rot)[g] : 0u;
        rs[q] = S.sp[g];
      }
    }
    // the step's move (positions, and velocities a specular face reversed);
    // a particle that left through an open face is in no list
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      if (tid + 256u * q < n_old) {
        double x = __longlong_as_double((long long)rp[q][0]), y = __longlong_as_double((long long)rp[q][1]),
               z = __longlong_as_double((long long)rp[q][2]);
        double vx, vy, vz;
        if (f32) {
          vx = (double)__uint_as_float((uint32_t)rv[q][0]);
          vy = (double)__uint_as_float((uint32_t)rv[q][1]);
          vz = (double)__uint_as_float((uint32_t)rv[q][2]);
        } else {
          vx = __longlong_as_double((long long)rv[q][0]);
          vy = __longlong_as_double((long long)rv[q][1]);
          vz = __longlong_as_double((long long)rv[q][2]);
        }
        bool flip = false;
        move_particle(x, y, z, vx, vy, vz, A.dt, A.len, A.periodic, A.open, flip);
        rp[q][0] = (uint64_t)__double_as_longlong(x);
        rp[q][1] = (uint64_t)__double_as_longlong(y);
        rp[q][2] = (uint64_t)__double_as_longlong(z);
        if (flip) {
          if (f32) {
            rv[q][0] = __float_as_uint((float)vx);
            rv[q][1] = __float_as_uint((float)vy);
            rv[q][2] = __float_as_uint((float)vz);
          } else {
            rv[q][0] = (uint64_t)__double_as_longlong(vx);
            rv[q][1] = (uint64_t)__double_as_longlong(vy);
            rv[q][2] = (uint64_t)__double_as_longlong(vz);
          }
        }
      }
    }
    // the cell's level rows as one run of n_old * L dwords, loaded in order
    // (lane t takes dwords t, t + 256, ...)
    const uint32_t L = S.lrow / 2u, n_lv = n_old * L;
    const uint32_t *lsrc = reinterpret_cast<const uint32_t *>(S.lvl) + base * L;
    uint32_t rl[kPerL];
#pragma unroll
    for (uint32_t q = 0; q < kPerL; ++q) {
      const uint32_t f = tid + 256u * q;
      rl[q] = f < n_lv ? lsrc[f] : 0u;
    }
    // output entries: the stayers in slot order, then the movers ranked by
    // new slot (dropped movers, kNoSlot, last)
    for (uint32_t t = tid; t < ns; t += blockDim.x) {
      const uint64_t to = base + own.below + t;
      s_src[t] = (uint16_t)A.list[base + t];
      s_to[t] = to < own.end ? HCAO_IDX(to, D.n_slots, A.err) : kNoSlot;
    }
    uint64_t *s_mto = s_pos[0];
    for (uint32_t r = tid; r < nm; r += blockDim.x) {
      const uint64_t m = HCAO_IDX(mb + r, A.m, A.err);
      const uint64_t to = entry_slot(A, m);
      s_mto[r] = to == kNoSlot ? kNoSlot : HCAO_IDX(to, D.n_slots, A.err);
      s_msrc[r] = (uint16_t)(A.mslot[m] - base);
    }
    __syncthreads();
    for (uint32_t r = tid; r < nm; r += blockDim.x) {
      const uint64_t me = s_mto[r];
      uint32_t rank = 0;
      for (uint32_t u = 0; u < nm; ++u) {
        const uint64_t o = s_mto[u];
        rank += (o < me || (o == me && u < r)) ? 1u : 0u;
      }
      s_src[ns + rank] = s_msrc[r];
      s_to[ns + rank] = me;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint32_t i = tid + 256u * q;
      if (i < n_old) {
        for (int a = 0; a < 3; ++a) {
          s_pos[a][i] = rp[q][a];
          s_vel[a][i] = rv[q][a];
        }
        s_rot[i] = rr[q];
        s_sp[i] = rs[q];
      }
    }
    __syncthreads();
    for (uint32_t w = tid; w < n_out; w += blockDim.x) {
      const uint64_t to = s_to[w];
      if (to == kNoSlot) continue;
      const uint32_t i = s_src[w];
      reinterpret_cast<uint64_t *>(D.px)[to] = s_pos[0][i];
      reinterpret_cast<uint64_t *>(D.py)[to] = s_pos[1][i];
      reinterpret_cast<uint64_t *>(D.pz)[to] = s_pos[2][i];
      if (f32) {
        reinterpret_cast<uint32_t *>(D.fx)[to] = (uint32_t)s_vel[0][i];
        reinterpret_cast<uint32_t *>(D.fy)[to] = (uint32_t)s_vel[1][i];
        reinterpret_cast<uint32_t *>(D.fz)[to] = (uint32_t)s_vel[2][i];
      } else {
        reinterpret_cast<uint64_t *>(D.vx)[to] = s_vel[0][i];
        reinterpret_cast<uint64_t *>(D.vy)[to] = s_vel[1][i];
        reinterpret_cast<uint64_t *>(D.vz)[to] = s_vel[2][i];
      }
      if (rot) reinterpret_cast<uint64_t *>(D.rot)[to] = s_rot[i];
      D.sp[to] = s_sp[i];
    }
    // level rows through LDS (over the staged positions and velocities, read
    // for the last time above), written dword by dword in output order, so
    // that reads and writes of a wave are runs of consecutive dwords:
    // output dword f is dword f mod L of entry f / L (exact as f * ceil(2^16
    // / L) >> 16 for f <= 3072, L <= 8)
    __syncthreads();
    uint32_t *s_lv = reinterpret_cast<uint32_t *>(&s_pv[0][0]);
#pragma unroll
    for (uint32_t q = 0; q < kPerL; ++q) {
      const uint32_t f = tid + 256u * q;
      if (f < n_lv) s_lv[f] = rl[q];
    }
    __syncthreads();
    uint32_t *ldst = reinterpret_cast<uint32_t *>(D.lvl);
    const uint32_t inv = (65536u + L - 1u) / L;
    for (uint32_t f = tid; f < n_out * L; f += blockDim.x) {
      const uint32_t w = (f * inv) >> 16, d = f - w * L;
      const uint64_t to = s_to[w];
      if (to != kNoSlot) ldst[to * L + d] = s_lv[(uint32_t)s_src[w] * L + d];
    }
  }
  __syncthreads();  // every wave has read the old count
  if (tid == 0) A.cnt[j] = (uint32_t)(own.end - base);
}

// the admissions of the step (list entries m_real .. m - 1, staged in ins in
// the order made): one thread each; one that left again (key n_cells) is
// dropped
__global__ __launch_bounds__(256) void k_rebin_admit(RebinArgs A) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t m = A.m_real + i;
  if (m >= A.m) return;
  const uint64_t to = entry_slot(A, m);
  if (to == kNoSlot) return;
  copy_particle(A.ins, A.dst, HCAO_IDX(A.mslot[m] - A.tot, A.ins.n_slots, A.err), HCAO_IDX(to, A.dst.n_slots, A.err),
                A.mm);
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers (host side)
// ---------------------------------------------------------------------------
size_t step_lds_bytes(const Tables &T, uint32_t max_cells, int block) {
  const uint32_t ns = T.n_species, nr = T.n_reactions;
  size_t b = sizeof(SpeciesTab) * ns + sizeof(PairTab) * ns * ns + sizeof(ReactionTab) * nr + 8 * (size_t)T.n_levels;
  b += sizeof(CellHdr) * max_cells + 2 * 8 * (size_t)(8 + nr) * max_cells;
  b += (size_t)2 * (2 + 3) * (T.max_modes ? T.max_modes : 1) * block;
  return (b + 15) & ~(size_t)15;
}

template <bool MIX, int EX>
static hipError_t launch_step_t(const StepArgs &a, size_t lds, int block, uint32_t n_groups, hipStream_t s) {
  switch (block) {
    case 64: hipLaunchKernelGGL((k_step<64, MIX, EX>), dim3(n_groups), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((k_step<128, MIX, EX>), dim3(n_groups), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((k_step<256, MIX, EX>), dim3(n_groups), dim3(256), lds, s, a); break;
    case 512: hipLaunchKernelGGL((k_step<512, MIX, EX>), dim3(n_groups), dim3(512), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// level 0: the collision step; 1: and positions (spatial mode); 2: and the
// exact sampler and rotors (positions included)
hipError_t launch_step(const StepArgs &a, size_t lds, int block, bool mixed, int level, uint32_t n_groups,
                       hipStream_t s) {
  if (n_groups == 0) return hipSuccess;
  if (level >= 2)
    return mixed ? launch_step_t<true, 2>(a, lds, block, n_groups, s)
                 : launch_step_t<false, 2>(a, lds, block, n_groups, s);
  if (level == 1)
    return mixed ? launch_step_t<true, 1>(a, lds, block, n_groups, s)
                 : launch_step_t<false, 1>(a, lds, block, n_groups, s);
  return mixed ? launch_step_t<true, 0>(a, lds, block, n_groups, s)
               : launch_step_t<false, 0>(a, lds, block, n_groups, s);
}

// Fixed device array for the allocation-free step (hcao_step_static): the
// work lists, pair flags, pair energy defects and products staging of one
// step call. Host code never passes the array's name to a kernel: it uses
// the device address that static_scratch_address() returns for the current
// device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch_address(void **ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

hipError_t launch_advance(uint32_t *step, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, step, n);
  return hipGetLastError();
}

// the dynamic LDS limit of every k_step instantiation the launcher can pick
// (block sizes 64..512, both precisions, levels 0..2)
template <bool MIX, int EX>
static hipError_t set_lds_limit_level(int bytes) {
  hipError_t e = hipSuccess;
  const void *fns[] = {(const void *)k_step<64, MIX, EX>, (const void *)k_step<128, MIX, EX>,
                       (const void *)k_step<256, MIX, EX>, (const void *)k_step<512, MIX, EX>};
  for (const void *f : fns) {
    const hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (r != hipSuccess) e = r;
  }
  return e;
}

hipError_t set_step_lds_limit(size_t bytes) {
  const int b = (int)bytes;
  const hipError_t r[] = {set_lds_limit_level<false, 0>(b), set_lds_limit_level<true, 0>(b),
                          set_lds_limit_level<false, 1>(b), set_lds_limit_level<true, 1>(b),
                          set_lds_limit_level<false, 2>(b), set_lds_limit_level<true, 2>(b)};
  for (hipError_t e : r)
    if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_init(const Tables *tab, const double *lev, const State &st, const uint64_t *off,
                       const uint32_t *counts, const double *tt, const double *tv, uint64_t seed, uint32_t n_cells,
                       const uint32_t grid[3], const double len[3], hipStream_t s) {
  InitArgs a{tab, lev, st, off, counts, tt, tv, seed, n_cells, grid[0], grid[1], grid[2], {len[0], len[1], len[2]}};
  hipLaunchKernelGGL(k_init, dim3(n_cells), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cell_init(const Tables *tab, const State &st, const CellArrays &cells, uint32_t n_cells,
                            hipStream_t s) {
  CellInitArgs a{tab, st, cells};
  hipLaunchKernelGGL(k_cell_init, dim3(n_cells), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_moments(const Tables *tab, const double *lev, const State &st, const uint64_t *off,
                          const uint32_t *cnt, double *out, uint32_t n_cells, hipStream_t s) {
  MomentArgs a{tab, lev, st, off, cnt, out};
  hipLaunchKernelGGL(k_moments, dim3(n_cells), dim3(256), 0, s, a);
  return hipGetLastError();
}

uint64_t scan_tmp_entries(uint64_t n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

// exclusive scan; tmp holds scan_tmp_entries(n) entries (at most
// kScanChunk chunks, i.e. n <= 2^28)
hipError_t launch_scan_u32(const uint32_t *in, uint64_t *out, uint64_t n, uint64_t *tmp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t nb = (n + kScanChunk - 1) / kScanChunk;
  if (nb > kScanChunk) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_chunk, dim3((unsigned)nb), dim3(1024), 0, s, in, out, n, tmp);
  if (nb > 1) {
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, tmp);
  }
  return hipGetLastError();
}

hipError_t launch_load_check(const Tables *tab, const uint32_t *cell, const uint8_t *sp, const double *vel,
                             const uint16_t *lvl, uint64_t n, uint32_t n_cells, uint32_t *count, uint32_t *err,
                             hipStream_t s) {
  LoadArgs a{tab, cell, sp, vel, lvl, n, n_cells, count, err};
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_load_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Stable sort of (key, index) by the low key_bits bits of the key; buffers
// of n entries each, hist and offs of sort_hist_entries(n) entries (u32,
// u64). The passes take digits of equal width up to 9 bits: one pass up to
// 9 bits, two up to 18, three up to 27 (19 bits: three of 7; two of 10 cost
// more in their larger histogram scans). Result in
// keys/idx or the tmp buffers (ping-pong handled here; returns which buffer
// holds the result).
hipError_t launch_sort(uint32_t *keys, uint32_t *idx, uint32_t *keys_tmp, uint32_t *idx_tmp, uint32_t *hist,
                       uint64_t *offs, uint64_t *scan_tmp, uint64_t n, uint32_t key_bits, hipStream_t s,
                       bool &result_in_tmp) {
  result_in_tmp = false;
  if (n == 0) return hipSuccess;
  const uint32_t tiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx, n);
  uint32_t *kin = keys, *iin = idx, *kout = keys_tmp, *iout = idx_tmp;
  if (key_bits > 32) return hipErrorInvalidValue;
  const uint32_t passes = (key_bits + kSortMaxBits - 1) / kSortMaxBits;
  const uint32_t bits = passes ? (key_bits + passes - 1) / passes : 0;
  for (uint32_t shift = 0; shift < key_bits; shift += bits) {
    hipLaunchKernelGGL(k_sort_hist, dim3(tiles), dim3(kSortBlock), 0, s, kin, n, shift, bits, hist, tiles);
    const hipError_t e = launch_scan_u32(hist, offs, (uint64_t)(1u << bits) * tiles, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_scatter, dim3(tiles), dim3(kSortBlock), 0, s, kin, iin, kout, iout, n, shift, bits,
                       offs, tiles);
    uint32_t *tk = kin, *ti = iin;
    kin = kout;
    iin = iout;
    kout = tk;
    iout = ti;
    result_in_tmp = !result_in_tmp;
  }
  return hipGetLastError();
}

uint64_t sort_tiles(uint64_t n) { return (n + kSortTile - 1) / kSortTile; }
uint64_t sort_hist_entries(uint64_t n) { return (uint64_t)kSortMaxBins * sort_tiles(n); }

hipError_t launch_move(const MoveArgs &a, hipStream_t s) {
  if (a.n_cells == 0) return hipSuccess;
  if (!a.off || !a.cnt || !a.cap || !a.key || !a.list || !a.n_stay || !a.n_move || !a.st.px || !a.st.py || !a.st.pz)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_move, dim3(a.n_cells), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_list_movers(const RebinArgs &a, hipStream_t s) {
  if (a.n_cells == 0 || a.m == 0) return hipSuccess;
  if (!a.off || !a.cap || !a.key || !a.list || !a.n_move || !a.mbase || !a.mkey || !a.mslot)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_list_movers, dim3((a.n_cells + 3u) / 4u), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_inflow_count(const InflowArgs &a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.face_base[6] * a.n_species;
  if (n == 0) return hipSuccess;
  if (!a.tab || !a.weight || !a.rem || !a.count || !a.err) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_inflow_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_inflow_make(const InflowArgs &a, hipStream_t s) {
  const uint64_t n = a.n_ins;
  if (n == 0 || a.face_base[6] == 0 || a.n_species == 0) return hipSuccess;
  if (!a.tab || !a.lev || !a.count || !a.ibase || !a.mbase || !a.mkey || !a.mslot || !a.flux || !a.err ||
      !a.ins.sp || !a.ins.lvl || !a.ins.px || !a.ins.py || !a.ins.pz || (!a.ins.vx && !a.ins.fx))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_inflow_make, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// run starts of the sorted list, the new cells' counts and destinations,
// every list entry's new slot, then the place pass from the old cells and
// the admissions
hipError_t launch_rebin_place(const RebinArgs &a, hipStream_t s) {
  if (a.n_cells == 0) return hipSuccess;
  if (!a.off || !a.cap || !a.list || !a.n_stay || !a.mbase || !a.packed || !a.dest || !a.cnt || !a.err ||
      a.m_real > a.m || (a.m && (!a.skey || !a.sidx || !a.mslot || !a.slot)))
    return hipErrorInvalidValue;
  if (a.m)
    hipLaunchKernelGGL(k_run_starts, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, s, a.skey, a.m, a.n_cells,
                       a.packed);
  hipLaunchKernelGGL(k_rebin_cells, dim3((a.n_cells + 255u) / 256u), dim3(256), 0, s, a);
  if (a.m) hipLaunchKernelGGL(k_rebin_slots, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_rebin_push, dim3(((a.n_cells + 7u) / 8u) * 8u), dim3(256), 0, s, a);
  if (a.m > a.m_real)
    hipLaunchKernelGGL(k_rebin_admit, dim3((unsigned)((a.m - a.m_real + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rec_enum(const RecEnumArgs &a, bool write, hipStream_t s) {
  if (a.n_prefix == 0) return hipSuccess;
  const dim3 grid((unsigned)((a.n_prefix + 255) / 256));
  if (write)
    hipLaunchKernelGGL(k_rec_enum<true>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_rec_enum<false>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rec_sum(const RecSumArgs &a, uint32_t n_t, size_t lds, hipStream_t s) {
  if (n_t == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rec_sum, dim3(n_t), dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_place(const Tables *tab, const uint32_t *sorted_cell, const uint32_t *sorted_idx,
                        const uint64_t *packed_start, const uint64_t *off, const uint8_t *sp, const double *vel,
                        const uint16_t *lvl, const double *rot, const double *pos, const State &st, uint64_t n,
                        hipStream_t s) {
  PlaceArgs a{tab, sorted_cell, sorted_idx, packed_start, off, sp, vel, lvl, rot, pos, st, n};
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_load_place, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hcao
