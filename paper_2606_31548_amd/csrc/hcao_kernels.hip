// hcao_kernels.hip -- gfx950 kernels of the HCAO DSMC collision step.
//
// One workgroup owns one reservoir cell for a whole step: it stages the
// cell's particles in LDS (or works in place in HBM for cells too large for
// LDS), forms NTC candidate pairs from a keyed permutation, tests them with
// the VHS acceptance, runs the reaction decision / Larsen-Borgnakke
// relaxation / isotropic scattering of each accepted pair in its lane,
// appends reaction products in pair order with a block scan, and writes the
// tile back with coalesced stores. Cells never exchange particles, so the
// launch needs no inter-workgroup communication and the result does not
// depend on the launch shape.
//
// Arithmetic is IEEE fp64 without contraction (built with -ffp-contract=off);
// log/exp are the library's own fixed-sequence versions, so that every
// decision is reproducible bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hcao_tables.h"

namespace hcao {
namespace {

constexpr double kBoltz = 1.380649e-23;
constexpr uint32_t kNone = 255u;

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
    const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
    const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
    const uint32_t y0 = hi1 ^ x1 ^ k0;
    const uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
}

// A stream (seed; pair, cell, step): each Philox block yields two 64-bit
// draws, low word first.
struct Rng {
  uint32_t k0, k1, pair, cell, step, block;
  uint32_t w0, w1, w2, w3;
  uint32_t used;

  __device__ __forceinline__ void open(uint64_t seed, uint32_t p, uint32_t c, uint32_t s) {
    k0 = (uint32_t)seed;
    k1 = (uint32_t)(seed >> 32);
    pair = p;
    cell = c;
    step = s;
    block = 0;
    used = 4;
  }
  __device__ __forceinline__ uint64_t next64() {
    if (used >= 4) {
      uint32_t x0 = block, x1 = pair, x2 = cell, x3 = step;
      philox10(k0, k1, x0, x1, x2, x3);
      w0 = x0;
      w1 = x1;
      w2 = x2;
      w3 = x3;
      block += 1;
      used = 0;
    }
    uint64_t r = (used == 0) ? (((uint64_t)w1 << 32) | w0) : (((uint64_t)w3 << 32) | w2);
    used += 2;
    return r;
  }
  __device__ __forceinline__ double uniform() { return (double)(next64() >> 11) * 0x1p-53; }
};

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

// ---------------------------------------------------------------------------
// keyed permutation of [0, n): 10-round Feistel network on 2b bits with
// cycle walking (Luby-Rackoff; Black-Rogaway)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t feistel_f(uint32_t r, uint32_t key, uint32_t mask) {
  uint32_t h = (r ^ key) * 0x9E3779B1u;
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  return h & mask;
}

struct Perm {
  uint32_t n, b, mask;
  uint32_t k[10];
  __device__ __forceinline__ uint32_t once(uint32_t x) const {
    uint32_t l = x >> b, r = x & mask;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
      const uint32_t nr = l ^ feistel_f(r, k[i], mask);
      l = r;
      r = nr;
    }
    return (l << b) | r;
  }
  __device__ __forceinline__ uint32_t operator()(uint32_t i) const {
    uint32_t y = once(i);
    while (y >= n) y = once(y);
    return y;
  }
};

__device__ __forceinline__ void make_perm(Perm &P, uint32_t n, uint64_t seed, uint32_t cell, uint32_t step) {
  P.n = n;
  uint32_t b = 1;
  while ((1ull << (2 * b)) < (unsigned long long)n) ++b;
  P.b = b;
  P.mask = (1u << b) - 1u;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  uint32_t w[12];
#pragma unroll
  for (uint32_t blk = 0; blk < 3; ++blk) {
    uint32_t x0 = blk, x1 = 0xFFFFFFFFu, x2 = cell, x3 = step;
    philox10(k0, k1, x0, x1, x2, x3);
    w[4 * blk] = x0;
    w[4 * blk + 1] = x1;
    w[4 * blk + 2] = x2;
    w[4 * blk + 3] = x3;
  }
#pragma unroll
  for (int i = 0; i < 10; ++i) P.k[i] = w[i];
}

// ---------------------------------------------------------------------------
// particle views
// ---------------------------------------------------------------------------
struct View {
  double *vx, *vy, *vz;
  uint8_t *sp;
  uint16_t *lvl;
  uint64_t stride;
};

struct Ctx {
  const Tables *T;
  const double *lev;
  unsigned long long *ctr;  // LDS counters
  uint16_t *scr;            // per-lane scratch, [2 * max_modes][block]
  uint32_t lane, block;
};

__device__ __forceinline__ double mode_energy(const SpeciesTab &S, const double *lev, uint32_t m, uint32_t i) {
  if (m < S.n_bend) return ((double)i + 0.5) * S.kt[m];
  return lev[S.lev_off[m] + i];
}

__device__ __forceinline__ double vib_energy(const SpeciesTab &S, const double *lev, const uint16_t *lv,
                                             uint64_t stride) {
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
  const double *L = lev + S.lev_off[m];
  const uint32_t idiss = S.idiss[m];
  uint32_t top = 0;
  while (top < idiss && L[top + 1] < e) ++top;
  return top;
}

__device__ __forceinline__ uint32_t pick_level(uint32_t top, double u) {
  const double span = (double)top + 1.0;
  uint32_t i = (uint32_t)floor(u * span);
  return i > top ? top : i;
}

// Larsen-Borgnakke relaxation of one molecule (levels at lv[m * stride]);
// e_tr is the pair's translational energy on entry and exit.
__device__ uint32_t relax(const Ctx &C, const SpeciesTab &S, uint16_t *lv, uint64_t stride, double &e_tr, double q,
                          Rng &rng, bool &capped) {
  uint32_t trials = 0;
  capped = false;
  const uint32_t nm = S.n_modes;
  if (S.sampler == HCAO_SAMPLER_JOINT) {
    const double e_coll = e_tr + vib_energy(S, C.lev, lv, stride);
    const double denom = e_coll - S.zpe;
    if (!(denom > 0.0)) return 0;
    uint16_t *tops = C.scr + C.lane;
    uint16_t *cand = C.scr + (size_t)nm * C.block + C.lane;
    for (uint32_t m = 0; m < nm; ++m) tops[m * C.block] = (uint16_t)mode_top(S, C.lev, m, e_coll);
    for (;;) {
      ++trials;
      double sum = 0.0;
      for (uint32_t m = 0; m < nm; ++m) {
        const uint32_t i = pick_level(tops[m * C.block], rng.uniform());
        cand[m * C.block] = (uint16_t)i;
        sum = sum + mode_energy(S, C.lev, m, i);
      }
      const double ua = rng.uniform();
      const bool ok = (sum < e_coll) && (ua < dpow((e_coll - sum) / denom, q));
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
  double et = e_tr;
  for (uint32_t m = 0; m < nm; ++m) {
    const double ec = et + mode_energy(S, C.lev, m, lv[m * stride]);
    const double den = ec - mode_energy(S, C.lev, m, 0);
    if (!(den > 0.0)) continue;
    const uint32_t top = mode_top(S, C.lev, m, ec);
    for (;;) {
      ++trials;
      const uint32_t i = pick_level(top, rng.uniform());
      const double ei = mode_energy(S, C.lev, m, i);
      const double ua = rng.uniform();
      const bool ok = (ei < ec) && (ua < dpow((ec - ei) / den, q));
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
__device__ __forceinline__ void unit_vector(Rng &rng, double &nx, double &ny, double &nz) {
  double x, y, s;
  for (;;) {
    x = 2.0 * rng.uniform() - 1.0;
    y = 2.0 * rng.uniform() - 1.0;
    s = x * x + y * y;
    if (s < 1.0) break;
  }
  const double f = 2.0 * sqrt(1.0 - s);
  nx = x * f;
  ny = y * f;
  nz = 1.0 - 2.0 * s;
}

struct Vec3 {
  double x, y, z;
};

__device__ __forceinline__ Vec3 com(const PairTab &P, Vec3 a, Vec3 b) {
  return Vec3{(P.m_a * a.x + P.m_b * b.x) / P.msum, (P.m_a * a.y + P.m_b * b.y) / P.msum,
              (P.m_a * a.z + P.m_b * b.z) / P.msum};
}

// two bodies about the centre-of-mass velocity with relative energy e
__device__ __forceinline__ void split(const PairTab &P, Vec3 vcm, double e, Rng &rng, Vec3 &va, Vec3 &vb) {
  const double g = sqrt((2.0 * e) / P.mr);
  double nx, ny, nz;
  unit_vector(rng, nx, ny, nz);
  const double ga = P.wa * g, gb = P.wb * g;
  va = Vec3{vcm.x + ga * nx, vcm.y + ga * ny, vcm.z + ga * nz};
  vb = Vec3{vcm.x - gb * nx, vcm.y - gb * ny, vcm.z - gb * nz};
}

__device__ __forceinline__ Vec3 load_v(const View &V, uint32_t i) { return Vec3{V.vx[i], V.vy[i], V.vz[i]}; }
__device__ __forceinline__ void store_v(const View &V, uint32_t i, Vec3 v) {
  V.vx[i] = v.x;
  V.vy[i] = v.y;
  V.vz[i] = v.z;
}

__device__ __forceinline__ void zero_levels(uint16_t *lv, uint64_t stride, uint32_t mm) {
  for (uint32_t m = 0; m < mm; ++m) lv[m * stride] = 0;
}

struct Channel {
  int32_t rx, side, mode;
};

// One accepted pair (slots p, q of the tile): reaction decision and
// application, or relaxation of both molecules, then scattering.
// A dissociation product is written to nb at index k.
__device__ void collide(const Ctx &C, const View &t, uint32_t p, uint32_t q, double g2, Rng &rng, const View &nb,
                        uint32_t k) {
  const Tables &T = *C.T;
  const uint32_t mm = T.max_modes;
  const uint32_t slot[2] = {p, q};
  const uint32_t spp = t.sp[p], spq = t.sp[q];
  const uint32_t sps[2] = {spp, spq};
  const PairTab &PP = T.pr[spp][spq];
  double e_tr = PP.hm * g2;
  const double ev0 = vib_energy(T.sp[spp], C.lev, t.lvl + p, t.stride);
  const double ev1 = vib_energy(T.sp[spq], C.lev, t.lvl + q, t.stride);

  // --- reaction decision: dissociation channels, then exchange channels ---
  uint32_t nch = 0;
  double total = 0.0;
  Channel first{-1, 0, 0}, last{-1, 0, 0};
  uint64_t steric_ok = 0;  // outcome of each matched exchange draw, in order
  uint32_t n_exch = 0;
  for (uint32_t side = 0; side < 2; ++side) {
    const uint32_t A = sps[side];
    const double evA = side ? ev1 : ev0;
    for (uint32_t r = 0; r < T.n_reactions; ++r) {
      const ReactionTab &R = T.rx[r];
      if (R.kind != HCAO_RX_DISSOCIATION || (uint32_t)R.a != A) continue;
      const SpeciesTab &SA = T.sp[A];
      const uint32_t nst = SA.n_modes - SA.n_bend;
      for (uint32_t j = 0; j < nst; ++j) {
        if (!((R.mask >> j) & 1ull)) continue;
        const uint32_t m = SA.n_bend + j;
        const double ecoll = ((e_tr + evA) - R.zsum) + C.lev[SA.lev_off[m]];
        const double eex = ecoll - SA.de[m];
        const double pool = (e_tr + evA) - R.dh;
        const double left = (pool - T.sp[R.c].zpe) - T.sp[R.d].zpe;
        if (eex > 0.0 && left > 0.0 && nch < (uint32_t)kMaxChannels) {
          const Channel ch{(int32_t)r, (int32_t)side, (int32_t)m};
          if (nch == 0) first = ch;
          last = ch;
          total = total + eex;
          ++nch;
        }
      }
    }
  }
  for (uint32_t side = 0; side < 2; ++side) {
    const uint32_t A = sps[side], B = sps[1 - side];
    const double evA = side ? ev1 : ev0, evB = side ? ev0 : ev1;
    const uint32_t sA = slot[side];
    for (uint32_t r = 0; r < T.n_reactions; ++r) {
      const ReactionTab &R = T.rx[r];
      if (R.kind != HCAO_RX_EXCHANGE || (uint32_t)R.a != A || (uint32_t)R.b != B) continue;
      const double us = rng.uniform();
      const SpeciesTab &SA = T.sp[A];
      double ecoll = e_tr;
      for (uint32_t m = 0; m < SA.n_modes; ++m)
        ecoll = ecoll + R.alpha[m] * mode_energy(SA, C.lev, m, t.lvl[m * t.stride + sA]);
      const double eex = ecoll - R.ea;
      const double pool = ((e_tr + evA) + evB) - R.dh;
      const double left = (pool - T.sp[R.c].zpe) - T.sp[R.d].zpe;
      const bool st_ok = us < R.steric;
      if (st_ok && n_exch < 64) steric_ok |= (1ull << n_exch);
      ++n_exch;
      if (st_ok && eex > 0.0 && left > 0.0 && nch < (uint32_t)kMaxChannels) {
        const Channel ch{(int32_t)r, (int32_t)side, -1};
        if (nch == 0) first = ch;
        last = ch;
        total = total + eex;
        ++nch;
      }
    }
  }

  if (nch > 0) {
    Channel pick = first;
    if (nch > 1) {
      // one draw over the open channels weighted by excess energy; the
      // channels are enumerated again in the same order
      const double target = rng.uniform() * total;
      double cum = 0.0;
      uint32_t seen = 0, ex_i = 0;
      bool found = false;
      pick = last;
      for (uint32_t side = 0; side < 2 && !found; ++side) {
        const uint32_t A = sps[side];
        const double evA = side ? ev1 : ev0;
        for (uint32_t r = 0; r < T.n_reactions && !found; ++r) {
          const ReactionTab &R = T.rx[r];
          if (R.kind != HCAO_RX_DISSOCIATION || (uint32_t)R.a != A) continue;
          const SpeciesTab &SA = T.sp[A];
          const uint32_t nst = SA.n_modes - SA.n_bend;
          for (uint32_t j = 0; j < nst && !found; ++j) {
            if (!((R.mask >> j) & 1ull)) continue;
            const uint32_t m = SA.n_bend + j;
            const double ecoll = ((e_tr + evA) - R.zsum) + C.lev[SA.lev_off[m]];
            const double eex = ecoll - SA.de[m];
            const double pool = (e_tr + evA) - R.dh;
            const double left = (pool - T.sp[R.c].zpe) - T.sp[R.d].zpe;
            if (eex > 0.0 && left > 0.0 && seen < (uint32_t)kMaxChannels) {
              ++seen;
              cum = cum + eex;
              if (target < cum) {
                pick = Channel{(int32_t)r, (int32_t)side, (int32_t)m};
                found = true;
              }
            }
          }
        }
      }
      for (uint32_t side = 0; side < 2 && !found; ++side) {
        const uint32_t A = sps[side], B = sps[1 - side];
        const double evA = side ? ev1 : ev0, evB = side ? ev0 : ev1;
        const uint32_t sA = slot[side];
        for (uint32_t r = 0; r < T.n_reactions && !found; ++r) {
          const ReactionTab &R = T.rx[r];
          if (R.kind != HCAO_RX_EXCHANGE || (uint32_t)R.a != A || (uint32_t)R.b != B) continue;
          const bool st_ok = ex_i < 64 ? ((steric_ok >> ex_i) & 1ull) != 0 : false;
          ++ex_i;
          const SpeciesTab &SA = T.sp[A];
          double ecoll = e_tr;
          for (uint32_t m = 0; m < SA.n_modes; ++m)
            ecoll = ecoll + R.alpha[m] * mode_energy(SA, C.lev, m, t.lvl[m * t.stride + sA]);
          const double eex = ecoll - R.ea;
          const double pool = ((e_tr + evA) + evB) - R.dh;
          const double left = (pool - T.sp[R.c].zpe) - T.sp[R.d].zpe;
          if (st_ok && eex > 0.0 && left > 0.0 && seen < (uint32_t)kMaxChannels) {
            ++seen;
            cum = cum + eex;
            if (target < cum) {
              pick = Channel{(int32_t)r, (int32_t)side, -1};
              found = true;
            }
          }
        }
      }
    }

    const ReactionTab &R = T.rx[pick.rx];
    const uint32_t a = (uint32_t)pick.side, b = 1 - a;
    const uint32_t sa = slot[a], sb = slot[b];
    const double eva = a ? ev1 : ev0, evb = a ? ev0 : ev1;
    uint64_t tr = 0;
    bool capped = false, c2 = false;
    if (R.kind == HCAO_RX_DISSOCIATION) {
      // A + M -> B + C + M: B takes A's slot, C is new
      const uint32_t spA = sps[a], spM = sps[b];
      const double pool = (e_tr + eva) - R.dh;
      double et = (pool - T.sp[R.c].zpe) - T.sp[R.d].zpe;
      uint16_t *lb = t.lvl + sa;
      uint16_t *lc = nb.lvl + k;
      zero_levels(lb, t.stride, mm);
      zero_levels(lc, nb.stride, mm);
      if (T.sp[R.c].n_modes > 0) tr += relax(C, T.sp[R.c], lb, t.stride, et, T.pr[R.c][spM].q, rng, capped);
      if (T.sp[R.d].n_modes > 0) {
        tr += relax(C, T.sp[R.d], lc, nb.stride, et, T.pr[R.d][spM].q, rng, c2);
        capped = capped || c2;
      }
      double beta;
      for (;;) {
        const double u1 = rng.uniform(), u2 = rng.uniform();
        if (u2 * 0.5 < sqrt(u1 * (1.0 - u1))) {
          beta = u1;
          break;
        }
      }
      const double ebc = beta * et;
      const double exm = et - ebc;
      const PairTab &PAM = T.pr[spA][spM];
      const Vec3 vcm = com(PAM, load_v(t, sa), load_v(t, sb));
      Vec3 vbc, vm, vbn, vcn;
      split(PAM, vcm, exm, rng, vbc, vm);
      split(T.pr[R.c][R.d], vbc, ebc, rng, vbn, vcn);
      store_v(t, sa, vbn);
      store_v(t, sb, vm);
      store_v(nb, k, vcn);
      t.sp[sa] = (uint8_t)R.c;
      nb.sp[k] = (uint8_t)R.d;
      atomicAdd(&C.ctr[HCAO_CTR_BIRTHS], 1ull);
    } else {
      // A + B -> C + D: C takes A's slot, D takes B's
      const uint32_t spA = sps[a], spB = sps[b];
      const double pool = ((e_tr + eva) + evb) - R.dh;
      double et = (pool - T.sp[R.c].zpe) - T.sp[R.d].zpe;
      uint16_t *lc = t.lvl + sa;
      uint16_t *ld = t.lvl + sb;
      zero_levels(lc, t.stride, mm);
      zero_levels(ld, t.stride, mm);
      const double qcd = T.pr[R.c][R.d].q;
      if (T.sp[R.c].n_modes > 0) tr += relax(C, T.sp[R.c], lc, t.stride, et, qcd, rng, capped);
      if (T.sp[R.d].n_modes > 0) {
        tr += relax(C, T.sp[R.d], ld, t.stride, et, qcd, rng, c2);
        capped = capped || c2;
      }
      const Vec3 vcm = com(T.pr[spA][spB], load_v(t, sa), load_v(t, sb));
      Vec3 vc, vd;
      split(T.pr[R.c][R.d], vcm, et, rng, vc, vd);
      store_v(t, sa, vc);
      store_v(t, sb, vd);
      t.sp[sa] = (uint8_t)R.c;
      t.sp[sb] = (uint8_t)R.d;
    }
    if (tr) atomicAdd(&C.ctr[HCAO_CTR_TRIALS], (unsigned long long)tr);
    if (capped) atomicAdd(&C.ctr[HCAO_CTR_CAPPED], 1ull);
    atomicAdd(&C.ctr[HCAO_CTR_REACTION0 + pick.rx], 1ull);
    return;
  }

  // --- no reaction: relax each molecule in turn, then scatter ---
  uint64_t tr = 0;
  uint32_t nrel = 0, ncap = 0;
  for (uint32_t x = 0; x < 2; ++x) {
    const SpeciesTab &S = T.sp[sps[x]];
    if (S.n_modes == 0) continue;
    const double u = rng.uniform();
    if (!(u < S.p_vib)) continue;
    bool capped = false;
    tr += relax(C, S, t.lvl + slot[x], t.stride, e_tr, PP.q, rng, capped);
    ++nrel;
    ncap += capped ? 1u : 0u;
  }
  if (tr) atomicAdd(&C.ctr[HCAO_CTR_TRIALS], (unsigned long long)tr);
  if (nrel) atomicAdd(&C.ctr[HCAO_CTR_RELAX], (unsigned long long)nrel);
  if (ncap) atomicAdd(&C.ctr[HCAO_CTR_CAPPED], (unsigned long long)ncap);
  const Vec3 vcm = com(PP, load_v(t, p), load_v(t, q));
  Vec3 va, vb;
  split(PP, vcm, e_tr, rng, va, vb);
  store_v(t, p, va);
  store_v(t, q, vb);
}

// block-wide exclusive scan of one value per thread (small blocks)
template <int BLOCK>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp, uint32_t &total) {
  const uint32_t tid = threadIdx.x;
  s_tmp[tid] = v;
  __syncthreads();
  for (uint32_t off = 1; off < BLOCK; off <<= 1) {
    const uint32_t add = tid >= off ? s_tmp[tid - off] : 0u;
    __syncthreads();
    s_tmp[tid] += add;
    __syncthreads();
  }
  total = s_tmp[BLOCK - 1];
  const uint32_t incl = s_tmp[tid];
  __syncthreads();
  return incl - v;
}

// LDS layout of one tile: [vx | vy | vz | nb.vx | nb.vy | nb.vz] doubles, then
// [lvl (mm x L) | nb.lvl (mm x L2) | scratch (2 mm x BLOCK)] u16, then
// [sp (L) | nb.sp (L2)] bytes.
__host__ __device__ inline size_t tile_lds_bytes(uint32_t L, uint32_t mm, uint32_t block) {
  const uint32_t L2 = L / 2 + 1;
  size_t bytes = (size_t)8 * (3 * L + 3 * L2);
  bytes += (size_t)2 * ((size_t)mm * L + (size_t)mm * L2 + (size_t)2 * mm * block);
  bytes += (size_t)L + L2;
  return (bytes + 15) & ~(size_t)15;
}

template <int BLOCK, bool kLds>
__global__ __launch_bounds__(BLOCK) void k_step(StepArgs A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ unsigned long long s_ctr[kNumCtr];
  __shared__ unsigned long long s_sgbits;
  __shared__ uint32_t s_scan[BLOCK];

  const uint32_t tid = threadIdx.x;
  const uint32_t c = A.cell_list ? A.cell_list[blockIdx.x] : blockIdx.x;
  const Tables *T = A.tab;
  const uint32_t mm = T->max_modes;
  const uint64_t base = A.cells.off[c];
  const uint32_t n = A.cells.cnt[c];
  const uint32_t cap = A.cells.cap[c];
  const double sgmax = A.cells.sgmax[c];

  // NTC candidate count: floor(1/2 N (N-1) F_N (sigma g)_max dt / V + remainder)
  const double x = 0.5 * (double)n * (double)(n - (n > 0 ? 1u : 0u)) * A.cells.weight[c] * sgmax * A.dt /
                       A.cells.volume[c] +
                   A.cells.rem[c];
  const double fl = floor(x);
  const double rem_new = x - fl;
  uint64_t ncand = (uint64_t)fl;
  uint64_t excess = 0;
  if (ncand > n / 2) {
    excess = ncand - n / 2;
    ncand = n / 2;
  }

  for (uint32_t i = tid; i < (uint32_t)kNumCtr; i += BLOCK) s_ctr[i] = 0ull;
  if (tid == 0) s_sgbits = 0ull;

  View t, nb;
  const uint32_t L = A.lds_cap, L2 = A.lds_cap / 2 + 1;
  uint16_t *scr;
  if (kLds) {
    double *d = reinterpret_cast<double *>(smem);
    t.vx = d;
    t.vy = d + L;
    t.vz = d + 2 * L;
    nb.vx = d + 3 * L;
    nb.vy = d + 3 * L + L2;
    nb.vz = d + 3 * L + 2 * L2;
    uint16_t *h = reinterpret_cast<uint16_t *>(d + 3 * L + 3 * L2);
    t.lvl = h;
    nb.lvl = h + (size_t)mm * L;
    scr = h + (size_t)mm * (L + L2);
    uint8_t *bt = reinterpret_cast<uint8_t *>(scr + (size_t)2 * mm * BLOCK);
    t.sp = bt;
    nb.sp = bt + L;
    t.stride = L;
    nb.stride = L2;
    for (uint32_t i = tid; i < n; i += BLOCK) {
      t.vx[i] = A.st.vx[base + i];
      t.vy[i] = A.st.vy[base + i];
      t.vz[i] = A.st.vz[base + i];
      t.sp[i] = A.st.sp[base + i];
    }
    for (uint32_t m = 0; m < mm; ++m)
      for (uint32_t i = tid; i < n; i += BLOCK) t.lvl[m * L + i] = A.st.lvl[m * A.st.stride + base + i];
  } else {
    scr = reinterpret_cast<uint16_t *>(smem);
    t.vx = A.st.vx + base;
    t.vy = A.st.vy + base;
    t.vz = A.st.vz + base;
    t.sp = A.st.sp + base;
    t.lvl = A.st.lvl + base;
    t.stride = A.st.stride;
    nb.vx = A.scratch.vx + base;
    nb.vy = A.scratch.vy + base;
    nb.vz = A.scratch.vz + base;
    nb.sp = A.scratch.sp + base;
    nb.lvl = A.scratch.lvl + base;
    nb.stride = A.scratch.stride;
  }
  __syncthreads();

  Ctx C{T, A.lev, s_ctr, scr, tid, BLOCK};
  if (ncand > 0) {
    Perm P;
    make_perm(P, n, A.seed, c, A.step);
    double sg_seen = 0.0;
    uint32_t ncoll = 0;
    for (uint32_t k = tid; k < (uint32_t)ncand; k += BLOCK) {
      const uint32_t p = P(2 * k), q = P(2 * k + 1);
      Rng rng;
      rng.open(A.seed, k, c, A.step);
      const double dx = t.vx[p] - t.vx[q], dy = t.vy[p] - t.vy[q], dz = t.vz[p] - t.vz[q];
      const double g2 = (dx * dx + dy * dy) + dz * dz;
      const PairTab &PP = T->pr[t.sp[p]][t.sp[q]];
      const double sg = (g2 > 0.0) ? PP.csg * dpow(g2, PP.esg) : 0.0;
      sg_seen = sg > sg_seen ? sg : sg_seen;
      const double ua = rng.uniform();
      nb.sp[k] = (uint8_t)kNone;
      if (!(ua < sg / sgmax)) continue;
      ++ncoll;
      collide(C, t, p, q, g2, rng, nb, k);
    }
    atomicMax(&s_sgbits, (unsigned long long)__double_as_longlong(sg_seen));
    if (ncoll) atomicAdd(&s_ctr[HCAO_CTR_COLLISIONS], (unsigned long long)ncoll);
  }
  __syncthreads();

  // births: products in pair order after the survivors
  uint32_t births = 0;
  bool overflow = false;
  if (ncand > 0) {
    const uint32_t nc = (uint32_t)ncand;
    const uint32_t chunk = (nc + BLOCK - 1) / BLOCK;
    const uint32_t k0 = tid * chunk, k1 = min(nc, k0 + chunk);
    uint32_t mine = 0;
    for (uint32_t k = k0; k < k1; ++k) mine += (nb.sp[k] != kNone) ? 1u : 0u;
    const int any = __syncthreads_or(mine != 0);
    if (any) {
      uint32_t total;
      uint32_t rank = block_exclusive_scan<BLOCK>(mine, s_scan, total);
      births = total;
      const uint32_t limit = kLds ? min(cap, L) : cap;
      overflow = n + births > limit;
      if (!overflow) {
        for (uint32_t k = k0; k < k1; ++k) {
          if (nb.sp[k] == kNone) continue;
          const uint32_t dst = n + rank;
          ++rank;
          t.vx[dst] = nb.vx[k];
          t.vy[dst] = nb.vy[k];
          t.vz[dst] = nb.vz[k];
          t.sp[dst] = nb.sp[k];
          for (uint32_t m = 0; m < mm; ++m) t.lvl[m * t.stride + dst] = nb.lvl[m * nb.stride + k];
        }
      }
    }
  }
  const uint32_t n_out = overflow ? n : n + births;
  if (kLds) {
    __syncthreads();
    for (uint32_t i = tid; i < n_out; i += BLOCK) {
      A.st.vx[base + i] = t.vx[i];
      A.st.vy[base + i] = t.vy[i];
      A.st.vz[base + i] = t.vz[i];
      A.st.sp[base + i] = t.sp[i];
    }
    for (uint32_t m = 0; m < mm; ++m)
      for (uint32_t i = tid; i < n_out; i += BLOCK) A.st.lvl[m * A.st.stride + base + i] = t.lvl[m * L + i];
  }
  __syncthreads();
  if (tid == 0) {
    if (overflow) atomicOr(A.err, kErrCapacity);
    A.cells.cnt[c] = n_out;
    const double seen = __longlong_as_double((long long)s_sgbits);
    A.cells.sgmax[c] = seen > sgmax ? seen : sgmax;
    A.cells.rem[c] = rem_new;
    unsigned long long *ctr = A.cells.ctr + (size_t)c * kNumCtr;
    ctr[HCAO_CTR_CANDIDATES] += ncand;
    ctr[HCAO_CTR_SUPPRESSED] += excess;
    for (int i = 0; i < kNumCtr; ++i)
      if (i != HCAO_CTR_CANDIDATES && i != HCAO_CTR_SUPPRESSED) ctr[i] += s_ctr[i];
  }
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

struct InitArgs {
  const Tables *tab;
  const double *lev;
  State st;
  const uint64_t *off;
  const uint32_t *counts;  // [n_cells][n_species]
  const double *t_trans, *t_vib;
  uint64_t seed;
  uint32_t n_cells;
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
    A.st.vx[g] = sigma * n1;
    A.st.vy[g] = sigma * n2;
    A.st.vz[g] = sigma * n3;
    A.st.sp[g] = (uint8_t)s;
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
          const double *L = A.lev + S.lev_off[m];
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
      A.st.lvl[m * A.st.stride + g] = (uint16_t)l;
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
    const double vx = A.st.vx[base + i], vy = A.st.vy[base + i], vz = A.st.vz[base + i];
    const double v2 = (vx * vx + vy * vy) + vz * vz;
    vmax2 = v2 > vmax2 ? v2 : vmax2;
    mask |= 1u << A.st.sp[base + i];
  }
  atomicMax(&s_v, (unsigned long long)__double_as_longlong(vmax2));
  atomicOr(&s_mask, mask);
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
  double *out;  // [n_cells][6 + 2 S]
};

__global__ __launch_bounds__(256) void k_moments(MomentArgs A) {
  constexpr int kB = 256;
  constexpr int kW = 6 + 2 * kMaxSpecies;
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
    const double vx = A.st.vx[g], vy = A.st.vy[g], vz = A.st.vz[g];
    acc[0] += m * vx;
    acc[1] += m * vy;
    acc[2] += m * vz;
    acc[3] += m * ((vx * vx + vy * vy) + vz * vz);
    acc[4] += m;
    acc[5] += S.formation;
    double ev = 0.0;
    for (uint32_t q = 0; q < S.n_modes; ++q) ev = ev + mode_energy(S, A.lev, q, A.st.lvl[q * A.st.stride + g]);
#pragma unroll
    for (int j = 0; j < kMaxSpecies; ++j) {
      if ((uint32_t)j == s) {
        acc[6 + j] += 1.0;
        acc[6 + kMaxSpecies + j] += ev - S.zpe;
      }
    }
  }
  double *out = A.out + (size_t)c * (6 + 2 * ns);
#pragma unroll
  for (int j = 0; j < kW; ++j) {
    const bool used = j < 6 || (j >= 6 && j < 6 + (int)ns) || (j >= 6 + kMaxSpecies && j < 6 + kMaxSpecies + (int)ns);
    if (!used) continue;
    s_red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) s_red[threadIdx.x] += s_red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int dst = j < 6 ? j : (j < 6 + kMaxSpecies ? j : j - kMaxSpecies + (int)ns);
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

__global__ __launch_bounds__(kSortBlock) void k_sort_hist(const uint32_t *keys, uint64_t n, uint32_t shift,
                                                          uint32_t *hist, uint32_t n_tiles) {
  __shared__ uint32_t s_h[256];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const uint64_t i = t0 + (uint64_t)it * kSortBlock + threadIdx.x;
    if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * n_tiles + blockIdx.x] = s_h[threadIdx.x];
}

// single-workgroup exclusive scan of a u32 array into u64 offsets
__global__ __launch_bounds__(1024) void k_scan_u32(const uint32_t *in, uint64_t *out, uint64_t n) {
  __shared__ uint64_t s_part[1024];
  const uint64_t per = (n + 1023) / 1024;
  const uint64_t b = threadIdx.x * per, e = min(n, b + per);
  uint64_t s = 0;
  for (uint64_t i = b; i < e; ++i) s += in[i];
  s_part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const uint64_t v = s_part[i];
      s_part[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  uint64_t acc = s_part[threadIdx.x];
  for (uint64_t i = b; i < e; ++i) {
    out[i] = acc;
    acc += in[i];
  }
}

__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(const uint32_t *keys_in, const uint32_t *idx_in,
                                                             uint32_t *keys_out, uint32_t *idx_out, uint64_t n,
                                                             uint32_t shift, const uint64_t *offs,
                                                             uint32_t n_tiles) {
  constexpr int kWaves = kSortBlock / 64;
  __shared__ uint32_t s_run[256];
  __shared__ uint32_t s_wave[kWaves][256];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  s_run[tid] = 0;
  __syncthreads();
  const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
  const unsigned long long lt = lane ? ((1ull << lane) - 1ull) : 0ull;
  for (int it = 0; it < kSortItems; ++it) {
    for (int w = 0; w < kWaves; ++w) s_wave[w][tid] = 0;
    __syncthreads();
    const uint64_t i = t0 + (uint64_t)it * kSortBlock + tid;
    const bool valid = i < n;
    const uint32_t key = valid ? keys_in[i] : 0u;
    const uint32_t d = (key >> shift) & 0xffu;
    unsigned long long same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long bb = __ballot(((d >> bit) & 1u) != 0u);
      same &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt);
    if (valid && rank == 0) s_wave[wave][d] = (uint32_t)__popcll(same);
    __syncthreads();
    uint32_t before = s_run[d];
    for (uint32_t w = 0; w < wave; ++w) before += s_wave[w][d];
    if (valid) {
      const uint64_t pos = offs[(uint64_t)d * n_tiles + blockIdx.x] + before + rank;
      keys_out[pos] = key;
      idx_out[pos] = idx_in[i];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kWaves; ++w) add += s_wave[w][tid];
    s_run[tid] += add;
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
  A.st.vx[g] = A.vel[3 * src];
  A.st.vy[g] = A.vel[3 * src + 1];
  A.st.vz[g] = A.vel[3 * src + 2];
  A.st.sp[g] = A.sp[src];
  for (uint32_t m = 0; m < mm; ++m) A.st.lvl[m * A.st.stride + g] = A.lvl[src * mm + m];
}

__global__ void k_iota(uint32_t *x, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (uint32_t)i;
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers (host side)
// ---------------------------------------------------------------------------
size_t step_lds_bytes(uint32_t lds_cap, uint32_t mm, int block) {
  if (lds_cap == 0) return (size_t)2 * 2 * mm * block;
  return tile_lds_bytes(lds_cap, mm, (uint32_t)block);
}

hipError_t launch_step(const StepArgs &a, uint32_t mm, int block, uint32_t n_blocks, hipStream_t s) {
  const size_t lds = step_lds_bytes(a.lds_cap, mm, block);
  if (n_blocks == 0) return hipSuccess;
  switch (block) {
    case 64:
      if (a.lds_cap)
        hipLaunchKernelGGL((k_step<64, true>), dim3(n_blocks), dim3(64), lds, s, a);
      else
        hipLaunchKernelGGL((k_step<64, false>), dim3(n_blocks), dim3(64), lds, s, a);
      break;
    case 128:
      if (a.lds_cap)
        hipLaunchKernelGGL((k_step<128, true>), dim3(n_blocks), dim3(128), lds, s, a);
      else
        hipLaunchKernelGGL((k_step<128, false>), dim3(n_blocks), dim3(128), lds, s, a);
      break;
    case 256:
      if (a.lds_cap)
        hipLaunchKernelGGL((k_step<256, true>), dim3(n_blocks), dim3(256), lds, s, a);
      else
        hipLaunchKernelGGL((k_step<256, false>), dim3(n_blocks), dim3(256), lds, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t set_step_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
  const void *fns[] = {(const void *)k_step<64, true>, (const void *)k_step<128, true>,
                       (const void *)k_step<256, true>};
  for (const void *f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  }
  return e;
}

hipError_t launch_init(const Tables *tab, const double *lev, const State &st, const uint64_t *off,
                       const uint32_t *counts, const double *tt, const double *tv, uint64_t seed, uint32_t n_cells,
                       hipStream_t s) {
  InitArgs a{tab, lev, st, off, counts, tt, tv, seed, n_cells};
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

hipError_t launch_scan_u32(const uint32_t *in, uint64_t *out, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, s, in, out, n);
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

// Stable sort of (key, index) by key; buffers of n entries each, hist of
// 256 * tiles u32 and offs of 256 * tiles u64. Result in keys/idx (ping-pong
// handled here; returns which buffer holds the result).
hipError_t launch_sort(uint32_t *keys, uint32_t *idx, uint32_t *keys_tmp, uint32_t *idx_tmp, uint32_t *hist,
                       uint64_t *offs, uint64_t n, uint32_t key_bits, hipStream_t s, bool &result_in_tmp) {
  result_in_tmp = false;
  if (n == 0) return hipSuccess;
  const uint32_t tiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx, n);
  uint32_t *kin = keys, *iin = idx, *kout = keys_tmp, *iout = idx_tmp;
  for (uint32_t shift = 0; shift < key_bits; shift += 8) {
    hipLaunchKernelGGL(k_sort_hist, dim3(tiles), dim3(kSortBlock), 0, s, kin, n, shift, hist, tiles);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, s, hist, offs, (uint64_t)256 * tiles);
    hipLaunchKernelGGL(k_sort_scatter, dim3(tiles), dim3(kSortBlock), 0, s, kin, iin, kout, iout, n, shift, offs,
                       tiles);
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

hipError_t launch_place(const Tables *tab, const uint32_t *sorted_cell, const uint32_t *sorted_idx,
                        const uint64_t *packed_start, const uint64_t *off, const uint8_t *sp, const double *vel,
                        const uint16_t *lvl, const State &st, uint64_t n, hipStream_t s) {
  PlaceArgs a{tab, sorted_cell, sorted_idx, packed_start, off, sp, vel, lvl, st, n};
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_load_place, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hcao
