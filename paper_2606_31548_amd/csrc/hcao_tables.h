// hcao_tables.h -- device-resident tables and kernel argument blocks shared
// by the host runtime (hcao_runtime.cpp) and the gfx950 kernels
// (hcao_kernels.hip). Plain structs, no methods.
#pragma once
#include <stdint.h>

#include "hcao.h"

namespace hcao {

constexpr int kMaxSpecies = HCAO_MAX_SPECIES;
constexpr int kMaxModes = HCAO_MAX_MODES;
constexpr int kMaxReactions = HCAO_MAX_REACTIONS;
constexpr int kMaxLevels = HCAO_MAX_LEVELS;
constexpr int kMaxChannels = 64;
constexpr uint64_t kMaxTrials = 1000000;
constexpr int kNumCtr = HCAO_N_CTR;

// error bits of the device status word
constexpr uint32_t kErrCapacity = 1u;
constexpr uint32_t kErrInvalid = 2u;
constexpr uint32_t kErrLevel = 4u;
constexpr uint32_t kErrNonFinite = 8u;
constexpr uint32_t kErrBounds = 16u;  // bounds-checked builds: an index outside its array

struct SpeciesTab {
  double mass, zpe, formation, p_vib, p_rot;
  uint32_t n_modes, n_bend, sampler;
  uint32_t concave;             // bit m: the level spacings of mode m never increase
  uint32_t zeta_rot, pad_rot;   // rotational degrees of freedom (0, 2 or 3)
  double kt[kMaxModes];         // bends: k_B Theta
  double theta[kMaxModes];      // bends: Theta
  double de[kMaxModes];         // stretches: D_e
  uint32_t lev_off[kMaxModes];  // stretches: offset of level 0 in the level array
  uint32_t idiss[kMaxModes];    // stretches: top bound level
};

// PairTab::react bits
constexpr uint32_t kReactAny = 1u;    // some reaction lists the pair (as A, or as A + B / B + C), in either order
constexpr uint32_t kReactRecomb = 2u;  // a recombination lists it as B + C, in either order

// Words per work-list entry: the pair as found (candidate j, p, q, the sort
// key in bits 0-7 with the index of the pair's cell in its group from bit 8,
// words 1-3 of the pair stream's first Philox block), then the sorted list
// (the index of an entry as found).
constexpr uint32_t kWorkFound = 7;
constexpr uint32_t kWorkSorted = 1;
constexpr uint32_t kWorkWords = kWorkFound + kWorkSorted;

// Bounds of the pair's dissociation and exchange channels, per side (0: a is
// A, 1: b is A), for the test that lets a pair skip the channel scan when no
// channel can open: a dissociation channel's excess energy is at most
// (E_tr + E_rot,A) + E_vib,A + dis_c[side], an exchange channel's at most
// (E_tr + E_rot,A) + ex_a[side] E_vib,A - ex_e[side] (its alpha-weighted
// energy is at most alpha_max E_vib,A); -inf / ex_a < 0 mark no channel.
// n_steric: the scan's steric draws, one per exchange reaction matched on
// either side, whether or not anything opens.
struct PairBound {
  double dis_c[2], ex_a[2], ex_e[2];
  uint32_t n_steric, pad;
};

struct PairTab {
  double mr, hm, m_a, m_b, msum, wa, wb, csg, esg, q;
  uint32_t react;     // kReact* bits
  uint32_t beta_off;  // exact sampler: offset of the beta table of species a with exponent q
  PairBound bound;
};

// Recombination B + C (+M) -> A (+M) is stored with a = B, b = C, c = A,
// d = -1; its probability factors k_b / <sigma g>_BC [m^3] per third-body
// species and log-spaced temperature node start at rec_off in the
// recombination array.
struct ReactionTab {
  int32_t kind, a, b, c, d, pad;
  uint64_t mask;
  double alpha[kMaxModes];
  double steric, ea, dh, zsum;
  double gamma_rot;  // rotation coupling of dissociation / exchange
  uint64_t rec_off;
};

// Exact sampler: inverse temperature of the proposal per bin of the energy
// E' above the zero point; bin = (bit pattern of E') >> 48, clamped to
// [kExactBinLo, kExactBinHi] (2^-90 .. 2^-49 J, 1/16 octave per bin)
constexpr uint32_t kExactBinLo = 14928u;
constexpr uint32_t kExactBinHi = 15583u;
constexpr uint32_t kExactBins = kExactBinHi - kExactBinLo + 1;
constexpr uint32_t kExactNBeta = 960u;  // beta grid (1 + (j mod 16) / 16) 2^(40 + j div 16)

// bytes of the fixed device array behind the allocation-free step
constexpr uint64_t kStaticScratchBytes = HCAO_STATIC_SCRATCH_BYTES;

constexpr uint32_t kRecNodes = 1024;
constexpr double kRecTmin = 100.0;
constexpr double kRecTmax = 5.0e4;

struct Tables {
  uint32_t n_species, n_reactions, max_modes, n_levels;
  uint32_t has_recomb, rec_nt, has_rot, pad1;
  double rec_l0, rec_inv_step;  // log T of node 0; nodes per unit of log T
  SpeciesTab sp[kMaxSpecies];
  PairTab pr[kMaxSpecies][kMaxSpecies];
  ReactionTab rx[kMaxReactions];
};

// Particle state in HBM: structure of arrays, cell-major segments with
// per-cell slot capacity. Slot i of cell c lives at index off[c] + i. The
// quantum numbers of a slot are one row of lrow uint16 (lrow = max_modes
// rounded up to even, so rows are dword aligned): mode m at lvl[index *
// lrow + m], modes the species does not have (and the padding) 0.
// Velocities are fp64 (vx, vy, vz) in the fp64 form and fp32 (fx, fy, fz)
// in the mixed form; the other set is null.
struct State {
  double *vx, *vy, *vz;
  float *fx, *fy, *fz;
  uint8_t *sp;
  uint16_t *lvl;
  double *rot;      // rotational energy [J]; null when no species has a rotor
  double *px, *py, *pz;  // positions [m]; null outside the spatial mode
  uint32_t lrow;    // uint16 per level row (even)
#ifdef HCAO_CHECKED
  uint64_t n_slots;  // slots the arrays hold: the bounds-checked build tests slot indices against it
#endif
};

// records how many slots the arrays of s hold (bounds-checked builds only)
inline void set_slots(State &s, uint64_t n) {
#ifdef HCAO_CHECKED
  s.n_slots = n;
#else
  (void)s;
  (void)n;
#endif
}

// level row length for max_modes modes: even, at least 2
inline uint32_t level_row(uint32_t max_modes) { return max_modes < 2 ? 2u : (max_modes + 1u) & ~1u; }

struct CellArrays {
  const uint64_t *off;
  uint32_t *cnt;
  const uint32_t *cap;
  const double *volume, *weight;
  double *sgmax, *rem;
  double *defect;           // mixed form: energy the cell's particles lack [J]
  unsigned long long *ctr;  // [n_cells][kNumCtr]
  double *tsum;             // recombination: [5][n_cells] running sums m, m v_x, m v_y, m v_z, m |v|^2 (else null)
  uint32_t n_cells;
};

// Phases of the step kernel, for the clock sums of instrumented builds
// (HCAO_PHASE_CLOCKS): table and cell loads of a launch, NTC counts and
// permutation keys, cell temperature, candidate acceptance, work-list sort,
// collisions, product placement, and the launch's final stores.
// The collision phase is further split per wave (sums over waves, in the
// leading active lane's clock): gathering a pair's state, the reaction
// decision, the relaxation sampler, scattering and reaction application,
// and the write-back.
enum StepPhase {
  kPhaseLoad = 0,
  kPhaseNtc,
  kPhaseTemperature,
  kPhaseAccept,
  kPhaseSort,
  kPhaseCollide,
  kPhasePlace,
  kPhaseStore,
  kPhaseCollideGather,
  kPhaseCollideDecide,
  kPhaseCollideRelax,
  kPhaseCollideScatter,
  kPhaseCollideWrite,
  kPhases
};
static_assert(kPhases == HCAO_N_PHASES, "phase list and ABI disagree");

// bflag bits of a candidate pair
constexpr uint8_t kFlagBorn = 1;      // it left a dissociation product in the products staging
constexpr uint8_t kFlagCollided = 2;  // it collided (its running-sum change is in tdelta)

// Workgroup b processes the consecutive cells [grp[2b], grp[2b+1]); its work
// list, product flags and pair energy defects are the entries
// [grp_work[2b], grp_work[2b+1]) of work (kWorkWords words each: the pair as
// found and its place in the sorted list) / bflag / wdef
// (sum over its cells of cap/2 + 1 entries).
struct StepArgs {
  const Tables *tab;
  const double *lev;
  State st;
  State born;  // products of the step, at the workgroup's work base + candidate index
  CellArrays cells;
  const double *rec;   // recombination factors
  const double *beta;  // exact sampler's beta tables (PairTab::beta_off)
  const uint32_t *grp;
  const uint64_t *grp_work;
  uint32_t *work;
  uint8_t *bflag;
  double *wdef;  // mixed form: energy defect of each candidate pair, indexed like bflag
  double *tdelta;  // recombination: [5][tdelta_stride] each colliding pair's change of its cell's running sums
  uint64_t tdelta_stride;
  uint32_t *err;
  unsigned long long *clk;   // per-phase clock sums [kPhases] (instrumented builds) or null
  uint64_t seed;
  const uint32_t *step_dev;  // device step index (graph replays) or null
  uint32_t step;             // index of the launch's first step (plus *step_dev when set)
  uint32_t n_steps;          // steps advanced by this launch
  double dt;
};

// Spatial mode, move pass: block c moves the particles of cell c over dt
// to find their new cells (the state is left as it is: the place pass
// applies the same move as it copies each particle to its new slot); its
// stayers (new cell = c) and its movers are listed by cell-relative slot
// in list[], stayers in slot order from the cell's first slot up, movers in
// slot order from its last slot down, each mover's new cell in key[] at the
// same place as its list entry; n_stay[c] and n_move[c] count them. A particle that crosses an open
// face (bit 2 axis + side of open) is in neither list; flux[1] counts them.
struct MoveArgs {
  State st;
  const uint64_t *off;
  const uint32_t *cnt, *cap;
  uint32_t n_cells, nx, ny, nz, periodic, open;
  double len[3];
  double dt;
  uint32_t *key, *list, *n_stay, *n_move;
  unsigned long long *flux;  // [2]: admitted, left (null without open faces)
};

// Spatial mode, admission through open faces; one thread per (face cell,
// species), face cells numbered over all six faces (face f = 2 axis + side
// starts at face_base[f]). The count pass sets count[t] = floor(x) with x =
// ((flux_s A) dt) / F_N + rem[t] and keeps the fraction in rem[t]; the make
// pass (one thread per admission) writes admission j of the step (j =
// ibase[t] + i) to slot j of the staging state ins and to the mover list at movers + j with the virtual
// old slot tot + j and its new cell (n_cells if it leaves again during its
// partial flight).
struct InflowArgs {
  const Tables *tab;
  const double *lev;
  State ins;
  const double *weight;        // per cell F_N
  double *rem;                 // [n_face_cells * n_species]
  uint32_t *count;             // [n_face_cells * n_species]
  const uint64_t *ibase;       // exclusive scan of count
  const uint64_t *mbase;       // movers' scan: mbase[n_cells] = movers
  uint32_t *mkey, *mslot;
  unsigned long long *flux;    // [2]: admitted, left
  uint32_t *err;
  double flux_s[HCAO_MAX_SPECIES];  // n_s sqrt(k T / (2 pi m_s)) [m^-2 s^-1]
  double len[3];
  double dt, t_trans, t_vib;
  uint64_t seed, tot, cap_ins;
  uint64_t n_ins;              // admissions of the step (make pass)
  uint32_t face_base[7];
  uint32_t nx, ny, nz, n_cells, periodic, open, n_species, step;
};

// Spatial mode, re-bin after the move pass. The new order of cell k is the
// stable order by (new cell, old slot): movers from lower slots, then k's
// stayers, then movers from higher slots. Only the movers are sorted: the
// list pass writes them in slot order (position mbase[c] + rank), a stable
// radix sort orders them by new cell and packed[k] is the start of k's run.
// The place pass then writes every particle of each old cell to its new
// slot.
//
// Where the re-bin puts new cell k's particles: a list entry at sorted
// position pos (its run in the sorted keys starts at lo) goes to slot
// first + pos, plus ns (the cell's stayers, which fill the gap) when pos >=
// split = lo + below; stayer r goes to off[k] + below + r; a slot at or past
// end (off[k] + the capped count) is dropped. first = off[k] - lo, modulo
// 2^64.
struct alignas(16) RebinDest {
  uint64_t first, split, end;
  uint32_t below, ns;
};

struct RebinArgs {
  State src, dst;
  State ins;                                     // admitted particles (virtual old slots tot + j)
  uint64_t tot;
  const uint64_t *off;
  const uint32_t *cap;
  const uint32_t *key, *list, *n_stay, *n_move;  // from the move pass (key: movers' new cells, beside list)
  const uint64_t *mbase;                         // exclusive scan of n_move
  uint32_t *mkey, *mslot;                        // movers in slot order: new cell, old slot
  const uint32_t *skey, *sidx;                   // sorted movers: new cell, position in the list
  uint64_t *packed;                              // run starts in skey (n_cells + 1)
  uint32_t *slot;                                // new slot of each list entry (~0u: dropped)
  RebinDest *dest;                               // per new cell (n_cells)
  uint32_t *cnt, *err;
  uint64_t m;                                    // number of list entries (movers, then admissions)
  uint64_t m_real;                               // movers out of real slots (the admissions follow)
  uint32_t n_cells, mm;
  double dt, len[3];                             // the step's move, applied by the place pass
  uint32_t periodic, open;
};

// Forward recombination probability summed over every level combination of
// a species (Eq. recomb-correct). Enumeration pass: thread i takes prefix i
// of the levels of the first n_prefix_modes modes (mixed radix over box[])
// and walks the remaining modes depth first, emitting one record per
// combination below de (a leaf: energy above ground, code kRecLeaf) and one
// per point where the walk first crosses de at mode m, level j (energy of
// that partial combination, code m | j << 8). With offset == null it only
// counts a thread's records into count[i].
constexpr uint32_t kRecLeaf = 0xFFu;

struct RecEnumArgs {
  const Tables *tab;
  const double *lev;
  uint32_t species, n_prefix_modes;
  uint32_t box[kMaxModes];
  uint64_t n_prefix;
  double de;
  uint32_t *count;
  const uint64_t *offset;
  double *rec_e;
  uint32_t *rec_code;
};

// Sum pass: block b evaluates temperature t[b]; leaves contribute
// Q(a, (de - e)/kT) exp(-e/kT), crossings exp(-e/kT) times the Boltzmann sum
// of the crossing mode's levels from j up (relative to level j) times the
// partition sums of the later modes. num[b] / den[b] is the probability.
struct RecSumArgs {
  const Tables *tab;
  const double *lev;
  uint32_t species;
  double de, a, lgamma_a;
  const double *t;
  const double *rec_e;
  const uint32_t *rec_code;
  uint64_t n_rec;
  double *num, *den;
};

}  // namespace hcao
