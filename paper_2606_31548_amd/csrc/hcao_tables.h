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

struct SpeciesTab {
  double mass, zpe, formation, p_vib;
  uint32_t n_modes, n_bend, sampler, pad;
  double kt[kMaxModes];         // bends: k_B Theta
  double theta[kMaxModes];      // bends: Theta
  double de[kMaxModes];         // stretches: D_e
  uint32_t lev_off[kMaxModes];  // stretches: offset of level 0 in the level array
  uint32_t idiss[kMaxModes];    // stretches: top bound level
};

struct PairTab {
  double mr, hm, m_a, m_b, msum, wa, wb, csg, esg, q;
};

struct ReactionTab {
  int32_t kind, a, b, c, d, pad;
  uint64_t mask;
  double alpha[kMaxModes];
  double steric, ea, dh, zsum;
};

struct Tables {
  uint32_t n_species, n_reactions, max_modes, n_levels;
  SpeciesTab sp[kMaxSpecies];
  PairTab pr[kMaxSpecies][kMaxSpecies];
  ReactionTab rx[kMaxReactions];
};

// Particle state in HBM: structure of arrays, cell-major segments with
// per-cell slot capacity. Slot i of cell c lives at index off[c] + i;
// level of mode m at lvl[m * stride + index].
struct State {
  double *vx, *vy, *vz;
  uint8_t *sp;
  uint16_t *lvl;
  uint64_t stride;  // total slots (all cells)
};

struct CellArrays {
  const uint64_t *off;
  uint32_t *cnt;
  const uint32_t *cap;
  const double *volume, *weight;
  double *sgmax, *rem;
  unsigned long long *ctr;  // [n_cells][kNumCtr]
};

struct StepArgs {
  const Tables *tab;
  const double *lev;
  State st;
  State scratch;  // newborn staging for cells processed from global memory
  CellArrays cells;
  const uint32_t *cell_list;  // cells of this launch (nullptr: cell = block index)
  uint32_t n_launch_cells;
  uint32_t lds_cap;  // slot capacity of the LDS tile (0: global-memory path)
  uint32_t *err;
  uint64_t seed;
  uint32_t step;
  double dt;
};

}  // namespace hcao
