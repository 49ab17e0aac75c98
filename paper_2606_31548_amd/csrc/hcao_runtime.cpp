// hcao_runtime.cpp -- host runtime behind the C ABI of include/hcao.h.
//
// Builds the species, pair and reaction tables on the host, owns the
// device buffers of the structure-of-arrays particle state, and issues the
// gfx950 kernels of hcao_kernels.hip on the context's stream.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "hcao.h"
#include "hcao_host_tables.h"
#include "hcao_tables.h"

namespace {
// A roctx range over one host-side phase of the library (the step, the
// spatial move and re-bin, loads, moments, tuning), shown by rocprofv3
// --marker-trace beside the kernels it launched.
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};
}  // namespace

namespace hcao {
// kernels (hcao_kernels.hip)
size_t step_lds_bytes(const Tables &T, uint32_t max_cells, int block);
hipError_t launch_step(const StepArgs &a, size_t lds, int block, bool mixed, int level, uint32_t n_groups,
                       hipStream_t s);
hipError_t set_step_lds_limit(size_t bytes);
hipError_t launch_advance(uint32_t *step, uint32_t n, hipStream_t s);
hipError_t static_scratch_address(void **ptr);
hipError_t launch_init(const Tables *tab, const double *lev, const State &st, const uint64_t *off,
                       const uint32_t *counts, const double *tt, const double *tv, uint64_t seed, uint32_t n_cells,
                       const uint32_t grid[3], const double len[3], hipStream_t s);
hipError_t launch_move(const MoveArgs &a, hipStream_t s);
hipError_t launch_list_movers(const RebinArgs &a, hipStream_t s);
hipError_t launch_inflow_count(const InflowArgs &a, hipStream_t s);
hipError_t launch_inflow_make(const InflowArgs &a, hipStream_t s);
hipError_t launch_rebin_place(const RebinArgs &a, hipStream_t s);
hipError_t launch_cell_init(const Tables *tab, const State &st, const CellArrays &cells, uint32_t n_cells,
                            hipStream_t s);
hipError_t launch_moments(const Tables *tab, const double *lev, const State &st, const uint64_t *off,
                          const uint32_t *cnt, double *out, uint32_t n_cells, hipStream_t s);
hipError_t launch_load_check(const Tables *tab, const uint32_t *cell, const uint8_t *sp, const double *vel,
                             const uint16_t *lvl, uint64_t n, uint32_t n_cells, uint32_t *count, uint32_t *err,
                             hipStream_t s);
hipError_t launch_scan_u32(const uint32_t *in, uint64_t *out, uint64_t n, uint64_t *tmp, hipStream_t s);
uint64_t scan_tmp_entries(uint64_t n);
hipError_t launch_rec_enum(const RecEnumArgs &a, bool write, hipStream_t s);
hipError_t launch_rec_sum(const RecSumArgs &a, uint32_t n_t, size_t lds, hipStream_t s);
hipError_t launch_sort(uint32_t *keys, uint32_t *idx, uint32_t *keys_tmp, uint32_t *idx_tmp, uint32_t *hist,
                       uint64_t *offs, uint64_t *scan_tmp, uint64_t n, uint32_t key_bits, hipStream_t s,
                       bool &result_in_tmp);
uint64_t sort_tiles(uint64_t n);
uint64_t sort_hist_entries(uint64_t n);
hipError_t launch_place(const Tables *tab, const uint32_t *sorted_cell, const uint32_t *sorted_idx,
                        const uint64_t *packed_start, const uint64_t *off, const uint8_t *sp, const double *vel,
                        const uint16_t *lvl, const double *rot, const double *pos, const State &st, uint64_t n,
                        hipStream_t s);
}  // namespace hcao

using namespace hcao;

namespace {

constexpr double kB = 1.380649e-23;
constexpr double kPi = 3.141592653589793;
constexpr size_t kLdsBudget = 64 * 1024;  // LDS bytes per workgroup of the step kernel
constexpr uint32_t kMaxGroupCells = 64;   // cells per workgroup at most

struct SpeciesHost {
  hcao_species_desc d;
  std::vector<double> theta;
  std::vector<std::vector<double>> levels;  // per stretch
  std::vector<double> de;
  double zpe = 0.0;
  int sampler = HCAO_SAMPLER_JOINT;
  uint32_t n_modes = 0;
};

struct ReactionHost {
  hcao_reaction_desc d;
  std::vector<double> alpha;
};

template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  hipError_t alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = count;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

}  // namespace

struct hcao_ctx {
  hcao_config cfg{};
  std::vector<double> rec_host;   // recombination factors, all reactions
  std::vector<double> beta_host;  // exact sampler: beta per E' bin, per (species, LB exponent)
  bool has_exact = false;         // some species uses the exact sampler
  DevBuf<double> d_rec;
  DevBuf<double> d_beta;
  std::vector<double> volume, weight;
  hipStream_t stream = nullptr;
  int device = 0;
  bool finalized = false, loaded = false;
  hcao_status sticky = HCAO_OK;
  std::string last_error;
  std::vector<SpeciesHost> species;
  std::vector<host::VibrationalThermometer> thermo;  // per species, built at finalize
  std::vector<ReactionHost> reactions;
  uint32_t max_modes = 0;
  Tables tab{};
  std::vector<double> lev_host;
  DevBuf<Tables> d_tab;
  DevBuf<double> d_lev;
  // particle state
  uint64_t total_slots = 0;
  std::vector<uint32_t> cap_host;
  std::vector<uint64_t> off_host;
  bool mixed = false;                         // fp32 velocities (mixed form)
  DevBuf<double> vx, vy, vz, bvx, bvy, bvz;  // fp64 form
  DevBuf<float> fx, fy, fz, bfx, bfy, bfz;   // mixed form
  DevBuf<uint8_t> sp, bsp;
  DevBuf<uint16_t> lvl, blvl;
  DevBuf<double> rot, brot;  // rotational energies (only when some species has a rotor)
  // spatial mode: positions, and the re-bin's sort buffers (all slots)
  bool spatial = false;
  uint32_t grid[3] = {1, 1, 1}, periodic = 0;
  double len[3] = {0.0, 0.0, 0.0};
  DevBuf<double> px, py, pz, bpx, bpy, bpz;
  DevBuf<uint32_t> mv_key, mv_list, mv_mkey, mv_mslot, mv_sidx, mv_sidx_tmp, mv_hist;
  DevBuf<uint32_t> mv_nstay, mv_nmove, mv_ktmp;
  DevBuf<uint64_t> mv_offs, mv_packed, mv_stmp, mv_mbase;
  DevBuf<RebinDest> mv_dest;  // per new cell: where the place pass puts its particles
  uint64_t list_cap = 0;  // entries of the mover list arrays (movers and admissions)
  // open faces: the reservoir's one-sided flux per species, per (face cell,
  // species) inflow remainders and counts, the admissions' staging state,
  // and the counts of particles admitted and gone
  uint32_t open_faces = 0, face_base[7] = {0, 0, 0, 0, 0, 0, 0};
  double in_flux[kMaxSpecies] = {}, in_t = 0.0, in_tv = 0.0;
  DevBuf<double> in_rem;
  DevBuf<uint32_t> in_count;
  DevBuf<uint64_t> in_base;
  DevBuf<unsigned long long> flux;
  uint64_t ins_cap = 0;
  DevBuf<double> ivx, ivy, ivz, irot, ipx, ipy, ipz;
  DevBuf<float> ifx, ify, ifz;
  DevBuf<uint8_t> isp;
  DevBuf<uint16_t> ilvl;
  DevBuf<uint64_t> off;
  DevBuf<uint32_t> cnt, cap;
  DevBuf<double> d_volume, d_weight, sgmax, rem, defect;
  DevBuf<double> tsum;    // recombination: running sums of the cell temperature [5][n_cells]
  DevBuf<double> tdelta;  // recombination: each work entry's change of the running sums [5][work_entries]
  DevBuf<unsigned long long> ctr;
  DevBuf<uint32_t> err;
  DevBuf<uint32_t> grp, work;
  DevBuf<uint64_t> grp_work;
  DevBuf<uint8_t> bflag;
  DevBuf<double> wdef;
  uint64_t work_entries = 0;  // entries of work / bflag / wdef
  uint32_t n_groups = 0, max_group_cells = 1;
  size_t step_lds = 0;
  int block = 64;
  uint32_t group_slots = 1024;  // target slot capacity per workgroup
  uint32_t step = 0;
  bool timing = false;
  double timed_ms = 0.0;
  uint64_t timed_launches = 0, timed_steps = 0;
  uint32_t steps_per_launch = 1u << 30;  // all steps of an hcao_step call in one launch
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // graph form of the step
  uint64_t shape_gen = 0;          // bumped whenever the workgroup layout changes
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  double graph_dt = 0.0;
  uint32_t graph_n = 0, graph_launches = 0;
  uint64_t graph_gen = ~0ull;
  DevBuf<uint32_t> d_step;      // step index read by graph replays
  int64_t d_step_value = -1;    // value d_step holds (-1: unknown)
  DevBuf<unsigned long long> clk;  // per-phase clock sums of the step kernel (instrumented builds)
};

namespace {

thread_local std::string g_create_error;  // failure text of the last hcao_create on this thread

// Device address of the fixed scratch array of the allocation-free step, per
// device: looked up once per device, with that device current, when the
// first context is created on it.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

hipError_t lookup_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = static_scratch_address(&p);
  if (e == hipSuccess) g_scratch_dev[device] = p;
  return e;
}

void *static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_dev[device];
}

hcao_status fail(hcao_ctx *c, hcao_status s, const std::string &msg) {
  if (c) c->last_error = msg;
  return s;
}

hcao_status hip_fail(hcao_ctx *c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (c) {
    c->last_error = m;
    c->sticky = HCAO_EDEVICE;
  }
  return HCAO_EDEVICE;
}

#define HIP_TRY(ctx, expr)                               \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

// Level ladder of one stretch: explicit energies, or the Morse ladder of
// (w_e, x_e) capped at D_e (D_e = h c w_e / (4 x_e) when not given).
hcao_status build_stretch(hcao_ctx *c, double we, double xe, double de, uint32_t n_explicit, const double *expl,
                          std::vector<double> &out, double &de_out) {
  const char *why = n_explicit > 0 ? host::explicit_ladder(expl, n_explicit, de, out) : host::morse_ladder(we, xe, de, out);
  if (why) return fail(c, HCAO_EINVAL, why);
  de_out = de;
  return HCAO_OK;
}

// the vibrational modes of a species for the host tables
host::ModeSet modes_of(const SpeciesHost &s) {
  host::ModeSet m;
  m.theta = s.theta;
  for (const std::vector<double> &L : s.levels) m.ladder.push_back(&L);
  return m;
}

double host_mode_energy(const SpeciesHost &s, uint32_t m, uint32_t i) {
  const uint32_t nb = s.d.n_bend;
  if (m < nb) return ((double)i + 0.5) * (kB * s.theta[m]);
  return s.levels[m - nb][i];
}

void release_ins(hcao_ctx *c) {
  c->ivx.release();
  c->ivy.release();
  c->ivz.release();
  c->ifx.release();
  c->ify.release();
  c->ifz.release();
  c->isp.release();
  c->ilvl.release();
  c->irot.release();
  c->ipx.release();
  c->ipy.release();
  c->ipz.release();
  c->ins_cap = 0;
}

void free_state(hcao_ctx *c) {
  c->vx.release();
  c->vy.release();
  c->vz.release();
  c->fx.release();
  c->fy.release();
  c->fz.release();
  c->sp.release();
  c->lvl.release();
  c->bvx.release();
  c->bvy.release();
  c->bvz.release();
  c->bfx.release();
  c->bfy.release();
  c->bfz.release();
  c->bsp.release();
  c->blvl.release();
  c->rot.release();
  c->brot.release();
  c->px.release();
  c->py.release();
  c->pz.release();
  c->bpx.release();
  c->bpy.release();
  c->bpz.release();
  c->mv_key.release();
  c->mv_list.release();
  c->mv_mkey.release();
  c->mv_mslot.release();
  c->mv_sidx.release();
  c->mv_sidx_tmp.release();
  c->mv_nstay.release();
  c->mv_nmove.release();
  c->mv_mbase.release();
  c->mv_hist.release();
  c->mv_offs.release();
  c->mv_packed.release();
  c->mv_dest.release();
  c->mv_stmp.release();
  c->mv_ktmp.release();
  c->list_cap = 0;
  release_ins(c);
  c->off.release();
  c->cnt.release();
  c->cap.release();
  c->d_volume.release();
  c->d_weight.release();
  c->sgmax.release();
  c->rem.release();
  c->defect.release();
  c->tsum.release();
  c->ctr.release();
  c->grp.release();
  c->grp_work.release();
  c->work.release();
  c->bflag.release();
  c->wdef.release();
  c->work_entries = 0;
  c->loaded = false;
}

uint32_t default_cap(const hcao_ctx *c, uint32_t n) {
  if (c->cfg.capacity_per_cell) return c->cfg.capacity_per_cell;
  return n + n / 4 + 32;
}

// staging state of the admissions through open faces (stride ins_cap)
State ins_state(hcao_ctx *c) {
  State s{c->ivx.p, c->ivy.p, c->ivz.p, c->ifx.p, c->ify.p, c->ifz.p, c->isp.p, c->ilvl.p, c->irot.p,
          c->ipx.p, c->ipy.p, c->ipz.p, level_row(c->max_modes)};
  set_slots(s, c->ins_cap);
  return s;
}

State state_of(hcao_ctx *c) {
  State s{c->vx.p, c->vy.p, c->vz.p, c->fx.p, c->fy.p, c->fz.p, c->sp.p, c->lvl.p, c->rot.p,
          c->px.p, c->py.p, c->pz.p, level_row(c->max_modes)};
  set_slots(s, c->total_slots);
  return s;
}
State staging_of(hcao_ctx *c) {
  State s{c->bvx.p, c->bvy.p, c->bvz.p, c->bfx.p, c->bfy.p, c->bfz.p, c->bsp.p, c->blvl.p, c->brot.p,
          c->bpx.p, c->bpy.p, c->bpz.p, level_row(c->max_modes)};
  set_slots(s, c->total_slots);
  return s;
}
CellArrays cells_of(hcao_ctx *c) {
  return CellArrays{c->off.p,    c->cnt.p, c->cap.p,    c->d_volume.p, c->d_weight.p,
                    c->sgmax.p,  c->rem.p, c->defect.p, c->ctr.p,      c->tab.has_recomb ? c->tsum.p : nullptr,
                    c->cfg.n_cells};
}

// velocity arrays of the context's precision (three, fp64 or fp32)
hipError_t alloc_vel(hcao_ctx *c, DevBuf<double> &x, DevBuf<double> &y, DevBuf<double> &z, DevBuf<float> &fx,
                     DevBuf<float> &fy, DevBuf<float> &fz, uint64_t n) {
  hipError_t e;
  if (c->mixed) {
    if ((e = fx.alloc(n)) != hipSuccess) return e;
    if ((e = fy.alloc(n)) != hipSuccess) return e;
    return fz.alloc(n);
  }
  if ((e = x.alloc(n)) != hipSuccess) return e;
  if ((e = y.alloc(n)) != hipSuccess) return e;
  return z.alloc(n);
}

// all velocity slots as fp64 (synchronous)
hcao_status download_vel(hcao_ctx *c, std::vector<double> &vx, std::vector<double> &vy, std::vector<double> &vz) {
  const uint64_t tot = c->total_slots;
  vx.resize(tot);
  vy.resize(tot);
  vz.resize(tot);
  if (c->mixed) {
    std::vector<float> fx(tot), fy(tot), fz(tot);
    HIP_TRY(c, hipMemcpyAsync(fx.data(), c->fx.p, tot * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(fy.data(), c->fy.p, tot * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(fz.data(), c->fz.p, tot * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (uint64_t i = 0; i < tot; ++i) {
      vx[i] = fx[i];
      vy[i] = fy[i];
      vz[i] = fz[i];
    }
    return HCAO_OK;
  }
  HIP_TRY(c, hipMemcpyAsync(vx.data(), c->vx.p, tot * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(vy.data(), c->vy.p, tot * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(vz.data(), c->vz.p, tot * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return HCAO_OK;
}

// all velocity slots from fp64 (rounded to fp32 in the mixed form; synchronous)
hcao_status upload_vel(hcao_ctx *c, const std::vector<double> &vx, const std::vector<double> &vy,
                       const std::vector<double> &vz) {
  const uint64_t tot = c->total_slots;
  if (c->mixed) {
    std::vector<float> fx(tot), fy(tot), fz(tot);
    for (uint64_t i = 0; i < tot; ++i) {
      fx[i] = (float)vx[i];
      fy[i] = (float)vy[i];
      fz[i] = (float)vz[i];
    }
    HIP_TRY(c, hipMemcpyAsync(c->fx.p, fx.data(), tot * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->fy.p, fy.data(), tot * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->fz.p, fz.data(), tot * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return HCAO_OK;
  }
  HIP_TRY(c, hipMemcpyAsync(c->vx.p, vx.data(), tot * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->vy.p, vy.data(), tot * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->vz.p, vz.data(), tot * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return HCAO_OK;
}

// Workgroups of the step kernel: runs of consecutive cells of at most
// kMaxGroupCells cells (fewer when the per-cell LDS records of a wide
// workgroup would not fit) and about group_slots slots each. Workgroup w
// takes cells [grp[2w], grp[2w+1]) and work-list entries [grp_work[2w],
// grp_work[2w+1]) (cap/2 + 1 per cell). Workgroups are dispatched longest
// first (by slot capacity), so that the largest cells start earliest.
hcao_status build_groups(hcao_ctx *c) {
  const uint32_t nc = c->cfg.n_cells;
  uint32_t cell_limit = kMaxGroupCells;
  while (cell_limit > 0 && step_lds_bytes(c->tab, cell_limit, c->block) > kLdsBudget) --cell_limit;
  if (cell_limit == 0) return fail(c, HCAO_EUNSUPPORTED, "step kernel LDS budget exceeded");
  struct G {
    uint32_t c0, c1;
    uint64_t w0, w1, slots;
  };
  std::vector<G> groups;
  uint64_t slots = 0, wsum = 0, w0 = 0;
  uint32_t in_group = 0, max_cells = 1, first = 0;
  for (uint32_t i = 0; i < nc; ++i) {
    if (in_group > 0 && (in_group >= cell_limit || slots + c->cap_host[i] > c->group_slots)) {
      groups.push_back(G{first, i, w0, wsum, slots});
      max_cells = std::max(max_cells, in_group);
      in_group = 0;
      slots = 0;
      first = i;
      w0 = wsum;
    }
    ++in_group;
    slots += c->cap_host[i];
    wsum += c->cap_host[i] / 2 + 1;
  }
  groups.push_back(G{first, nc, w0, wsum, slots});
  max_cells = std::max(max_cells, in_group);
  std::stable_sort(groups.begin(), groups.end(), [](const G &x, const G &y) { return x.slots > y.slots; });
  std::vector<uint32_t> grp;
  std::vector<uint64_t> gw;
  for (const G &g : groups) {
    grp.push_back(g.c0);
    grp.push_back(g.c1);
    gw.push_back(g.w0);
    gw.push_back(g.w1);
  }
  c->n_groups = (uint32_t)groups.size();
  c->max_group_cells = max_cells;
  ++c->shape_gen;
  HIP_TRY(c, c->grp.alloc(grp.size()));
  HIP_TRY(c, c->grp_work.alloc(gw.size()));
  if (c->work_entries != wsum) {
    HIP_TRY(c, c->work.alloc((uint64_t)kWorkWords * wsum));  // the pairs as found, then sorted
    HIP_TRY(c, c->bflag.alloc(wsum));
    if (c->mixed) HIP_TRY(c, c->wdef.alloc(wsum));
    if (c->tab.has_recomb) HIP_TRY(c, c->tdelta.alloc(5 * wsum));
    c->work_entries = wsum;
  }
  HIP_TRY(c, hipMemcpyAsync(c->grp.p, grp.data(), grp.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->grp_work.p, gw.data(), gw.size() * 8, hipMemcpyHostToDevice, c->stream));
  c->step_lds = step_lds_bytes(c->tab, c->max_group_cells, c->block);
  if (c->step_lds > kLdsBudget) return fail(c, HCAO_EUNSUPPORTED, "step kernel LDS budget exceeded");
  return HCAO_OK;
}

// the mover list and its sort buffers for up to n entries (movers plus
// admissions), and the scan scratch for every scan of the re-bin
hipError_t grow_list(hcao_ctx *c, uint64_t n) {
  hipError_t e;
  if (n > c->list_cap) {
    if ((e = c->mv_mkey.alloc(n)) != hipSuccess) return e;
    if ((e = c->mv_mslot.alloc(n)) != hipSuccess) return e;
    if ((e = c->mv_sidx.alloc(n)) != hipSuccess) return e;
    if ((e = c->mv_sidx_tmp.alloc(n)) != hipSuccess) return e;
    if ((e = c->mv_ktmp.alloc(n)) != hipSuccess) return e;
    if ((e = c->mv_hist.alloc(sort_hist_entries(n))) != hipSuccess) return e;
    if ((e = c->mv_offs.alloc(sort_hist_entries(n))) != hipSuccess) return e;
    c->list_cap = n;
  }
  const uint64_t faces = (uint64_t)c->face_base[6] * c->species.size();
  const size_t need = std::max({scan_tmp_entries(sort_hist_entries(c->list_cap)),
                                scan_tmp_entries((uint64_t)c->cfg.n_cells + 1), scan_tmp_entries(faces + 1)});
  if (c->mv_stmp.n < need && (e = c->mv_stmp.alloc(need)) != hipSuccess) return e;
  return hipSuccess;
}

// a new particle state starts the inflow remainders and flux counts afresh
hipError_t reset_inflow(hcao_ctx *c) {
  hipError_t e;
  if (!c->open_faces) return hipSuccess;
  if ((e = hipMemsetAsync(c->in_rem.p, 0, c->in_rem.n * sizeof(double), c->stream)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(c->in_count.p, 0, c->in_count.n * sizeof(uint32_t), c->stream)) != hipSuccess) return e;
  return hipMemsetAsync(c->flux.p, 0, 2 * sizeof(unsigned long long), c->stream);
}

// staging for n admissions (state arrays of the context's precision)
hipError_t grow_ins(hcao_ctx *c, uint64_t n) {
  if (n <= c->ins_cap) return hipSuccess;
  const uint64_t cap = n + n / 4 + 1024;
  const uint32_t mm = c->max_modes ? c->max_modes : 1;
  release_ins(c);
  hipError_t e;
  if ((e = alloc_vel(c, c->ivx, c->ivy, c->ivz, c->ifx, c->ify, c->ifz, cap)) != hipSuccess) return e;
  if ((e = c->isp.alloc(cap)) != hipSuccess) return e;
  if ((e = c->ilvl.alloc(cap * level_row(mm))) != hipSuccess) return e;
  if (c->tab.has_rot && (e = c->irot.alloc(cap)) != hipSuccess) return e;
  if ((e = c->ipx.alloc(cap)) != hipSuccess) return e;
  if ((e = c->ipy.alloc(cap)) != hipSuccess) return e;
  if ((e = c->ipz.alloc(cap)) != hipSuccess) return e;
  c->ins_cap = cap;
  return hipSuccess;
}

// Allocates the particle state and its products staging for per-cell counts
// (capacities from caps, else the default headroom) and sets the offsets.
hcao_status alloc_state(hcao_ctx *c, const std::vector<uint32_t> &counts,
                        const std::vector<uint32_t> *caps = nullptr) {
  free_state(c);
  const uint32_t nc = c->cfg.n_cells;
  c->cap_host.assign(nc, 0);
  c->off_host.assign(nc + 1, 0);
  uint64_t tot = 0;
  for (uint32_t i = 0; i < nc; ++i) {
    const uint32_t cp = caps ? (*caps)[i] : default_cap(c, counts[i]);
    if (counts[i] > cp) return fail(c, HCAO_ECAPACITY, "cell " + std::to_string(i) + " exceeds its capacity");
    c->cap_host[i] = cp;
    c->off_host[i] = tot;
    tot += cp;
  }
  c->off_host[nc] = tot;
  c->total_slots = tot;
  // the spatial re-bin keeps old slots as 32-bit indices
  if (c->spatial && tot > 0xFFFFFFFFull) return fail(c, HCAO_EINVAL, "spatial mode holds at most 2^32 - 1 slots");
  const uint32_t mm = c->max_modes ? c->max_modes : 1;
  HIP_TRY(c, alloc_vel(c, c->vx, c->vy, c->vz, c->fx, c->fy, c->fz, tot));
  HIP_TRY(c, c->sp.alloc(tot));
  HIP_TRY(c, c->lvl.alloc(tot * level_row(mm)));
  if (c->tab.has_rot) {
    HIP_TRY(c, c->rot.alloc(tot));
    HIP_TRY(c, c->brot.alloc(tot));
    HIP_TRY(c, hipMemsetAsync(c->rot.p, 0, tot * sizeof(double), c->stream));
  }
  if (c->spatial) {
    HIP_TRY(c, c->px.alloc(tot));
    HIP_TRY(c, c->py.alloc(tot));
    HIP_TRY(c, c->pz.alloc(tot));
    HIP_TRY(c, c->bpx.alloc(tot));
    HIP_TRY(c, c->bpy.alloc(tot));
    HIP_TRY(c, c->bpz.alloc(tot));
    HIP_TRY(c, c->mv_key.alloc(tot));
    HIP_TRY(c, c->mv_list.alloc(tot));
    HIP_TRY(c, grow_list(c, tot));
    HIP_TRY(c, c->mv_packed.alloc(nc + 1));
    HIP_TRY(c, c->mv_dest.alloc(nc));
    HIP_TRY(c, c->mv_nstay.alloc(nc));
    HIP_TRY(c, c->mv_nmove.alloc(nc + 1));
    HIP_TRY(c, c->mv_mbase.alloc(nc + 1));
    // the entry past the last cell stays zero, so the scan's last output is
    // the number of movers
    HIP_TRY(c, hipMemsetAsync(c->mv_nmove.p, 0, (nc + 1) * sizeof(uint32_t), c->stream));
    release_ins(c);
    HIP_TRY(c, reset_inflow(c));
  }
  HIP_TRY(c, c->off.alloc(nc + 1));
  HIP_TRY(c, c->cnt.alloc(nc));
  HIP_TRY(c, c->cap.alloc(nc));
  HIP_TRY(c, c->d_volume.alloc(nc));
  HIP_TRY(c, c->d_weight.alloc(nc));
  HIP_TRY(c, c->sgmax.alloc(nc));
  HIP_TRY(c, c->rem.alloc(nc));
  HIP_TRY(c, c->defect.alloc(nc));
  if (c->tab.has_recomb) HIP_TRY(c, c->tsum.alloc(5 * (size_t)nc));
  HIP_TRY(c, c->ctr.alloc((size_t)nc * kNumCtr));
  HIP_TRY(c, hipMemsetAsync(c->defect.p, 0, nc * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->lvl.p, 0, tot * level_row(mm) * sizeof(uint16_t), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->ctr.p, 0, (size_t)nc * kNumCtr * sizeof(unsigned long long), c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->off.p, c->off_host.data(), (nc + 1) * sizeof(uint64_t), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->cap.p, c->cap_host.data(), nc * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->cnt.p, counts.data(), nc * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_volume.p, c->volume.data(), nc * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_weight.p, c->weight.data(), nc * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  // products staging (indexed like the state)
  HIP_TRY(c, alloc_vel(c, c->bvx, c->bvy, c->bvz, c->bfx, c->bfy, c->bfz, tot));
  HIP_TRY(c, c->bsp.alloc(tot));
  HIP_TRY(c, c->blvl.alloc(tot * level_row(mm)));
  if (hcao_status st = build_groups(c)) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return HCAO_OK;
}

hcao_status check_sticky(hcao_ctx *c) {
  if (!c) return HCAO_EINVAL;
  return c->sticky;
}

hcao_status read_err(hcao_ctx *c) {
  uint32_t e = 0;
  HIP_TRY(c, hipMemcpyAsync(&e, c->err.p, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (e & kErrBounds) {
    c->sticky = HCAO_EBOUNDS;
    return fail(c, HCAO_EBOUNDS, "a kernel index left its array (bounds-checked build)");
  }
  if (e & kErrCapacity) {
    c->sticky = HCAO_ECAPACITY;
    return fail(c, HCAO_ECAPACITY, "a cell exceeded its slot capacity");
  }
  return HCAO_OK;
}

// Eq. recomb-correct on the device for species sp of the device tables:
// every level combination below de is enumerated (count pass, scan, write
// pass), then one workgroup per temperature sums the records. p[i] receives
// the probability at t[i]; ms and n_rec (may be null) the device time and
// the number of records.
hcao_status exact_rec_probability(hcao_ctx *c, uint32_t sp, double de, double omega, uint32_t n_t, const double *t,
                                  double *p, double *ms, uint64_t *n_rec) {
  const SpeciesTab &S = c->tab.sp[sp];
  const uint32_t nm = S.n_modes;
  if (nm == 0 || !(de > 0.0) || !(omega >= 0.5 && omega < 1.5)) return fail(c, HCAO_EINVAL, "bad exact recombination input");
  RecEnumArgs ea{};
  ea.tab = c->d_tab.p;
  ea.lev = c->d_lev.p;
  ea.species = sp;
  ea.de = de;
  // box of the prefix modes: the levels below de and the first one above
  uint32_t box[kMaxModes];
  size_t n_sl = 0;
  for (uint32_t m = 0; m < nm; ++m) {
    uint32_t below = 0;
    if (m < S.n_bend) {
      while (((double)below + 0.5) * S.kt[m] - 0.5 * S.kt[m] < de) ++below;
      box[m] = below + 1;
    } else {
      const double *L = c->lev_host.data() + S.lev_off[m];
      while (below <= S.idiss[m] && L[below] - L[0] < de) ++below;
      box[m] = std::min(below + 1, S.idiss[m] + 1);
      n_sl += S.idiss[m] + 1;
    }
  }
  if (n_sl * sizeof(double) > kLdsBudget) return fail(c, HCAO_EUNSUPPORTED, "stretch ladders too long for the exact sum");
  uint64_t n_prefix = 1;
  uint32_t np = 0;
  while (np < nm && n_prefix * box[np] <= (1ull << 22)) n_prefix *= box[np++];
  if (np == 0) {
    np = 1;
    n_prefix = box[0];
  }
  ea.n_prefix_modes = np;
  for (uint32_t m = 0; m < np; ++m) ea.box[m] = box[m];
  ea.n_prefix = n_prefix;
  DevBuf<uint32_t> cnt;
  DevBuf<uint64_t> off;
  DevBuf<double> rec_e, d_t, d_num, d_den;
  DevBuf<uint32_t> rec_code;
  HIP_TRY(c, cnt.alloc(n_prefix));
  HIP_TRY(c, off.alloc(n_prefix));
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  HIP_TRY(c, hipEventRecord(e0, c->stream));
  ea.count = cnt.p;
  HIP_TRY(c, launch_rec_enum(ea, false, c->stream));
  DevBuf<uint64_t> stmp;
  HIP_TRY(c, stmp.alloc(scan_tmp_entries(n_prefix)));
  HIP_TRY(c, launch_scan_u32(cnt.p, off.p, n_prefix, stmp.p, c->stream));
  uint64_t last_off = 0;
  uint32_t last_cnt = 0;
  HIP_TRY(c, hipMemcpyAsync(&last_off, off.p + (n_prefix - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&last_cnt, cnt.p + (n_prefix - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const uint64_t total = last_off + last_cnt;
  HIP_TRY(c, rec_e.alloc(total));
  HIP_TRY(c, rec_code.alloc(total));
  ea.offset = off.p;
  ea.rec_e = rec_e.p;
  ea.rec_code = rec_code.p;
  HIP_TRY(c, launch_rec_enum(ea, true, c->stream));
  HIP_TRY(c, d_t.alloc(n_t));
  HIP_TRY(c, d_num.alloc(n_t));
  HIP_TRY(c, d_den.alloc(n_t));
  HIP_TRY(c, hipMemcpyAsync(d_t.p, t, n_t * sizeof(double), hipMemcpyHostToDevice, c->stream));
  RecSumArgs sa{};
  sa.tab = c->d_tab.p;
  sa.lev = c->d_lev.p;
  sa.species = sp;
  sa.de = de;
  sa.a = 2.5 - omega;
  sa.lgamma_a = std::lgamma(sa.a);
  sa.t = d_t.p;
  sa.rec_e = rec_e.p;
  sa.rec_code = rec_code.p;
  sa.n_rec = total;
  sa.num = d_num.p;
  sa.den = d_den.p;
  HIP_TRY(c, launch_rec_sum(sa, n_t, std::max<size_t>(n_sl, 1) * sizeof(double), c->stream));
  HIP_TRY(c, hipEventRecord(e1, c->stream));
  std::vector<double> num(n_t), den(n_t);
  HIP_TRY(c, hipMemcpyAsync(num.data(), d_num.p, n_t * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(den.data(), d_den.p, n_t * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float el = 0.0f;
  HIP_TRY(c, hipEventElapsedTime(&el, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (uint32_t i = 0; i < n_t; ++i) p[i] = num[i] / den[i];
  if (ms) *ms = el;
  if (n_rec) *n_rec = total;
  return HCAO_OK;
}

// k_b / <sigma g>_BC of a recombination reaction on the log-T nodes, per
// third-body species (appended to out); exact holds the device's Eq.
// recomb-correct probabilities per (A, third body) exponent, if any
void build_recombination_table(const hcao_ctx *c, const hcao_reaction_desc &d, const Tables &T,
                               std::vector<double> &out, const std::vector<std::pair<double, std::vector<double>>> &exact) {
  const SpeciesHost &B = c->species[d.reactant[0]], &C = c->species[d.reactant[1]], &A = c->species[d.product[0]];
  const host::ModeSet ma = modes_of(A), mb = modes_of(B), mc = modes_of(C);
  host::Recombination r{};
  r.a = &ma;
  r.b = &mb;
  r.c = &mc;
  r.mass_a = A.d.mass_kg;
  r.mass_b = B.d.mass_kg;
  r.mass_c = C.d.mass_kg;
  r.formation_a = A.d.formation_J;
  r.formation_b = B.d.formation_J;
  r.formation_c = C.d.formation_J;
  r.zpe_a = A.zpe;
  r.zpe_b = B.zpe;
  r.zpe_c = C.zpe;
  r.dref_a = A.d.dref_m;
  r.omega_a = A.d.omega;
  r.tref_a = A.d.Tref_K;
  const PairTab &bc = T.pr[d.reactant[0]][d.reactant[1]];
  r.bc_dref = (B.d.dref_m + C.d.dref_m) * 0.5;
  r.bc_tref = (B.d.Tref_K + C.d.Tref_K) * 0.5;
  r.bc_esg = bc.esg;
  r.bc_mr = bc.mr;
  uint32_t bond = 0;  // the first stretch the reaction names
  while (!((d.stretch_mask >> bond) & 1ull)) ++bond;
  r.de = A.de[bond];
  r.n_samp = d.n_samp ? d.n_samp : 1000;
  r.self = (uint32_t)d.product[0];
  for (const SpeciesHost &M : c->species) {
    r.m_dref.push_back(M.d.dref_m);
    r.m_omega.push_back(M.d.omega);
    r.m_tref.push_back(M.d.Tref_K);
    r.m_mass.push_back(M.d.mass_kg);
  }
  r.exact = &exact;
  host::recombination_factors(r, T.rec_l0, T.rec_inv_step, kRecNodes, out);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *hcao_status_string(hcao_status s) {
  switch (s) {
    case HCAO_OK: return "ok";
    case HCAO_EINVAL: return "invalid argument";
    case HCAO_ESTATE: return "call out of order";
    case HCAO_ENOMEM: return "out of memory";
    case HCAO_EDEVICE: return "HIP runtime error";
    case HCAO_ECAPACITY: return "cell capacity exceeded";
    case HCAO_ELEVEL: return "invalid quantum number";
    case HCAO_ENONFINITE: return "non-finite velocity";
    case HCAO_EUNSUPPORTED: return "unsupported feature";
    case HCAO_EBOUNDS: return "index outside its array (bounds-checked build)";
  }
  return "unknown status";
}

const char *hcao_last_error(const hcao_ctx *ctx) { return ctx ? ctx->last_error.c_str() : g_create_error.c_str(); }

hcao_status hcao_create(const hcao_config *cfg, hcao_ctx **out) {
  if (!cfg || !out) return HCAO_EINVAL;
  if (cfg->abi_version != HCAO_ABI_VERSION) return HCAO_EINVAL;
  if (cfg->n_cells == 0 || !cfg->cell_volume || !cfg->cell_weight) return HCAO_EINVAL;
  if (cfg->precision != HCAO_FP64 && cfg->precision != HCAO_MIXED) return HCAO_EINVAL;
  for (uint32_t i = 0; i < cfg->n_cells; ++i)
    if (!(cfg->cell_volume[i] > 0.0) || !(cfg->cell_weight[i] > 0.0) || !std::isfinite(cfg->cell_volume[i]) ||
        !std::isfinite(cfg->cell_weight[i]))
      return HCAO_EINVAL;
  hcao_ctx *c = new (std::nothrow) hcao_ctx();
  if (!c) return HCAO_ENOMEM;
  c->cfg = *cfg;
  c->mixed = cfg->precision == HCAO_MIXED;
  c->volume.assign(cfg->cell_volume, cfg->cell_volume + cfg->n_cells);
  c->weight.assign(cfg->cell_weight, cfg->cell_weight + cfg->n_cells);
  c->cfg.cell_volume = nullptr;
  c->cfg.cell_weight = nullptr;
  c->device = cfg->device;
  c->stream = (hipStream_t)cfg->hip_stream;
  if (const char *b = std::getenv("HCAO_BLOCK")) {
    const int v = std::atoi(b);
    if (v == 64 || v == 128 || v == 256 || v == 512) c->block = v;
  }
  if (const char *k = std::getenv("HCAO_STEPS_PER_LAUNCH")) {
    const long v = std::atol(k);
    if (v >= 1) c->steps_per_launch = (uint32_t)std::min<long>(v, 1L << 30);
  }
  if (const char *g = std::getenv("HCAO_GROUP_SLOTS")) {
    const long v = std::atol(g);
    if (v >= 1 && v <= (1L << 30)) c->group_slots = (uint32_t)v;
  }
  const char *step = "hipSetDevice";
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = lookup_static_scratch(c->device), step = "hipGetSymbolAddress";
  if (e == hipSuccess) e = hipEventCreate(&c->ev0), step = "hipEventCreate";
  if (e == hipSuccess) e = hipEventCreate(&c->ev1), step = "hipEventCreate";
  if (e == hipSuccess) e = c->err.alloc(1), step = "hipMalloc";
  if (e == hipSuccess) e = hipMemsetAsync(c->err.p, 0, sizeof(uint32_t), c->stream), step = "hipMemsetAsync";
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream), step = "hipStreamSynchronize";
  if (e != hipSuccess) {
    g_create_error = std::string(step) + ": " + hipGetErrorString(e);
    delete c;
    return HCAO_EDEVICE;
  }
  g_create_error.clear();
  *out = c;
  return HCAO_OK;
}

hcao_status hcao_add_species(hcao_ctx *c, const hcao_species_desc *d, int32_t *id) {
  if (!c || !d) return HCAO_EINVAL;
  if (c->finalized) return fail(c, HCAO_ESTATE, "add_species after finalize");
  if (c->species.size() >= (size_t)kMaxSpecies) return fail(c, HCAO_EINVAL, "too many species");
  if (!(d->mass_kg > 0.0) || !(d->dref_m > 0.0) || !(d->Tref_K > 0.0) || !(d->omega >= 0.5) || !(d->omega < 1.5))
    return fail(c, HCAO_EINVAL, "bad mass or VHS parameters");
  if (d->n_bend + d->n_stretch > (uint32_t)kMaxModes) return fail(c, HCAO_EINVAL, "too many modes");
  if (!(d->p_vib >= 0.0) || !(d->p_vib <= 1.0)) return fail(c, HCAO_EINVAL, "p_vib outside [0,1]");
  if (!(d->zeta_rot == 0 || d->zeta_rot == 2 || d->zeta_rot == 3))
    return fail(c, HCAO_EINVAL, "zeta_rot must be 0, 2 or 3");
  if (d->zeta_rot && (!(d->p_rot >= 0.0) || !(d->p_rot <= 1.0))) return fail(c, HCAO_EINVAL, "p_rot outside [0,1]");
  SpeciesHost s;
  s.d = *d;
  s.d.bend_theta_K = nullptr;
  s.d.omega_e_per_m = s.d.chi_e = s.d.De_J = nullptr;
  s.d.n_levels = nullptr;
  s.d.levels_J = nullptr;
  for (uint32_t j = 0; j < d->n_bend; ++j) {
    if (!d->bend_theta_K || !(d->bend_theta_K[j] > 0.0)) return fail(c, HCAO_EINVAL, "bend needs Theta > 0");
    s.theta.push_back(d->bend_theta_K[j]);
  }
  const double *lv = d->levels_J;
  for (uint32_t j = 0; j < d->n_stretch; ++j) {
    const uint32_t ne = d->n_levels ? d->n_levels[j] : 0;
    std::vector<double> L;
    double de_out = 0.0;
    hcao_status st = build_stretch(c, d->omega_e_per_m ? d->omega_e_per_m[j] : 0.0, d->chi_e ? d->chi_e[j] : 0.0,
                                   d->De_J ? d->De_J[j] : 0.0, ne, lv, L, de_out);
    if (st) return st;
    if (lv) lv += ne;
    s.levels.push_back(L);
    s.de.push_back(de_out);
  }
  s.n_modes = d->n_bend + d->n_stretch;
  double z = 0.0;
  for (uint32_t m = 0; m < s.n_modes; ++m) z = z + host_mode_energy(s, m, 0);
  s.zpe = z;
  if (d->sampler == HCAO_SAMPLER_AUTO)
    s.sampler = (s.n_modes >= 2 && s.n_modes <= 4) ? HCAO_SAMPLER_JOINT : HCAO_SAMPLER_GIBBS;
  else if (d->sampler == HCAO_SAMPLER_JOINT || d->sampler == HCAO_SAMPLER_GIBBS || d->sampler == HCAO_SAMPLER_EXACT)
    s.sampler = d->sampler;
  else
    return fail(c, HCAO_EINVAL, "unknown sampler");
  c->species.push_back(s);
  c->max_modes = std::max(c->max_modes, s.n_modes);
  if (id) *id = (int32_t)c->species.size() - 1;
  return HCAO_OK;
}

hcao_status hcao_add_reaction(hcao_ctx *c, const hcao_reaction_desc *d, int32_t *id) {
  if (!c || !d) return HCAO_EINVAL;
  if (c->finalized) return fail(c, HCAO_ESTATE, "add_reaction after finalize");
  if (c->reactions.size() >= (size_t)kMaxReactions) return fail(c, HCAO_EINVAL, "too many reactions");
  if (!(d->gamma_rot >= 0.0) || !(d->gamma_rot <= 1.0)) return fail(c, HCAO_EINVAL, "gamma_rot outside [0,1]");
  if (d->kind == HCAO_RX_RECOMBINATION && d->gamma_rot != 0.0)
    return fail(c, HCAO_EINVAL, "gamma_rot applies to dissociation and exchange");
  if (d->rec_model != HCAO_REC_WR && d->rec_model != HCAO_REC_EXACT) return fail(c, HCAO_EINVAL, "unknown recombination model");
  const int ns = (int)c->species.size();
  auto ok = [&](int s) { return s >= 0 && s < ns; };
  ReactionHost r;
  r.d = *d;
  r.d.alpha = nullptr;
  if (d->kind == HCAO_RX_DISSOCIATION) {
    if (!ok(d->reactant[0]) || !ok(d->product[0]) || !ok(d->product[1]))
      return fail(c, HCAO_EINVAL, "bad dissociation species");
    const SpeciesHost &A = c->species[d->reactant[0]];
    const uint32_t nst = A.d.n_stretch;
    if (nst == 0 || d->stretch_mask == 0 || (nst < 64 && (d->stretch_mask >> nst) != 0))
      return fail(c, HCAO_EINVAL, "stretch mask must name stretches of A");
    const double msum = c->species[d->product[0]].d.mass_kg + c->species[d->product[1]].d.mass_kg;
    if (std::fabs(msum - A.d.mass_kg) > 1e-9 * A.d.mass_kg) return fail(c, HCAO_EINVAL, "m_A != m_B + m_C");
  } else if (d->kind == HCAO_RX_EXCHANGE) {
    if (!ok(d->reactant[0]) || !ok(d->reactant[1]) || !ok(d->product[0]) || !ok(d->product[1]))
      return fail(c, HCAO_EINVAL, "bad exchange species");
    if (!(d->steric >= 0.0) || !(d->steric <= 1.0) || !(d->Ea_J >= 0.0))
      return fail(c, HCAO_EINVAL, "steric in [0,1] and Ea >= 0 required");
    const double m_in = c->species[d->reactant[0]].d.mass_kg + c->species[d->reactant[1]].d.mass_kg;
    const double m_out = c->species[d->product[0]].d.mass_kg + c->species[d->product[1]].d.mass_kg;
    if (std::fabs(m_in - m_out) > 1e-9 * m_in) return fail(c, HCAO_EINVAL, "exchange does not conserve mass");
    const uint32_t nm = c->species[d->reactant[0]].n_modes;
    for (uint32_t m = 0; m < nm; ++m) {
      const double a = d->alpha ? d->alpha[m] : 0.0;
      if (!(a >= 0.0) || !(a <= 1.0)) return fail(c, HCAO_EINVAL, "alpha outside [0,1]");
      r.alpha.push_back(a);
    }
  } else if (d->kind == HCAO_RX_RECOMBINATION) {
    const int b = d->reactant[0], cc = d->reactant[1], a = d->product[0];
    if (!ok(a) || !ok(b) || !ok(cc) || b == cc) return fail(c, HCAO_EINVAL, "bad recombination species");
    const SpeciesHost &A = c->species[a];
    const uint32_t nst = A.d.n_stretch;
    if (nst == 0 || d->stretch_mask == 0 || (nst < 64 && (d->stretch_mask >> nst) != 0))
      return fail(c, HCAO_EINVAL, "stretch mask must name stretches of A");
    const double msum = c->species[b].d.mass_kg + c->species[cc].d.mass_kg;
    if (std::fabs(msum - A.d.mass_kg) > 1e-9 * A.d.mass_kg) return fail(c, HCAO_EINVAL, "m_A != m_B + m_C");
  } else {
    return fail(c, HCAO_EINVAL, "unknown reaction kind");
  }
  c->reactions.push_back(r);
  if (id) *id = (int32_t)c->reactions.size() - 1;
  return HCAO_OK;
}

hcao_status hcao_finalize(hcao_ctx *c) {
  if (!c) return HCAO_EINVAL;
  if (c->finalized) return fail(c, HCAO_ESTATE, "finalize called twice");
  if (c->species.empty()) return fail(c, HCAO_EINVAL, "no species");
  Tables &T = c->tab;
  std::memset(&T, 0, sizeof(T));
  T.n_species = (uint32_t)c->species.size();
  T.n_reactions = (uint32_t)c->reactions.size();
  T.max_modes = c->max_modes;
  c->lev_host.clear();
  for (uint32_t s = 0; s < T.n_species; ++s) {
    const SpeciesHost &h = c->species[s];
    SpeciesTab &S = T.sp[s];
    S.mass = h.d.mass_kg;
    S.zpe = h.zpe;
    S.formation = h.d.formation_J;
    S.p_vib = h.d.p_vib;
    S.zeta_rot = h.d.zeta_rot;
    S.p_rot = h.d.zeta_rot ? h.d.p_rot : 0.0;
    if (S.zeta_rot) T.has_rot = 1;
    S.n_modes = h.n_modes;
    S.n_bend = h.d.n_bend;
    S.sampler = (uint32_t)h.sampler;
    for (uint32_t b = 0; b < h.d.n_bend; ++b) {
      S.theta[b] = h.theta[b];
      S.kt[b] = kB * h.theta[b];
    }
    // bends have equal spacings; a stretch qualifies when its spacings never
    // grow (Morse levels), which the Gibbs proposal's envelope needs
    S.concave = 0;
    for (uint32_t b = 0; b < h.d.n_bend; ++b) S.concave |= 1u << b;
    for (uint32_t j = 0; j < h.d.n_stretch; ++j) {
      const uint32_t m = h.d.n_bend + j;
      S.lev_off[m] = (uint32_t)c->lev_host.size();
      S.idiss[m] = (uint32_t)h.levels[j].size() - 1;
      S.de[m] = h.de[j];
      const std::vector<double> &L = h.levels[j];
      bool spacing_shrinks = true;
      for (size_t i = 1; i + 1 < L.size(); ++i)
        if (!((L[i + 1] - L[i]) <= (L[i] - L[i - 1]))) spacing_shrinks = false;
      if (spacing_shrinks) S.concave |= 1u << m;
      c->lev_host.insert(c->lev_host.end(), h.levels[j].begin(), h.levels[j].end());
    }
  }
  T.n_levels = (uint32_t)c->lev_host.size();
  c->thermo.clear();
  for (const SpeciesHost &h : c->species) c->thermo.emplace_back(modes_of(h));
  // VHS pair constants: sigma g = C (g^2)^(1-w), C = pi d^2 (2 k T_ref / m_r)^(w-1/2) / Gamma(5/2-w),
  // mixed-pair d, w, T_ref as species means; LB exponent 3/2 - w
  for (uint32_t a = 0; a < T.n_species; ++a)
    for (uint32_t b = 0; b < T.n_species; ++b) {
      const hcao_species_desc &A = c->species[a].d, &B = c->species[b].d;
      PairTab &P = T.pr[a][b];
      const double msum = A.mass_kg + B.mass_kg;
      const double mr = (A.mass_kg * B.mass_kg) / msum;
      const double w = (A.omega + B.omega) * 0.5;
      const double d = (A.dref_m + B.dref_m) * 0.5;
      const double tr = (A.Tref_K + B.Tref_K) * 0.5;
      const double base = ((2.0 * kB) * tr) / mr;
      P.mr = mr;
      P.hm = 0.5 * mr;
      P.m_a = A.mass_kg;
      P.m_b = B.mass_kg;
      P.msum = msum;
      P.wa = B.mass_kg / msum;
      P.wb = A.mass_kg / msum;
      P.csg = ((kPi * (d * d)) * std::pow(base, w - 0.5)) / std::tgamma(2.5 - w);
      P.esg = 1.0 - w;
      P.q = 1.5 - w;
    }
  // pairs some reaction can involve; the step skips the reaction decision for the others
  for (uint32_t a = 0; a < T.n_species; ++a)
    for (uint32_t b = 0; b < T.n_species; ++b) {
      uint32_t react = 0;
      for (const ReactionHost &h : c->reactions) {
        const int32_t ra = h.d.reactant[0], rb = h.d.reactant[1];
        if (h.d.kind == HCAO_RX_DISSOCIATION) {
          if (ra == (int32_t)a || ra == (int32_t)b) react |= kReactAny;
        } else if ((ra == (int32_t)a && rb == (int32_t)b) || (ra == (int32_t)b && rb == (int32_t)a)) {
          react |= kReactAny;
          if (h.d.kind == HCAO_RX_RECOMBINATION) react |= kReactRecomb;
        }
      }
      T.pr[a][b].react = react;
      // channel bounds for the scan's skip test (scan order: dissociation of
      // a then b, exchange with a then b as A)
      PairBound &pb = T.pr[a][b].bound;
      pb.n_steric = 0;
      for (uint32_t side = 0; side < 2; ++side) {
        const uint32_t sa = side ? b : a, sb = side ? a : b;
        pb.dis_c[side] = -std::numeric_limits<double>::infinity();
        pb.ex_a[side] = -1.0;
        pb.ex_e[side] = std::numeric_limits<double>::infinity();
        const SpeciesHost &A = c->species[sa];
        for (const ReactionHost &h : c->reactions) {
          if (h.d.kind == HCAO_RX_DISSOCIATION && (uint32_t)h.d.reactant[0] == sa) {
            const double zsum = (A.zpe + c->species[h.d.product[0]].zpe) + c->species[h.d.product[1]].zpe;
            for (uint32_t j = 0; j < A.d.n_stretch; ++j)
              if ((h.d.stretch_mask >> j) & 1ull)
                pb.dis_c[side] = std::max(pb.dis_c[side], (A.levels[j][0] - A.de[j]) - zsum);
          } else if (h.d.kind == HCAO_RX_EXCHANGE && (uint32_t)h.d.reactant[0] == sa &&
                     (uint32_t)h.d.reactant[1] == sb) {
            ++pb.n_steric;
            double amax = 0.0;
            for (double x : h.alpha) amax = std::max(amax, x);
            pb.ex_a[side] = std::max(pb.ex_a[side], amax);
            pb.ex_e[side] = std::min(pb.ex_e[side], h.d.Ea_J);
          }
        }
      }
    }
  // exact sampler: one beta table per (species, LB exponent), shared by the
  // pairs that use it
  c->beta_host.clear();
  c->has_exact = false;
  for (uint32_t a = 0; a < T.n_species; ++a)
    if (T.sp[a].sampler == HCAO_SAMPLER_EXACT && T.sp[a].n_modes > 0) c->has_exact = true;
  for (uint32_t a = 0; a < T.n_species; ++a)
    for (uint32_t b = 0; b < T.n_species; ++b) {
      T.pr[a][b].beta_off = 0xFFFFFFFFu;
      if (T.sp[a].sampler != HCAO_SAMPLER_EXACT || T.sp[a].n_modes == 0) continue;
      for (uint32_t b2 = 0; b2 < b; ++b2)
        if (T.pr[a][b2].q == T.pr[a][b].q) T.pr[a][b].beta_off = T.pr[a][b2].beta_off;
      if (T.pr[a][b].beta_off != 0xFFFFFFFFu) continue;
      T.pr[a][b].beta_off = (uint32_t)c->beta_host.size();
      // exact sampler: beta per bin of E' (energy above the zero point), the
      // smallest grid value whose proposal mean energy plus q / beta is at
      // most the bin's midpoint (any beta samples the target exactly; this one
      // puts the acceptance near its peak)
      std::vector<double> kt(T.sp[a].kt, T.sp[a].kt + T.sp[a].n_bend);
      host::exact_beta_bins(kt, modes_of(c->species[a]), T.pr[a][b].q, kExactBinLo, kExactBinHi, kExactNBeta,
                            c->beta_host);
    }
  if (c->beta_host.empty()) c->beta_host.push_back(0.0);
  T.rec_nt = kRecNodes;
  T.rec_l0 = std::log(kRecTmin);
  T.rec_inv_step = (double)(kRecNodes - 1) / std::log(kRecTmax / kRecTmin);
  c->rec_host.clear();
  for (uint32_t r = 0; r < T.n_reactions; ++r) {
    const ReactionHost &h = c->reactions[r];
    ReactionTab &R = T.rx[r];
    R.kind = (int32_t)h.d.kind;
    R.mask = h.d.stretch_mask;
    R.gamma_rot = h.d.gamma_rot;
    if (h.d.kind == HCAO_RX_RECOMBINATION) {
      const int b = h.d.reactant[0], cc = h.d.reactant[1], a = h.d.product[0];
      R.a = b;
      R.b = cc;
      R.c = a;
      R.d = -1;
      R.dh = c->species[a].d.formation_J - (c->species[b].d.formation_J + c->species[cc].d.formation_J);
      R.rec_off = c->rec_host.size();
      T.has_recomb = 1;
      // Eq. recomb-correct on the device, one probability curve per omega of
      // the (A, third body) pairs
      std::vector<std::pair<double, std::vector<double>>> exact;
      if (h.d.rec_model == HCAO_REC_EXACT) {
        HIP_TRY(c, c->d_tab.alloc(1));
        HIP_TRY(c, c->d_lev.alloc(c->lev_host.size()));
        HIP_TRY(c, hipMemcpyAsync(c->d_tab.p, &T, sizeof(Tables), hipMemcpyHostToDevice, c->stream));
        if (!c->lev_host.empty())
          HIP_TRY(c, hipMemcpyAsync(c->d_lev.p, c->lev_host.data(), c->lev_host.size() * sizeof(double),
                                    hipMemcpyHostToDevice, c->stream));
        const SpeciesHost &A = c->species[a];
        uint32_t jb = 0;
        while (!((h.d.stretch_mask >> jb) & 1ull)) ++jb;
        std::vector<double> temps(kRecNodes);
        for (uint32_t i = 0; i < kRecNodes; ++i) temps[i] = std::exp(T.rec_l0 + (double)i / T.rec_inv_step);
        for (uint32_t m = 0; m < T.n_species; ++m) {
          const double w = (A.d.omega + c->species[m].d.omega) * 0.5;
          bool have = false;
          for (const auto &ex : exact) have = have || ex.first == w;
          if (have) continue;
          std::vector<double> pr(kRecNodes);
          const hcao_status st = exact_rec_probability(c, (uint32_t)a, A.de[jb], w, kRecNodes, temps.data(),
                                                       pr.data(), nullptr, nullptr);
          if (st) return st;
          exact.emplace_back(w, pr);
        }
      }
      build_recombination_table(c, h.d, T, c->rec_host, exact);
    } else if (h.d.kind == HCAO_RX_DISSOCIATION) {
      const int a = h.d.reactant[0], pc = h.d.product[0], pd = h.d.product[1];
      R.a = a;
      R.b = -1;
      R.c = pc;
      R.d = pd;
      R.dh = (c->species[pc].d.formation_J + c->species[pd].d.formation_J) - c->species[a].d.formation_J;
      R.zsum = (c->species[a].zpe + c->species[pc].zpe) + c->species[pd].zpe;
    } else {
      const int a = h.d.reactant[0], b = h.d.reactant[1], pc = h.d.product[0], pd = h.d.product[1];
      R.a = a;
      R.b = b;
      R.c = pc;
      R.d = pd;
      for (size_t m = 0; m < h.alpha.size(); ++m) R.alpha[m] = h.alpha[m];
      R.steric = h.d.steric;
      R.ea = h.d.Ea_J;
      R.dh = (c->species[pc].d.formation_J + c->species[pd].d.formation_J) -
             (c->species[a].d.formation_J + c->species[b].d.formation_J);
    }
  }
  HIP_TRY(c, c->d_tab.alloc(1));
  HIP_TRY(c, c->d_lev.alloc(c->lev_host.size()));
  HIP_TRY(c, c->d_rec.alloc(c->rec_host.size()));
  HIP_TRY(c, c->d_beta.alloc(c->beta_host.size()));
  HIP_TRY(c, hipMemcpyAsync(c->d_beta.p, c->beta_host.data(), c->beta_host.size() * sizeof(double),
                            hipMemcpyHostToDevice, c->stream));
  if (!c->rec_host.empty())
    HIP_TRY(c, hipMemcpyAsync(c->d_rec.p, c->rec_host.data(), c->rec_host.size() * sizeof(double),
                              hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_tab.p, &T, sizeof(Tables), hipMemcpyHostToDevice, c->stream));
  if (!c->lev_host.empty())
    HIP_TRY(c, hipMemcpyAsync(c->d_lev.p, c->lev_host.data(), c->lev_host.size() * sizeof(double),
                              hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, set_step_lds_limit(kLdsBudget));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->finalized = true;
  return HCAO_OK;
}

hcao_status hcao_load_particles(hcao_ctx *c, uint64_t n, const uint32_t *cell, const uint8_t *species,
                                const double *vel, const uint16_t *levels, const double *rot, const double *pos) {
  Range range("hcao_load_particles");
  if (!c) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
  if (!c->finalized) return fail(c, HCAO_ESTATE, "load before finalize");
  if (n && (!cell || !species || !vel || !levels)) return fail(c, HCAO_EINVAL, "null particle array");
  if (n > 0xFFFFFFFFull) return fail(c, HCAO_EINVAL, "too many particles");
  const uint32_t nc = c->cfg.n_cells, mm = c->max_modes ? c->max_modes : 1;
  if (rot) {
    for (uint64_t i = 0; i < n; ++i) {
      const bool rotor = species[i] < c->species.size() && c->species[species[i]].d.zeta_rot > 0;
      if (!(rot[i] >= 0.0) || !std::isfinite(rot[i]) || (rot[i] != 0.0 && !rotor))
        return fail(c, HCAO_EINVAL, "rotational energy must be finite, >= 0, and 0 without a rotor");
    }
  }
  DevBuf<double> d_pos;
  if (c->spatial) {
    if (n && !pos) return fail(c, HCAO_EINVAL, "the spatial mode needs positions");
    for (uint64_t i = 0; i < n; ++i) {
      uint32_t ijk[3];
      for (int k = 0; k < 3; ++k) {
        const double x = pos[3 * i + k];
        if (!(x >= 0.0) || !(x <= c->len[k])) return fail(c, HCAO_EINVAL, "position outside the box");
        const double f = std::floor(x / (c->len[k] / (double)c->grid[k]));
        ijk[k] = !(f >= 0.0) ? 0u : (f >= (double)c->grid[k] ? c->grid[k] - 1 : (uint32_t)f);
      }
      if (ijk[0] + c->grid[0] * (ijk[1] + c->grid[1] * ijk[2]) != cell[i])
        return fail(c, HCAO_EINVAL, "position not in the particle's cell");
    }
    HIP_TRY(c, d_pos.alloc(3 * n));
    if (n) HIP_TRY(c, hipMemcpyAsync(d_pos.p, pos, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  DevBuf<double> d_rot;
  if (rot && c->tab.has_rot) {
    HIP_TRY(c, d_rot.alloc(n));
    if (n) HIP_TRY(c, hipMemcpyAsync(d_rot.p, rot, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  DevBuf<uint32_t> d_cell, d_count, keys_tmp, idx, idx_tmp, hist;
  DevBuf<uint8_t> d_sp;
  DevBuf<double> d_vel;
  DevBuf<uint16_t> d_lvl;
  DevBuf<uint64_t> offs, packed;
  HIP_TRY(c, d_cell.alloc(n));
  HIP_TRY(c, d_sp.alloc(n));
  HIP_TRY(c, d_vel.alloc(3 * n));
  HIP_TRY(c, d_lvl.alloc(n * mm));
  HIP_TRY(c, d_count.alloc(nc));
  HIP_TRY(c, hipMemsetAsync(d_count.p, 0, nc * sizeof(uint32_t), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->err.p, 0, sizeof(uint32_t), c->stream));
  if (n) {
    HIP_TRY(c, hipMemcpyAsync(d_cell.p, cell, n * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_sp.p, species, n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_vel.p, vel, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_lvl.p, levels, n * mm * sizeof(uint16_t), hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(c, launch_load_check(c->d_tab.p, d_cell.p, d_sp.p, d_vel.p, d_lvl.p, n, nc, d_count.p, c->err.p,
                               c->stream));
  std::vector<uint32_t> counts(nc);
  uint32_t err = 0;
  HIP_TRY(c, hipMemcpyAsync(counts.data(), d_count.p, nc * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&err, c->err.p, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (err & kErrInvalid) return fail(c, HCAO_EINVAL, "particle with bad cell or species");
  if (err & kErrNonFinite) return fail(c, HCAO_ENONFINITE, "non-finite velocity");
  if (err & kErrLevel) return fail(c, HCAO_ELEVEL, "quantum number out of range");
  if (hcao_status s = alloc_state(c, counts)) return s;
  // stable counting sort by cell, then placement into the padded layout
  uint32_t key_bits = 0;
  while (key_bits < 32 && ((uint64_t)1 << key_bits) < nc) ++key_bits;
  HIP_TRY(c, keys_tmp.alloc(n));
  HIP_TRY(c, idx.alloc(n));
  HIP_TRY(c, idx_tmp.alloc(n));
  HIP_TRY(c, hist.alloc(sort_hist_entries(n)));
  HIP_TRY(c, offs.alloc(sort_hist_entries(n)));
  HIP_TRY(c, packed.alloc(nc));
  bool in_tmp = false;
  DevBuf<uint64_t> stmp;
  HIP_TRY(c, stmp.alloc(std::max(scan_tmp_entries(sort_hist_entries(n)), scan_tmp_entries(nc))));
  HIP_TRY(c, launch_sort(d_cell.p, idx.p, keys_tmp.p, idx_tmp.p, hist.p, offs.p, stmp.p, n, key_bits, c->stream,
                         in_tmp));
  HIP_TRY(c, launch_scan_u32(c->cnt.p, packed.p, nc, stmp.p, c->stream));
  const uint32_t *sk = in_tmp ? keys_tmp.p : d_cell.p;
  const uint32_t *si = in_tmp ? idx_tmp.p : idx.p;
  HIP_TRY(c, launch_place(c->d_tab.p, sk, si, packed.p, c->off.p, d_sp.p, d_vel.p, d_lvl.p, d_rot.p, d_pos.p,
                          state_of(c), n, c->stream));
  HIP_TRY(c, launch_cell_init(c->d_tab.p, state_of(c), cells_of(c), nc, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  d_cell.release();
  c->step = 0;
  c->loaded = true;
  return HCAO_OK;
}

hcao_status hcao_init_thermal(hcao_ctx *c, const uint32_t *counts, const double *t_trans, const double *t_vib) {
  Range range("hcao_init_thermal");
  if (!c || !counts || !t_trans || !t_vib) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
  if (!c->finalized) return fail(c, HCAO_ESTATE, "init before finalize");
  const uint32_t nc = c->cfg.n_cells, ns = (uint32_t)c->species.size();
  std::vector<uint32_t> per(nc, 0);
  for (uint32_t i = 0; i < nc; ++i) {
    uint64_t s = 0;
    for (uint32_t j = 0; j < ns; ++j) s += counts[(size_t)i * ns + j];
    if (s > 0xFFFFFFFFull) return fail(c, HCAO_EINVAL, "cell too large");
    per[i] = (uint32_t)s;
    if (!(t_trans[i] >= 0.0) || !(t_vib[i] >= 0.0) || !std::isfinite(t_trans[i]) || !std::isfinite(t_vib[i]))
      return fail(c, HCAO_EINVAL, "bad temperature");
  }
  if (hcao_status s = alloc_state(c, per)) return s;
  DevBuf<uint32_t> d_counts;
  DevBuf<double> d_tt, d_tv;
  HIP_TRY(c, d_counts.alloc((size_t)nc * ns));
  HIP_TRY(c, d_tt.alloc(nc));
  HIP_TRY(c, d_tv.alloc(nc));
  HIP_TRY(c, hipMemcpyAsync(d_counts.p, counts, (size_t)nc * ns * sizeof(uint32_t), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_tt.p, t_trans, nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_tv.p, t_vib, nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_init(c->d_tab.p, c->d_lev.p, state_of(c), c->off.p, d_counts.p, d_tt.p, d_tv.p, c->cfg.seed, nc,
                         c->grid, c->len, c->stream));
  HIP_TRY(c, launch_cell_init(c->d_tab.p, state_of(c), cells_of(c), nc, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->step = 0;
  c->loaded = true;
  return HCAO_OK;
}

namespace {

StepArgs step_args(hcao_ctx *c, double dt) {
  StepArgs a{};
  a.tab = c->d_tab.p;
  a.lev = c->d_lev.p;
  a.st = state_of(c);
  a.born = staging_of(c);
  a.cells = cells_of(c);
  a.err = c->err.p;
  a.seed = c->cfg.seed;
  a.dt = dt;
  a.rec = c->d_rec.p;
  a.beta = c->d_beta.p;
  a.grp = c->grp.p;
  a.grp_work = c->grp_work.p;
  a.work = c->work.p;
  a.bflag = c->bflag.p;
  a.wdef = c->wdef.p;
  a.tdelta = c->tab.has_recomb ? c->tdelta.p : nullptr;
  a.tdelta_stride = c->work_entries;
  a.clk = c->clk.p;
  return a;
}

// Issues the step-kernel launches of n_steps steps on stream s. With
// step_dev, the launches read their base step index from the device and a
// final kernel advances it; otherwise base is the first step's index.
// spatial mode: move every particle over dt, then re-bin all of them by a
// stable radix sort on the new cell into the staging buffers, which then
// become the state (the old state becomes the products staging)
hcao_status move_rebin(hcao_ctx *c, double dt, uint32_t step, hipStream_t s) {
  Range range("hcao_move_rebin");
  const uint32_t nc = c->cfg.n_cells, mm = c->max_modes ? c->max_modes : 1;
  const uint32_t ns = (uint32_t)c->species.size();
  const uint64_t tot = c->total_slots, faces = (uint64_t)c->face_base[6] * ns;
  HIP_TRY(c, grow_list(c, c->list_cap));  // scan scratch for open faces set after the load
  MoveArgs m{};
  m.st = state_of(c);
  m.off = c->off.p;
  m.cnt = c->cnt.p;
  m.cap = c->cap.p;
  m.n_cells = nc;
  m.nx = c->grid[0];
  m.ny = c->grid[1];
  m.nz = c->grid[2];
  m.periodic = c->periodic;
  m.open = c->open_faces;
  for (int k = 0; k < 3; ++k) m.len[k] = c->len[k];
  m.dt = dt;
  m.key = c->mv_key.p;
  m.list = c->mv_list.p;
  m.n_stay = c->mv_nstay.p;
  m.n_move = c->mv_nmove.p;
  m.flux = c->open_faces ? c->flux.p : nullptr;
  HIP_TRY(c, launch_move(m, s));
  HIP_TRY(c, launch_scan_u32(c->mv_nmove.p, c->mv_mbase.p, (uint64_t)nc + 1, c->mv_stmp.p, s));
  InflowArgs in{};
  if (c->open_faces) {
    in.tab = c->d_tab.p;
    in.lev = c->d_lev.p;
    in.weight = c->d_weight.p;
    in.rem = c->in_rem.p;
    in.count = c->in_count.p;
    in.ibase = c->in_base.p;
    in.mbase = c->mv_mbase.p;
    in.flux = c->flux.p;
    in.err = c->err.p;
    for (uint32_t k = 0; k < ns; ++k) in.flux_s[k] = c->in_flux[k];
    for (int k = 0; k < 3; ++k) in.len[k] = c->len[k];
    in.dt = dt;
    in.t_trans = c->in_t;
    in.t_vib = c->in_tv;
    in.seed = c->cfg.seed;
    in.tot = tot;
    for (int k = 0; k < 7; ++k) in.face_base[k] = c->face_base[k];
    in.nx = c->grid[0];
    in.ny = c->grid[1];
    in.nz = c->grid[2];
    in.n_cells = nc;
    in.periodic = c->periodic;
    in.open = c->open_faces;
    in.n_species = ns;
    in.step = step;
    HIP_TRY(c, launch_inflow_count(in, s));
    // the entry past the last (face cell, species) stays zero: the scan's
    // last output is the number of admissions
    HIP_TRY(c, launch_scan_u32(c->in_count.p, c->in_base.p, faces + 1, c->mv_stmp.p, s));
  }
  // the numbers of movers and admissions size the sort: one small read-back
  // per step
  uint64_t movers = 0, n_ins = 0;
  HIP_TRY(c, hipMemcpyAsync(&movers, c->mv_mbase.p + nc, sizeof movers, hipMemcpyDeviceToHost, s));
  if (c->open_faces) HIP_TRY(c, hipMemcpyAsync(&n_ins, c->in_base.p + faces, sizeof n_ins, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (n_ins) {
    if (tot + n_ins + n_ins / 4 + 1024 > 0xFFFFFFFFull)
      return fail(c, HCAO_ECAPACITY, "admissions of one step exceed the 32-bit slot range");
    HIP_TRY(c, grow_ins(c, n_ins));
  }
  HIP_TRY(c, grow_list(c, movers + n_ins));
  RebinArgs r{};
  r.src = state_of(c);
  r.dst = staging_of(c);
  r.ins = ins_state(c);
  r.tot = tot;
  r.off = c->off.p;
  r.cap = c->cap.p;
  r.key = c->mv_key.p;
  r.list = c->mv_list.p;
  r.n_stay = c->mv_nstay.p;
  r.n_move = c->mv_nmove.p;
  r.mbase = c->mv_mbase.p;
  r.mkey = c->mv_mkey.p;
  r.mslot = c->mv_mslot.p;
  r.packed = c->mv_packed.p;
  r.dest = c->mv_dest.p;
  r.cnt = c->cnt.p;
  r.err = c->err.p;
  r.m = movers + n_ins;
  r.m_real = movers;
  r.n_cells = nc;
  r.mm = mm;
  r.dt = dt;
  for (int k = 0; k < 3; ++k) r.len[k] = c->len[k];
  r.periodic = c->periodic;
  r.open = c->open_faces;
  HIP_TRY(c, launch_list_movers(r, s));
  if (n_ins) {
    in.ins = ins_state(c);
    in.cap_ins = c->ins_cap;
    in.n_ins = n_ins;
    in.mkey = c->mv_mkey.p;
    in.mslot = c->mv_mslot.p;
    HIP_TRY(c, launch_inflow_make(in, s));
  }
  // keys 0..nc-1, and nc for an admission that leaves again (it sorts last)
  const uint64_t top_key = c->open_faces ? nc : nc - 1;
  uint32_t key_bits = 0;
  while (key_bits < 32 && ((uint64_t)1 << key_bits) <= top_key) ++key_bits;
  bool in_tmp = false;
  HIP_TRY(c, launch_sort(c->mv_mkey.p, c->mv_sidx.p, c->mv_ktmp.p, c->mv_sidx_tmp.p, c->mv_hist.p, c->mv_offs.p,
                         c->mv_stmp.p, movers + n_ins, key_bits, s, in_tmp));
  r.skey = in_tmp ? c->mv_ktmp.p : c->mv_mkey.p;
  r.sidx = in_tmp ? c->mv_sidx_tmp.p : c->mv_sidx.p;
  r.slot = in_tmp ? c->mv_sidx.p : c->mv_sidx_tmp.p;  // the sort's other index buffer is free now
  HIP_TRY(c, launch_rebin_place(r, s));
  std::swap(c->vx, c->bvx);
  std::swap(c->vy, c->bvy);
  std::swap(c->vz, c->bvz);
  std::swap(c->fx, c->bfx);
  std::swap(c->fy, c->bfy);
  std::swap(c->fz, c->bfz);
  std::swap(c->sp, c->bsp);
  std::swap(c->lvl, c->blvl);
  std::swap(c->rot, c->brot);
  std::swap(c->px, c->bpx);
  std::swap(c->py, c->bpy);
  std::swap(c->pz, c->bpz);
  return HCAO_OK;
}

// which k_step instantiation a context needs: the exact sampler or rotors
// (2), positions only (1), or neither (0)
int step_level(const hcao_ctx *c) { return (c->has_exact || c->tab.has_rot) ? 2 : (c->spatial ? 1 : 0); }

// Where one step call keeps its work lists, pair flags, pair energy defects
// and products: the context's buffers, or the fixed device array.
struct StepScratch {
  uint32_t *work;
  uint8_t *bflag;
  double *wdef;
  double *tdelta;
  State born;
};

// Carves the allocation-free step's scratch out of the fixed array at base
// (256-byte aligned pieces, products staged per work entry); returns the
// bytes it needs.
uint64_t static_layout(const hcao_ctx *c, unsigned char *base, StepScratch &out) {
  const uint64_t w = c->work_entries;
  const uint32_t mm = c->max_modes ? c->max_modes : 1;
  uint64_t at = 0;
  auto take = [&](uint64_t bytes) {
    unsigned char *p = base + at;
    at += (bytes + 255) & ~uint64_t(255);
    return p;
  };
  out = StepScratch{};
  out.work = reinterpret_cast<uint32_t *>(take((uint64_t)kWorkWords * w * sizeof(uint32_t)));
  out.bflag = take(w);
  if (c->mixed) out.wdef = reinterpret_cast<double *>(take(w * sizeof(double)));
  if (c->tab.has_recomb) out.tdelta = reinterpret_cast<double *>(take(5 * w * sizeof(double)));
  State &b = out.born;
  if (c->mixed) {
    b.fx = reinterpret_cast<float *>(take(w * sizeof(float)));
    b.fy = reinterpret_cast<float *>(take(w * sizeof(float)));
    b.fz = reinterpret_cast<float *>(take(w * sizeof(float)));
  } else {
    b.vx = reinterpret_cast<double *>(take(w * sizeof(double)));
    b.vy = reinterpret_cast<double *>(take(w * sizeof(double)));
    b.vz = reinterpret_cast<double *>(take(w * sizeof(double)));
  }
  b.sp = take(w);
  set_slots(b, w);
  b.lrow = level_row(mm);
  b.lvl = reinterpret_cast<uint16_t *>(take(w * b.lrow * sizeof(uint16_t)));
  if (c->tab.has_rot) b.rot = reinterpret_cast<double *>(take(w * sizeof(double)));
  return at;
}

hcao_status issue_steps(hcao_ctx *c, double dt, uint32_t n_steps, uint32_t base, uint32_t *step_dev,
                        hipStream_t s, uint32_t *launches, const StepScratch *sc = nullptr) {
  if (c->spatial) {
    // one collision launch per step, each after the move and re-bin
    for (uint32_t d = 0; d < n_steps; ++d) {
      if (hcao_status st = move_rebin(c, dt, base + d, s)) return st;
      StepArgs a = step_args(c, dt);
      a.step = base + d;
      a.n_steps = 1;
      HIP_TRY(c, launch_step(a, c->step_lds, c->block, c->mixed, step_level(c), c->n_groups, s));
    }
    if (launches) *launches = n_steps;
    return HCAO_OK;
  }
  StepArgs a = step_args(c, dt);
  if (sc) {
    a.work = sc->work;
    a.bflag = sc->bflag;
    a.wdef = sc->wdef;
    a.tdelta = sc->tdelta;  // stride: work entries, as the context's own
    a.born = sc->born;
  }
  a.step_dev = step_dev;
  uint32_t n = 0;
  for (uint32_t done = 0; done < n_steps;) {
    const uint32_t k = std::min(n_steps - done, c->steps_per_launch);
    a.step = (step_dev ? 0u : base) + done;
    a.n_steps = k;
    HIP_TRY(c, launch_step(a, c->step_lds, c->block, c->mixed, step_level(c),
                           c->n_groups, s));
    done += k;
    ++n;
  }
  if (step_dev) HIP_TRY(c, launch_advance(step_dev, n_steps, s));
  if (launches) *launches = n;
  return HCAO_OK;
}

hcao_status timing_begin(hcao_ctx *c) {
  if (c->timing) HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  return HCAO_OK;
}

hcao_status timing_end(hcao_ctx *c, uint32_t launches, uint32_t n_steps) {
  if (!c->timing) return HCAO_OK;
  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  HIP_TRY(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  c->timed_ms += ms;
  c->timed_launches += launches;
  c->timed_steps += n_steps;
  return HCAO_OK;
}

hcao_status check_step_args(hcao_ctx *c, double dt) {
  if (!c) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "step before load");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, HCAO_EINVAL, "dt must be > 0");
  return HCAO_OK;
}

void drop_graph(hcao_ctx *c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_gen = ~0ull;
}

}  // namespace

hcao_status hcao_step(hcao_ctx *c, double dt, uint32_t n_steps) {
  Range range("hcao_step");
  if (hcao_status s = check_step_args(c, dt)) return s;
  if (hcao_status s = timing_begin(c)) return s;
  uint32_t launches = 0;
  if (hcao_status s = issue_steps(c, dt, n_steps, c->step, nullptr, c->stream, &launches)) return s;
  c->step += n_steps;
  return timing_end(c, launches, n_steps);
}

hcao_status hcao_step_static(hcao_ctx *c, double dt, uint32_t n_steps) {
  Range range("hcao_step_static");
  if (hcao_status s = check_step_args(c, dt)) return s;
  if (c->spatial)
    return fail(c, HCAO_EUNSUPPORTED,
                "the allocation-free step does not run the spatial mode (its re-bin needs buffers as large as the "
                "state)");
  unsigned char *base = static_cast<unsigned char *>(static_scratch(c->device));
  if (!base) return fail(c, HCAO_ESTATE, "the fixed scratch array has no address on this device");
  StepScratch sc;
  const uint64_t need = static_layout(c, base, sc);
  if (need > kStaticScratchBytes)
    return fail(c, HCAO_ECAPACITY,
                "the allocation-free step needs " + std::to_string(need) + " bytes of scratch for " +
                    std::to_string(c->work_entries) + " work entries; the fixed device array holds " +
                    std::to_string(kStaticScratchBytes));
  if (hcao_status s = timing_begin(c)) return s;
  uint32_t launches = 0;
  if (hcao_status s = issue_steps(c, dt, n_steps, c->step, nullptr, c->stream, &launches, &sc)) return s;
  c->step += n_steps;
  return timing_end(c, launches, n_steps);
}

hcao_status hcao_step_graph(hcao_ctx *c, double dt, uint32_t n_steps) {
  Range range("hcao_step_graph");
  if (hcao_status s = check_step_args(c, dt)) return s;
  if (c->spatial) return fail(c, HCAO_EUNSUPPORTED, "graph replay is not available in the spatial mode");
  if (n_steps == 0) return HCAO_OK;
  if (!c->graph_exec || c->graph_dt != dt || c->graph_n != n_steps || c->graph_gen != c->shape_gen) {
    drop_graph(c);
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (!c->d_step.p) HIP_TRY(c, c->d_step.alloc(1));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    uint32_t launches = 0;
    const hcao_status st = issue_steps(c, dt, n_steps, 0, c->d_step.p, c->cap_stream, &launches);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != HCAO_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    c->graph = g;
    HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    c->graph_dt = dt;
    c->graph_n = n_steps;
    c->graph_launches = launches;
    c->graph_gen = c->shape_gen;
  }
  if (c->d_step_value != (int64_t)c->step) {
    HIP_TRY(c, hipMemcpyAsync(c->d_step.p, &c->step, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));  // the source is host memory that changes below
  }
  if (hcao_status s = timing_begin(c)) return s;
  HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
  c->step += n_steps;
  c->d_step_value = c->step;
  return timing_end(c, c->graph_launches, n_steps);
}

hcao_status hcao_get_launch_shape(const hcao_ctx *c, hcao_launch_shape *shape) {
  if (!c || !shape) return HCAO_EINVAL;
  shape->block = (uint32_t)c->block;
  shape->group_slots = c->group_slots;
  shape->steps_per_launch = c->steps_per_launch >= (1u << 30) ? 0u : c->steps_per_launch;
  return HCAO_OK;
}

hcao_status hcao_set_launch_shape(hcao_ctx *c, const hcao_launch_shape *shape) {
  if (!c || !shape) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
  const uint32_t b = shape->block;
  if ((b != 64 && b != 128 && b != 256 && b != 512) || shape->group_slots == 0)
    return fail(c, HCAO_EINVAL, "launch shape: block must be 64, 128, 256 or 512 and group_slots > 0");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int old_block = c->block;
  const uint32_t old_slots = c->group_slots;
  c->block = (int)b;
  c->group_slots = shape->group_slots;
  c->steps_per_launch = shape->steps_per_launch ? shape->steps_per_launch : (1u << 30);
  ++c->shape_gen;
  if (c->loaded) {
    if (hcao_status s = build_groups(c)) {
      c->block = old_block;
      c->group_slots = old_slots;
      (void)build_groups(c);
      return s;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return HCAO_OK;
}

extern "C++" {
namespace {

// Device copy of everything a step changes, for the autotuner's trials.
struct Snapshot {
  DevBuf<double> vx, vy, vz, sgmax, rem, defect, rot, tsum;
  DevBuf<float> fx, fy, fz;
  DevBuf<uint8_t> sp;
  DevBuf<uint16_t> lvl;
  DevBuf<uint32_t> cnt, err;
  DevBuf<unsigned long long> ctr;
  uint32_t step = 0;
  Snapshot() = default;
  Snapshot(const Snapshot &) = delete;
  Snapshot &operator=(const Snapshot &) = delete;
  // the copy is freed when it goes out of scope (early returns included);
  // hipFree waits for work still using it
  ~Snapshot() {
    vx.release();
    vy.release();
    vz.release();
    sgmax.release();
    rem.release();
    defect.release();
    rot.release();
    tsum.release();
    fx.release();
    fy.release();
    fz.release();
    sp.release();
    lvl.release();
    cnt.release();
    err.release();
    ctr.release();
  }
};

template <class T>
hipError_t dcopy(DevBuf<T> &dst, const DevBuf<T> &src, bool alloc, hipStream_t s) {
  if (!src.p) return hipSuccess;
  if (alloc) {
    hipError_t e = dst.alloc(src.n);
    if (e != hipSuccess) return e;
  }
  return hipMemcpyAsync(dst.p, src.p, src.n * sizeof(T), hipMemcpyDeviceToDevice, s);
}

// direction: true = context -> snapshot (allocating), false = snapshot -> context
hcao_status snapshot(hcao_ctx *c, Snapshot &S, bool take) {
  hipStream_t st = c->stream;
#define SNAP(f) HIP_TRY(c, take ? dcopy(S.f, c->f, true, st) : dcopy(c->f, S.f, false, st))
  SNAP(vx);
  SNAP(vy);
  SNAP(vz);
  SNAP(fx);
  SNAP(fy);
  SNAP(fz);
  SNAP(sp);
  SNAP(rot);
  SNAP(lvl);
  SNAP(cnt);
  SNAP(sgmax);
  SNAP(rem);
  SNAP(defect);
  SNAP(tsum);
  SNAP(ctr);
  SNAP(err);
#undef SNAP
  if (take)
    S.step = c->step;
  else
    c->step = S.step;
  HIP_TRY(c, hipStreamSynchronize(st));
  return HCAO_OK;
}

// cache key: cell capacities, species and precision
std::string tune_key(const hcao_ctx *c) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the capacities
  for (uint32_t v : c->cap_host) {
    for (int i = 0; i < 4; ++i) {
      h ^= (v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  }
  char buf[160];
  std::snprintf(buf, sizeof(buf), "cells=%u slots=%llu caps=%016llx species=%u modes=%u rx=%u mixed=%d",
                c->cfg.n_cells, (unsigned long long)c->total_slots, (unsigned long long)h,
                (unsigned)c->species.size(), c->max_modes, (unsigned)c->reactions.size(), c->mixed ? 1 : 0);
  return buf;
}

}  // namespace
}  // extern "C++"

hcao_status hcao_autotune(hcao_ctx *c, double dt, uint32_t trial_steps, const char *cache_path,
                          hcao_launch_shape *chosen) {
  Range range("hcao_autotune");
  if (hcao_status s = check_step_args(c, dt)) return s;
  if (c->spatial) return fail(c, HCAO_EUNSUPPORTED, "autotuning is not available in the spatial mode");
  if (trial_steps == 0) return fail(c, HCAO_EINVAL, "trial_steps must be > 0");
  if (!cache_path) cache_path = std::getenv("HCAO_AUTOTUNE_CACHE");
  const std::string key = tune_key(c);
  hcao_launch_shape best{(uint32_t)c->block, c->group_slots, 0};
  const uint32_t spl = c->steps_per_launch;
  bool found = false;
  if (cache_path) {
    if (FILE *f = std::fopen(cache_path, "r")) {
      char line[320];
      while (std::fgets(line, sizeof(line), f)) {
        unsigned b = 0, g = 0;
        const size_t kl = key.size();
        if (std::strncmp(line, key.c_str(), kl) == 0 && line[kl] == ' ' &&
            std::sscanf(line + kl, " block=%u group_slots=%u", &b, &g) == 2) {
          best.block = b;
          best.group_slots = g;
          found = true;
        }
      }
      std::fclose(f);
    }
  }
  if (!found) {
    Snapshot S, W;
    if (hcao_status s = snapshot(c, S, true)) return s;
    const hcao_launch_shape orig{(uint32_t)c->block, c->group_slots, spl >= (1u << 30) ? 0u : spl};
    const bool was_timing = c->timing;
    double best_ms = 0.0;
    // candidates are timed from a copy advanced past the first steps, whose
    // (sigma g)_max still settles from its initial bound and would favour
    // other shapes
    auto trials = [&]() -> hcao_status {
      const uint32_t warm = trial_steps > 10u ? trial_steps : 10u;
      uint32_t launches = 0;
      if (hcao_status st = issue_steps(c, dt, warm, c->step, nullptr, c->stream, &launches)) return st;
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      if (hcao_status e = read_err(c)) return e;
      if (hcao_status s = snapshot(c, W, true)) return s;
      const uint32_t blocks[] = {64, 128, 256};
      const uint32_t slots[] = {256, 512, 1024, 1536, 2048, 2560, 3072, 3584, 4096, 6144};
      for (uint32_t b : blocks) {
        for (uint32_t g : slots) {
          if (g < b) continue;
          hcao_launch_shape t{b, g, orig.steps_per_launch};
          const hcao_status ss = hcao_set_launch_shape(c, &t);
          if (ss == HCAO_EUNSUPPORTED) continue;  // its LDS does not fit: skipped
          if (ss != HCAO_OK) return ss;
          HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
          if (hcao_status st = issue_steps(c, dt, trial_steps, c->step + warm, nullptr, c->stream, &launches))
            return st;
          HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
          HIP_TRY(c, hipEventSynchronize(c->ev1));
          float ms = 0.f;
          HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
          if (hcao_status e = read_err(c)) return e;
          if (!found || ms < best_ms) {
            best_ms = ms;
            best = t;
            found = true;
          }
          if (hcao_status s = snapshot(c, W, false)) return s;
        }
      }
      return HCAO_OK;
    };
    const hcao_status tried = trials();
    // every way out puts back the state before the call; a failed search also
    // its launch shape (a device error stays sticky)
    c->timing = was_timing;
    const hcao_status back = snapshot(c, S, false);
    if (tried != HCAO_OK) {
      if (c->sticky == HCAO_OK) (void)hcao_set_launch_shape(c, &orig);
      return tried;
    }
    if (back != HCAO_OK) return back;
    if (cache_path) {
      if (FILE *f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s block=%u group_slots=%u ms_per_step=%.6g\n", key.c_str(), best.block, best.group_slots,
                     best_ms / trial_steps);
        std::fclose(f);
      }
    }
  }
  best.steps_per_launch = spl >= (1u << 30) ? 0u : spl;
  if (hcao_status s = hcao_set_launch_shape(c, &best)) return s;
  if (chosen) *chosen = best;
  return HCAO_OK;
}

hcao_status hcao_sync(hcao_ctx *c) {
  if (!c) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->loaded) return read_err(c);
  return HCAO_OK;
}

hcao_status hcao_get_counts(hcao_ctx *c, uint64_t *per_cell, uint64_t *total) {
  if (!c) return HCAO_EINVAL;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "no particles");
  std::vector<uint32_t> cnt(c->cfg.n_cells);
  HIP_TRY(c, hipMemcpyAsync(cnt.data(), c->cnt.p, cnt.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  uint64_t t = 0;
  for (size_t i = 0; i < cnt.size(); ++i) {
    if (per_cell) per_cell[i] = cnt[i];
    t += cnt[i];
  }
  if (total) *total = t;
  return HCAO_OK;
}

uint32_t hcao_max_modes(const hcao_ctx *c) { return c ? c->max_modes : 0; }
uint32_t hcao_step_index(const hcao_ctx *c) { return c ? c->step : 0; }

hcao_status hcao_read_cell_particles(hcao_ctx *c, uint32_t cell, uint32_t max_n, uint8_t *species, double *vel,
                                     uint16_t *levels, uint32_t *n_out) {
  if (!c || (max_n && (!species || !vel || !levels))) return HCAO_EINVAL;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "no particles");
  if (cell >= c->cfg.n_cells) return fail(c, HCAO_EINVAL, "cell index out of range");
  const uint64_t b = c->off_host[cell];
  const uint32_t mm = c->max_modes ? c->max_modes : 1;
  uint32_t n = 0;
  HIP_TRY(c, hipMemcpyAsync(&n, c->cnt.p + cell, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (n_out) *n_out = n;
  const uint32_t k = std::min(n, max_n);
  if (k == 0) return HCAO_OK;
  std::vector<double> v(3 * (size_t)k);
  const uint32_t lr = level_row(c->max_modes);
  std::vector<uint16_t> lv((size_t)k * lr);
  if (c->mixed) {
    std::vector<float> f(3 * (size_t)k);
    HIP_TRY(c, hipMemcpyAsync(f.data(), c->fx.p + b, k * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(f.data() + k, c->fy.p + b, k * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(f.data() + 2 * (size_t)k, c->fz.p + b, k * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < v.size(); ++i) v[i] = f[i];
  } else {
    HIP_TRY(c, hipMemcpyAsync(v.data(), c->vx.p + b, k * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(v.data() + k, c->vy.p + b, k * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(v.data() + 2 * (size_t)k, c->vz.p + b, k * 8, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(c, hipMemcpyAsync(species, c->sp.p + b, k, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(lv.data(), c->lvl.p + b * lr, (size_t)k * lr * 2, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (uint32_t i = 0; i < k; ++i) {
    vel[3 * i] = v[i];
    vel[3 * i + 1] = v[k + i];
    vel[3 * i + 2] = v[2 * (size_t)k + i];
    for (uint32_t m = 0; m < mm; ++m) levels[(size_t)i * mm + m] = lv[(size_t)i * lr + m];
  }
  return HCAO_OK;
}

hcao_status hcao_read_particles(hcao_ctx *c, uint8_t *species, double *vel, uint16_t *levels) {
  if (!c || !species || !vel || !levels) return HCAO_EINVAL;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "no particles");
  const uint64_t tot = c->total_slots;
  const uint32_t nc = c->cfg.n_cells, mm = c->max_modes ? c->max_modes : 1;
  std::vector<double> vx(tot), vy(tot), vz(tot);
  std::vector<uint8_t> sp(tot);
  const uint32_t lr = level_row(c->max_modes);
  std::vector<uint16_t> lv(tot * lr);
  std::vector<uint32_t> cnt(nc);
  if (hcao_status s = download_vel(c, vx, vy, vz)) return s;
  HIP_TRY(c, hipMemcpyAsync(sp.data(), c->sp.p, tot, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(lv.data(), c->lvl.p, tot * lr * 2, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(cnt.data(), c->cnt.p, nc * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  uint64_t j = 0;
  for (uint32_t cell = 0; cell < nc; ++cell) {
    const uint64_t b = c->off_host[cell];
    for (uint32_t i = 0; i < cnt[cell]; ++i, ++j) {
      const uint64_t g = b + i;
      species[j] = sp[g];
      vel[3 * j] = vx[g];
      vel[3 * j + 1] = vy[g];
      vel[3 * j + 2] = vz[g];
      for (uint32_t m = 0; m < mm; ++m) levels[j * mm + m] = lv[g * lr + m];
    }
  }
  return HCAO_OK;
}

hcao_status hcao_read_rotational_energy(hcao_ctx *c, double *rot) {
  if (!c || !rot) return HCAO_EINVAL;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "no particles");
  const uint64_t tot = c->total_slots;
  const uint32_t nc = c->cfg.n_cells;
  std::vector<uint32_t> cnt(nc);
  std::vector<double> r(c->rot.p ? tot : 0);
  HIP_TRY(c, hipMemcpyAsync(cnt.data(), c->cnt.p, nc * 4, hipMemcpyDeviceToHost, c->stream));
  if (c->rot.p) HIP_TRY(c, hipMemcpyAsync(r.data(), c->rot.p, tot * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  uint64_t j = 0;
  for (uint32_t cell = 0; cell < nc; ++cell)
    for (uint32_t i = 0; i < cnt[cell]; ++i, ++j) rot[j] = c->rot.p ? r[c->off_host[cell] + i] : 0.0;
  return HCAO_OK;
}

hcao_status hcao_read_cell_state(hcao_ctx *c, double *sgmax, double *rem, uint64_t *counters) {
  if (!c) return HCAO_EINVAL;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "no particles");
  const uint32_t nc = c->cfg.n_cells;
  if (sgmax) HIP_TRY(c, hipMemcpyAsync(sgmax, c->sgmax.p, nc * 8, hipMemcpyDeviceToHost, c->stream));
  if (rem) HIP_TRY(c, hipMemcpyAsync(rem, c->rem.p, nc * 8, hipMemcpyDeviceToHost, c->stream));
  if (counters)
    HIP_TRY(c, hipMemcpyAsync(counters, c->ctr.p, (size_t)nc * kNumCtr * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return HCAO_OK;
}

hcao_status hcao_read_moments(hcao_ctx *c, hcao_moments *per_cell, hcao_moments *total) {
  Range range("hcao_read_moments");
  if (!c) return HCAO_EINVAL;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "no particles");
  const uint32_t nc = c->cfg.n_cells, ns = (uint32_t)c->species.size();
  const uint32_t w = 6 + 3 * ns;
  DevBuf<double> d_out;
  HIP_TRY(c, d_out.alloc((size_t)nc * w));
  HIP_TRY(c, launch_moments(c->d_tab.p, c->d_lev.p, state_of(c), c->off.p, c->cnt.p, d_out.p, nc, c->stream));
  std::vector<double> raw((size_t)nc * w), df(nc);
  HIP_TRY(c, hipMemcpyAsync(raw.data(), d_out.p, raw.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(df.data(), c->defect.p, nc * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  auto fill = [&](hcao_moments &M, const double *r, double vol, double wgt) {
    std::memset(&M, 0, sizeof(M));
    for (int k = 0; k < 3; ++k) M.momentum[k] = r[k];
    const double mass = r[4];
    const double p2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    M.E_kin_J = 0.5 * r[3];
    M.E_trans_J = mass > 0.0 ? 0.5 * (r[3] - p2 / mass) : 0.0;
    M.E_formation_J = r[5];
    uint64_t ntot = 0;
    for (uint32_t s = 0; s < ns; ++s) {
      const uint64_t k = (uint64_t)std::llround(r[6 + s]);
      M.n_species[s] = k;
      ntot += k;
      M.E_vib_J[s] = r[6 + ns + s];
      if (vol > 0.0) M.number_density[s] = (double)k * wgt / vol;
      M.T_vib_K[s] = k ? c->thermo[s].temperature(r[6 + ns + s] / (double)k) : 0.0;
      M.E_rot_J[s] = r[6 + 2 * ns + s];
      const uint32_t z = c->species[s].d.zeta_rot;
      M.T_rot_K[s] = (k && z) ? (2.0 * M.E_rot_J[s]) / ((double)z * kB * (double)k) : 0.0;
    }
    M.n_total = ntot;
    M.T_trans_K = ntot ? 2.0 * M.E_trans_J / (3.0 * kB * (double)ntot) : 0.0;
  };
  std::vector<double> sum(w, 0.0);
  double vol_tot = 0.0, def_tot = 0.0;
  std::vector<double> dens(ns, 0.0);
  for (uint32_t i = 0; i < nc; ++i) {
    const double *r = raw.data() + (size_t)i * w;
    if (per_cell) {
      fill(per_cell[i], r, c->volume[i], c->weight[i]);
      per_cell[i].E_defect_J = df[i];
    }
    def_tot += df[i];
    for (uint32_t k = 0; k < w; ++k) sum[k] += r[k];
    vol_tot += c->volume[i];
    for (uint32_t s = 0; s < ns; ++s) dens[s] += r[6 + s] * c->weight[i];
  }
  if (total) {
    fill(*total, sum.data(), 0.0, 0.0);
    for (uint32_t s = 0; s < ns; ++s) total->number_density[s] = dens[s] / vol_tot;
    total->E_defect_J = def_tot;
  }
  return HCAO_OK;
}

hcao_status hcao_read_reaction_counts(hcao_ctx *c, uint64_t *counts) {
  if (!c || !counts) return HCAO_EINVAL;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "no particles");
  const uint32_t nc = c->cfg.n_cells;
  std::vector<uint64_t> ctr((size_t)nc * kNumCtr);
  if (hcao_status s = hcao_read_cell_state(c, nullptr, nullptr, ctr.data())) return s;
  for (size_t r = 0; r < c->reactions.size(); ++r) {
    uint64_t t = 0;
    for (uint32_t i = 0; i < nc; ++i) t += ctr[(size_t)i * kNumCtr + HCAO_CTR_REACTION0 + r];
    counts[r] = t;
  }
  return HCAO_OK;
}

hcao_status hcao_get_levels(const hcao_ctx *c, uint32_t species, uint32_t mode, double *out, uint32_t max_n,
                            uint32_t *n_out) {
  if (!c || !out || species >= c->species.size()) return HCAO_EINVAL;
  const SpeciesHost &s = c->species[species];
  if (mode >= s.n_modes) return HCAO_EINVAL;
  uint32_t n = 0;
  if (mode < s.d.n_bend) {
    for (; n < max_n; ++n) out[n] = host_mode_energy(s, mode, n);
  } else {
    const auto &L = s.levels[mode - s.d.n_bend];
    for (; n < max_n && n < L.size(); ++n) out[n] = L[n];
    n = (uint32_t)L.size();
  }
  if (n_out) *n_out = n;
  return HCAO_OK;
}

hcao_status hcao_get_pair(const hcao_ctx *c, uint32_t a, uint32_t b, double *out8) {
  if (!c || !out8 || !c->finalized || a >= c->species.size() || b >= c->species.size()) return HCAO_EINVAL;
  const PairTab &P = c->tab.pr[a][b];
  const double v[8] = {P.mr, P.hm, P.msum, P.wa, P.wb, P.csg, P.esg, P.q};
  std::memcpy(out8, v, sizeof(v));
  return HCAO_OK;
}

hcao_status hcao_get_recombination_table(const hcao_ctx *c, uint32_t reaction, double *out, uint32_t max_n,
                                         uint32_t *n_out) {
  if (!c || !c->finalized || reaction >= c->reactions.size()) return HCAO_EINVAL;
  const ReactionTab &R = c->tab.rx[reaction];
  if (R.kind != HCAO_RX_RECOMBINATION) return HCAO_EINVAL;
  const uint32_t n = (uint32_t)c->species.size() * kRecNodes;
  for (uint32_t i = 0; i < n && i < max_n; ++i) out[i] = c->rec_host[R.rec_off + i];
  if (n_out) *n_out = n;
  return HCAO_OK;
}

hcao_status hcao_recombination_exact(hcao_ctx *c, uint32_t species, double de_J, double omega, uint32_t n_t,
                                     const double *t_K, double *p_out, double *elapsed_ms, uint64_t *n_records) {
  Range range("hcao_recombination_exact");
  if (!c || !c->finalized || species >= c->species.size() || (n_t && (!t_K || !p_out))) return HCAO_EINVAL;
  for (uint32_t i = 0; i < n_t; ++i)
    if (!(t_K[i] > 0.0)) return fail(c, HCAO_EINVAL, "temperatures must be positive");
  if (c->species[species].n_modes == 0) return fail(c, HCAO_EINVAL, "species has no vibrational modes");
  return exact_rec_probability(c, species, de_J, omega, n_t, t_K, p_out, elapsed_ms, n_records);
}

hcao_status hcao_set_domain(hcao_ctx *c, const hcao_domain *d) {
  if (!c || !d) return HCAO_EINVAL;
  if (c->finalized) return fail(c, HCAO_ESTATE, "set_domain after finalize");
  const uint32_t nc = c->cfg.n_cells;
  if (d->nx == 0 || d->ny == 0 || d->nz == 0 || (uint64_t)d->nx * d->ny * d->nz != nc)
    return fail(c, HCAO_EINVAL, "the grid must have n_cells cells");
  if (!(d->lx > 0.0) || !(d->ly > 0.0) || !(d->lz > 0.0) || d->periodic > 7u)
    return fail(c, HCAO_EINVAL, "bad box lengths or periodic bits");
  const double vc = ((d->lx * d->ly) * d->lz) / (double)nc;
  for (uint32_t i = 0; i < nc; ++i)
    if (std::fabs(c->volume[i] - vc) > 1e-9 * vc) return fail(c, HCAO_EINVAL, "cell volume differs from the grid cell");
  c->spatial = true;
  c->grid[0] = d->nx;
  c->grid[1] = d->ny;
  c->grid[2] = d->nz;
  c->periodic = d->periodic;
  c->len[0] = d->lx;
  c->len[1] = d->ly;
  c->len[2] = d->lz;
  return HCAO_OK;
}

hcao_status hcao_set_inflow(hcao_ctx *c, const hcao_inflow *in) {
  if (!c || !in) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
  if (!c->spatial || !c->finalized) return fail(c, HCAO_ESTATE, "open faces need the spatial mode, after finalize");
  const uint32_t ns = (uint32_t)c->species.size();
  if (in->open_faces > 63u) return fail(c, HCAO_EINVAL, "open_faces has bits beyond the six faces");
  for (int k = 0; k < 3; ++k)
    if (((c->periodic >> k) & 1u) && ((in->open_faces >> (2 * k)) & 3u))
      return fail(c, HCAO_EINVAL, "an open face on a periodic axis");
  if (in->open_faces) {
    if (!in->number_density) return fail(c, HCAO_EINVAL, "number densities missing");
    if (!(in->t_trans_K > 0.0) || !(in->t_vib_K > 0.0) || !std::isfinite(in->t_trans_K) || !std::isfinite(in->t_vib_K))
      return fail(c, HCAO_EINVAL, "bad reservoir temperature");
    for (uint32_t k = 0; k < ns; ++k)
      if (!(in->number_density[k] >= 0.0) || !std::isfinite(in->number_density[k]))
        return fail(c, HCAO_EINVAL, "bad reservoir number density");
  }
  c->face_base[0] = 0;
  for (uint32_t f = 0; f < 6; ++f) {
    const uint32_t k = f >> 1, a = k == 0 ? 1u : 0u, b = k == 2 ? 1u : 2u;
    c->face_base[f + 1] = c->face_base[f] + c->grid[a] * c->grid[b];
  }
  c->open_faces = in->open_faces;
  c->in_rem.release();
  c->in_count.release();
  c->in_base.release();
  c->flux.release();
  if (!c->open_faces) return HCAO_OK;
  c->in_t = in->t_trans_K;
  c->in_tv = in->t_vib_K;
  for (uint32_t k = 0; k < ns; ++k)
    c->in_flux[k] = in->number_density[k] * std::sqrt((kB * c->in_t) / ((2.0 * kPi) * c->species[k].d.mass_kg));
  const uint64_t faces = (uint64_t)c->face_base[6] * ns;
  HIP_TRY(c, c->in_rem.alloc(faces));
  HIP_TRY(c, c->in_count.alloc(faces + 1));
  HIP_TRY(c, c->in_base.alloc(faces + 1));
  HIP_TRY(c, c->flux.alloc(2));
  HIP_TRY(c, reset_inflow(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return HCAO_OK;
}

hcao_status hcao_read_flux_counts(hcao_ctx *c, uint64_t *out) {
  if (!c || !out) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
  out[0] = out[1] = 0;
  if (!c->open_faces) return HCAO_OK;
  unsigned long long v[2];
  HIP_TRY(c, hipMemcpyAsync(v, c->flux.p, sizeof v, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  out[0] = v[0];
  out[1] = v[1];
  return HCAO_OK;
}

hcao_status hcao_read_positions(hcao_ctx *c, double *pos) {
  if (!c || !pos) return HCAO_EINVAL;
  if (!c->loaded || !c->spatial) return fail(c, HCAO_ESTATE, "no positions (spatial mode only)");
  const uint64_t tot = c->total_slots;
  const uint32_t nc = c->cfg.n_cells;
  std::vector<uint32_t> cnt(nc);
  std::vector<double> x(tot), y(tot), z(tot);
  HIP_TRY(c, hipMemcpyAsync(cnt.data(), c->cnt.p, nc * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(x.data(), c->px.p, tot * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(y.data(), c->py.p, tot * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(z.data(), c->pz.p, tot * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  uint64_t j = 0;
  for (uint32_t cell = 0; cell < nc; ++cell)
    for (uint32_t i = 0; i < cnt[cell]; ++i, ++j) {
      const uint64_t g = c->off_host[cell] + i;
      pos[3 * j] = x[g];
      pos[3 * j + 1] = y[g];
      pos[3 * j + 2] = z[g];
    }
  return HCAO_OK;
}

hcao_status hcao_get_exact_beta(const hcao_ctx *c, uint32_t species, uint32_t partner, double e_J, double *beta) {
  if (!c || !beta || !c->finalized || species >= c->species.size() || partner >= c->species.size() || !(e_J > 0.0))
    return HCAO_EINVAL;
  const PairTab &P = c->tab.pr[species][partner];
  if (P.beta_off == 0xFFFFFFFFu) return HCAO_EINVAL;
  uint64_t bits;
  std::memcpy(&bits, &e_J, sizeof(bits));
  uint32_t bin = (uint32_t)(bits >> 48);
  bin = bin < kExactBinLo ? kExactBinLo : (bin > kExactBinHi ? kExactBinHi : bin);
  double b = c->beta_host[P.beta_off + (bin - kExactBinLo)];
  if (b * e_J < P.q) b = P.q / e_J;
  *beta = b;
  return HCAO_OK;
}

hcao_status hcao_set_timing(hcao_ctx *c, int enable) {
  if (!c) return HCAO_EINVAL;
  c->timing = enable != 0;
  c->timed_ms = 0.0;
  c->timed_launches = 0;
  c->timed_steps = 0;
  return HCAO_OK;
}

hcao_status hcao_kernel_time(hcao_ctx *c, double *ms, uint64_t *launches, uint64_t *steps) {
  if (!c) return HCAO_EINVAL;
  if (ms) *ms = c->timed_ms;
  if (launches) *launches = c->timed_launches;
  if (steps) *steps = c->timed_steps;
  return HCAO_OK;
}

hcao_status hcao_phase_clocks(hcao_ctx *c, uint64_t *out, uint32_t n, int reset) {
  if (!c || (n && !out)) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
#ifdef HCAO_PHASE_CLOCKS
  if (!c->finalized) return fail(c, HCAO_ESTATE, "phase clocks before finalize");
  if (!c->clk.p) {
    HIP_TRY(c, c->clk.alloc(kPhases));
    HIP_TRY(c, hipMemsetAsync(c->clk.p, 0, kPhases * sizeof(unsigned long long), c->stream));
  }
  unsigned long long h[kPhases] = {};
  HIP_TRY(c, hipMemcpyAsync(h, c->clk.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (uint32_t k = 0; k < n && k < (uint32_t)kPhases; ++k) out[k] = h[k];
  if (reset) {
    HIP_TRY(c, hipMemsetAsync(c->clk.p, 0, kPhases * sizeof(unsigned long long), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return HCAO_OK;
#else
  (void)reset;
  return fail(c, HCAO_EUNSUPPORTED, "phase clocks need a library built with HCAO_PHASE_CLOCKS");
#endif
}

hcao_status hcao_save(hcao_ctx *c, const char *path) {
  if (!c || !path) return HCAO_EINVAL;
  if (!c->loaded) return fail(c, HCAO_ESTATE, "no particles");
  if (hcao_status s = hcao_sync(c)) return s;
  const uint64_t tot = c->total_slots;
  const uint32_t nc = c->cfg.n_cells, mm = c->max_modes ? c->max_modes : 1;
  std::vector<double> vx, vy, vz, sg(nc), rm(nc), df(nc), ts(c->tsum.p ? 5 * (size_t)nc : 0);
  std::vector<uint8_t> sp(tot);
  std::vector<uint16_t> lv(tot * mm);
  std::vector<uint32_t> cnt(nc);
  std::vector<unsigned long long> ctr((size_t)nc * kNumCtr);
  if (hcao_status s = download_vel(c, vx, vy, vz)) return s;
  HIP_TRY(c, hipMemcpy(df.data(), c->defect.p, nc * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(sp.data(), c->sp.p, tot, hipMemcpyDeviceToHost));
  {
    // the file holds n x max_modes rows; the device rows are level_row long
    const uint32_t lr = level_row(c->max_modes);
    std::vector<uint16_t> rows(tot * lr);
    HIP_TRY(c, hipMemcpy(rows.data(), c->lvl.p, tot * lr * 2, hipMemcpyDeviceToHost));
    for (uint64_t g = 0; g < tot; ++g)
      for (uint32_t m = 0; m < mm; ++m) lv[g * mm + m] = rows[g * lr + m];
  }
  HIP_TRY(c, hipMemcpy(cnt.data(), c->cnt.p, nc * 4, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(sg.data(), c->sgmax.p, nc * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(rm.data(), c->rem.p, nc * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(ctr.data(), c->ctr.p, ctr.size() * 8, hipMemcpyDeviceToHost));
  if (!ts.empty()) HIP_TRY(c, hipMemcpy(ts.data(), c->tsum.p, ts.size() * 8, hipMemcpyDeviceToHost));
  std::vector<double> rt(c->rot.p ? tot : 0);
  if (c->rot.p) HIP_TRY(c, hipMemcpy(rt.data(), c->rot.p, tot * 8, hipMemcpyDeviceToHost));
  std::vector<double> pos(c->spatial ? 3 * tot : 0);
  if (c->spatial) {
    HIP_TRY(c, hipMemcpy(pos.data(), c->px.p, tot * 8, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(pos.data() + tot, c->py.p, tot * 8, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(pos.data() + 2 * tot, c->pz.p, tot * 8, hipMemcpyDeviceToHost));
  }
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(c, HCAO_EINVAL, std::string("cannot open ") + path);
  std::vector<double> irem(c->open_faces ? c->in_rem.n : 0);
  unsigned long long fl[2] = {0, 0};
  if (c->open_faces) {
    HIP_TRY(c, hipMemcpy(irem.data(), c->in_rem.p, irem.size() * 8, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(fl, c->flux.p, sizeof fl, hipMemcpyDeviceToHost));
  }
  // velocities are stored as fp64 in both forms (exact for fp32 values);
  // word 6: bit 0 mixed form, bit 1 rotational energies follow the levels,
  // bit 2 positions (x, y, z arrays) follow, bit 3 the open faces' inflow
  // remainders and the two flux counts follow, bit 4 the cells' running
  // sums of the recombination temperature follow ([5][n_cells])
  const uint64_t form = (c->mixed ? 1ull : 0ull) | (c->rot.p ? 2ull : 0ull) | (c->spatial ? 4ull : 0ull) |
                        (c->open_faces ? 8ull : 0ull) | (ts.empty() ? 0ull : 16ull);
  const uint64_t hdr[7] = {0x48434130534156ull, HCAO_ABI_VERSION, nc, tot, mm, c->step, form};
  bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1;
  ok = ok && std::fwrite(c->cap_host.data(), 4, nc, f) == nc;
  ok = ok && std::fwrite(cnt.data(), 4, nc, f) == nc;
  ok = ok && std::fwrite(sg.data(), 8, nc, f) == nc;
  ok = ok && std::fwrite(rm.data(), 8, nc, f) == nc;
  ok = ok && std::fwrite(df.data(), 8, nc, f) == nc;
  ok = ok && std::fwrite(ctr.data(), 8, ctr.size(), f) == ctr.size();
  ok = ok && std::fwrite(vx.data(), 8, tot, f) == tot;
  ok = ok && std::fwrite(vy.data(), 8, tot, f) == tot;
  ok = ok && std::fwrite(vz.data(), 8, tot, f) == tot;
  ok = ok && std::fwrite(sp.data(), 1, tot, f) == tot;
  ok = ok && std::fwrite(lv.data(), 2, lv.size(), f) == lv.size();
  ok = ok && std::fwrite(rt.data(), 8, rt.size(), f) == rt.size();
  ok = ok && std::fwrite(pos.data(), 8, pos.size(), f) == pos.size();
  ok = ok && std::fwrite(irem.data(), 8, irem.size(), f) == irem.size();
  if (c->open_faces) ok = ok && std::fwrite(fl, 8, 2, f) == 2;
  ok = ok && std::fwrite(ts.data(), 8, ts.size(), f) == ts.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, HCAO_EINVAL, "write failed");
  return HCAO_OK;
}

hcao_status hcao_restore(hcao_ctx *c, const char *path) {
  if (!c || !path) return HCAO_EINVAL;
  if (hcao_status s = check_sticky(c)) return s;
  if (!c->finalized) return fail(c, HCAO_ESTATE, "restore before finalize");
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(c, HCAO_EINVAL, std::string("cannot open ") + path);
  uint64_t hdr[7];
  const uint32_t nc = c->cfg.n_cells, mm = c->max_modes ? c->max_modes : 1;
  if (std::fread(hdr, sizeof(hdr), 1, f) != 1 || hdr[0] != 0x48434130534156ull || hdr[1] != HCAO_ABI_VERSION ||
      hdr[2] != nc || hdr[4] != mm ||
      hdr[6] != ((c->mixed ? 1ull : 0ull) | (c->tab.has_rot ? 2ull : 0ull) | (c->spatial ? 4ull : 0ull) |
                 (c->open_faces ? 8ull : 0ull) | (c->tab.has_recomb ? 16ull : 0ull))) {
    std::fclose(f);
    return fail(c, HCAO_EINVAL, "checkpoint does not match this context");
  }
  const uint64_t tot = hdr[3];
  std::vector<uint32_t> capv(nc), cnt(nc);
  std::vector<double> sg(nc), rm(nc), df(nc), vx(tot), vy(tot), vz(tot);
  std::vector<unsigned long long> ctr((size_t)nc * kNumCtr);
  std::vector<uint8_t> sp(tot);
  std::vector<uint16_t> lv(tot * mm);
  bool ok = std::fread(capv.data(), 4, nc, f) == nc;
  ok = ok && std::fread(cnt.data(), 4, nc, f) == nc;
  ok = ok && std::fread(sg.data(), 8, nc, f) == nc;
  ok = ok && std::fread(rm.data(), 8, nc, f) == nc;
  ok = ok && std::fread(df.data(), 8, nc, f) == nc;
  ok = ok && std::fread(ctr.data(), 8, ctr.size(), f) == ctr.size();
  ok = ok && std::fread(vx.data(), 8, tot, f) == tot;
  ok = ok && std::fread(vy.data(), 8, tot, f) == tot;
  ok = ok && std::fread(vz.data(), 8, tot, f) == tot;
  ok = ok && std::fread(sp.data(), 1, tot, f) == tot;
  ok = ok && std::fread(lv.data(), 2, lv.size(), f) == lv.size();
  std::vector<double> rt(c->tab.has_rot ? tot : 0);
  ok = ok && std::fread(rt.data(), 8, rt.size(), f) == rt.size();
  std::vector<double> pos(c->spatial ? 3 * tot : 0);
  ok = ok && std::fread(pos.data(), 8, pos.size(), f) == pos.size();
  std::vector<double> irem(c->open_faces ? c->in_rem.n : 0);
  unsigned long long fl[2] = {0, 0};
  ok = ok && std::fread(irem.data(), 8, irem.size(), f) == irem.size();
  if (c->open_faces) ok = ok && std::fread(fl, 8, 2, f) == 2;
  std::vector<double> ts(c->tab.has_recomb ? 5 * (size_t)nc : 0);
  ok = ok && std::fread(ts.data(), 8, ts.size(), f) == ts.size();
  std::fclose(f);
  if (!ok) return fail(c, HCAO_EINVAL, "truncated checkpoint");
  uint64_t t2 = 0;
  for (uint32_t v : capv) t2 += v;
  if (t2 != tot) return fail(c, HCAO_EINVAL, "checkpoint capacities inconsistent");
  if (hcao_status st = alloc_state(c, cnt, &capv)) return st;
  if (hcao_status s = upload_vel(c, vx, vy, vz)) return s;
  HIP_TRY(c, hipMemcpy(c->defect.p, df.data(), nc * 8, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->sp.p, sp.data(), tot, hipMemcpyHostToDevice));
  {
    const uint32_t lr = level_row(c->max_modes);
    std::vector<uint16_t> rows(tot * lr, 0);
    for (uint64_t g = 0; g < tot; ++g)
      for (uint32_t m = 0; m < mm; ++m) rows[g * lr + m] = lv[g * mm + m];
    HIP_TRY(c, hipMemcpy(c->lvl.p, rows.data(), tot * lr * 2, hipMemcpyHostToDevice));
  }
  HIP_TRY(c, hipMemcpy(c->sgmax.p, sg.data(), nc * 8, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->rem.p, rm.data(), nc * 8, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->ctr.p, ctr.data(), ctr.size() * 8, hipMemcpyHostToDevice));
  if (!ts.empty()) HIP_TRY(c, hipMemcpy(c->tsum.p, ts.data(), ts.size() * 8, hipMemcpyHostToDevice));
  if (c->rot.p) HIP_TRY(c, hipMemcpy(c->rot.p, rt.data(), tot * 8, hipMemcpyHostToDevice));
  if (c->spatial) {
    HIP_TRY(c, hipMemcpy(c->px.p, pos.data(), tot * 8, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->py.p, pos.data() + tot, tot * 8, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->pz.p, pos.data() + 2 * tot, tot * 8, hipMemcpyHostToDevice));
  }
  if (c->open_faces) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(c->in_rem.p, irem.data(), irem.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->flux.p, fl, sizeof fl, hipMemcpyHostToDevice));
  }
  c->step = (uint32_t)hdr[5];
  c->loaded = true;
  return HCAO_OK;
}

void hcao_destroy(hcao_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->d_step.release();
  free_state(c);
  c->d_tab.release();
  c->d_lev.release();
  c->d_rec.release();
  c->d_beta.release();
  c->err.release();
  c->in_rem.release();
  c->in_count.release();
  c->in_base.release();
  c->flux.release();
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
}

}  // extern "C"
