// lbf.hip -- host side of the C ABI declared in include/lbf.h: argument
// validation, per-lattice coefficient tables, contexts, kernel dispatch,
// HIP-graph replay of step chunks, ensembles and the schedule autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "lbf.h"
#include "lbf_kernels.h"
#include "lbf_fused2d.h"

using namespace lbf;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(LB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

size_t elem_size(int storage) { return storage == LB_F32 ? 4 : 2; }

int validate(const lb_params* p) {
  if (!p) return fail(LB_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LB_EINVAL, "box dimensions must be >= 1");
  if (p->storage < LB_F32 || p->storage > LB_BF16) return fail(LB_EINVAL, "unknown storage type");
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail(LB_EINVAL, "rho0 must be finite and > 0");
  if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return fail(LB_EINVAL, "kT must be finite and >= 0");
  const double g[4] = {p->gamma_bulk, p->gamma_shear, p->gamma_odd, p->gamma_even};
  for (double v : g)
    if (!(v >= -1.0 && v <= 1.0)) return fail(LB_EINVAL, "every gamma must lie in [-1, 1]");
  if (p->thermal_modes != LB_THERMAL_ALL && p->thermal_modes != LB_THERMAL_STRESS_ONLY)
    return fail(LB_EINVAL, "unknown thermal_modes");
  if (p->lattice != LB_D3Q19 && p->lattice != LB_D2Q9) return fail(LB_EINVAL, "unknown lattice");
  if (p->lattice == LB_D2Q9 && p->nz != 1) return fail(LB_EINVAL, "a D2Q9 lattice needs nz = 1");
  const uint64_t n = (uint64_t)p->nx * (uint64_t)p->ny * (uint64_t)p->nz;
  // site indices are 32-bit, and a grid rounded up to whole workgroups must not wrap them
  if (n > (1ull << 32) - 1024)
    return fail(LB_EUNSUPPORTED, "lattices of more than 2^32 - 1024 sites are not supported");
  return LB_OK;
}

uint64_t sites_of(const lb_params& p) { return (uint64_t)p.nx * (uint64_t)p.ny * (uint64_t)p.nz; }
int q_of(int lattice) { return lattice == LB_D2Q9 ? D2Q9::Q : D3Q19::Q; }

// Division by an invariant integer d (Granlund & Montgomery 1994):
// q = (t + ((n - t) >> s1)) >> s2 with t = mulhi(n, m).
void div_magic(uint32_t d, uint32_t& m, uint32_t& s1, uint32_t& s2) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  s1 = l > 0 ? 1 : 0;
  s2 = l > 0 ? l - 1 : 0;
}

// Per-lattice descriptor: geometry, division constants, Philox key and the
// per-mode coefficients of the model's collision (rates by mode class).
template <class M>
LatDesc make_desc_m(const lb_params& p, uint64_t base) {
  static_assert(M::Q <= (int)(sizeof(LatDesc::ci) / sizeof(float)), "ci too small for this model");
  static_assert(M::Q - M::D - 1 <= (int)(sizeof(LatDesc::ca) / sizeof(float)), "ca/cc too small for this model");
  static_assert(M::NSTRESS <= (int)(sizeof(LatDesc::cb) / sizeof(float)), "cb too small for this model");
  LatDesc L;
  std::memset(&L, 0, sizeof(L));
  L.base = base;
  L.plane = sites_of(p);
  L.nsites = (uint32_t)L.plane;
  L.nx = p.nx; L.ny = p.ny; L.nz = p.nz;
  L.nxy = (uint32_t)p.nx * (uint32_t)p.ny;
  L.wx = p.nx - 1;
  L.wy = (uint32_t)(p.ny - 1) * (uint32_t)p.nx;
  L.wz = (uint32_t)(p.nz - 1) * L.nxy;
  div_magic(p.nx, L.dx_m, L.dx_s1, L.dx_s2);
  div_magic(p.ny, L.dy_m, L.dy_s1, L.dy_s2);
  L.key0 = (uint32_t)p.seed;
  L.key1 = (uint32_t)(p.seed >> 32);
  L.thermal = p.kT > 0.0 ? 1u : 0u;
  L.rho0 = (float)p.rho0;
  const double mu = 3.0 * p.kT;  // kT / c_s^2 in lattice units
  constexpr int K0 = M::D + 1;
  for (int k = K0; k < M::Q; ++k) {
    const int cls = M::CLS[k];  // 1 bulk, 2 shear, 3 odd kinetic, 4 even kinetic
    const double g = cls == 1 ? p.gamma_bulk : cls == 2 ? p.gamma_shear : cls == 3 ? p.gamma_odd : p.gamma_even;
    const bool stress = cls <= 2;
    const bool noisy = stress || p.thermal_modes == LB_THERMAL_ALL;
    const double wk = (double)M::W36[k] / 36.0;
    L.ca[k - K0] = (float)(g / (36.0 * wk));
    if (stress) L.cb[k - K0] = (float)((1.0 - g) / (36.0 * wk));
    L.cc[k - K0] = noisy ? (float)std::sqrt(mu * (1.0 - g * g) / (wk * p.rho0)) : 0.0f;
  }
  for (int k = 0; k < M::Q; ++k) L.ci[k] = (float)std::sqrt(mu / (p.rho0 * ((double)M::W36[k] / 36.0)));
  return L;
}
LatDesc make_desc(const lb_params& p, uint64_t base) {
  return p.lattice == LB_D2Q9 ? make_desc_m<D2Q9>(p, base) : make_desc_m<D3Q19>(p, base);
}

// Planes of 4 GiB or more need 64-bit offsets (buffer descriptors hold a
// 32-bit size).
bool is_wide(const lb_params& p) { return sites_of(p) * elem_size(p.storage) >= (1ull << 32); }

// ---------------------------------------------------------------- copy calibration
// The practical streaming ceiling: one float4 per lane, non-temporal load
// and store (the fastest plain copy form measured on MI355X).
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy4(const f32x4* __restrict__ src, f32x4* __restrict__ dst, uint64_t n4) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i < n4)
    __builtin_nontemporal_store(__builtin_nontemporal_load((const LBF_GLOBAL f32x4*)src + i), (LBF_GLOBAL f32x4*)dst + i);
}

// ---------------------------------------------------------------- kernel tables
// Step kernels (PROP = false) and their propagation-only twins (PROP = true),
// flat tiling, with the streaming or (RES) the resident cache policy; the
// resident kernels exist for planes below 4 GiB only.
template <class M, int S, int P, bool W, bool PROP, bool RES>
void* step_ptr_b(int block) {
  switch (block) {
    case 64: return PROP ? (void*)&k_propagate<M, S, P, W, 64, RES> : (void*)&k_step<M, S, P, W, 64, RES>;
    case 128: return PROP ? (void*)&k_propagate<M, S, P, W, 128, RES> : (void*)&k_step<M, S, P, W, 128, RES>;
    case 256: return PROP ? (void*)&k_propagate<M, S, P, W, 256, RES> : (void*)&k_step<M, S, P, W, 256, RES>;
    case 512: return PROP ? (void*)&k_propagate<M, S, P, W, 512, RES> : (void*)&k_step<M, S, P, W, 512, RES>;
  }
  return nullptr;
}
template <class M, int S, int P, bool PROP>
void* step_ptr_p(bool wide, bool res, int block) {
  if (wide) return res ? nullptr : step_ptr_b<M, S, P, true, PROP, false>(block);
  return res ? step_ptr_b<M, S, P, false, PROP, true>(block) : step_ptr_b<M, S, P, false, PROP, false>(block);
}
template <class M, int S, bool PROP>
void* step_ptr_s(int parity, bool wide, bool res, int block) {
  return parity ? step_ptr_p<M, S, 1, PROP>(wide, res, block) : step_ptr_p<M, S, 0, PROP>(wide, res, block);
}
template <class M, bool PROP>
void* step_ptr_m(int storage, int parity, bool wide, bool res, int block) {
  switch (storage) {
    case LB_F32: return step_ptr_s<M, ST_F32, PROP>(parity, wide, res, block);
    case LB_F16: return step_ptr_s<M, ST_F16, PROP>(parity, wide, res, block);
    case LB_BF16: return step_ptr_s<M, ST_BF16, PROP>(parity, wide, res, block);
  }
  return nullptr;
}
void* step_ptr(int lattice, int storage, int parity, bool wide, bool res, int block, bool prop) {
  if (prop)
    return lattice == LB_D2Q9 ? step_ptr_m<D2Q9, true>(storage, parity, wide, res, block)
                              : step_ptr_m<D3Q19, true>(storage, parity, wide, res, block);
  return lattice == LB_D2Q9 ? step_ptr_m<D2Q9, false>(storage, parity, wide, res, block)
                            : step_ptr_m<D3Q19, false>(storage, parity, wide, res, block);
}

// Row-tiled step kernels and their propagation-only twins (non-wide
// lattices only), both cache policies.
template <class M, int S, int P, bool PROP, bool RES>
void* rows_ptr_b(int block) {
  switch (block) {
    case 64: return PROP ? (void*)&k_propagate_rows<M, S, P, 64, RES> : (void*)&k_step_rows<M, S, P, 64, RES>;
    case 128: return PROP ? (void*)&k_propagate_rows<M, S, P, 128, RES> : (void*)&k_step_rows<M, S, P, 128, RES>;
    case 256: return PROP ? (void*)&k_propagate_rows<M, S, P, 256, RES> : (void*)&k_step_rows<M, S, P, 256, RES>;
    case 512: return PROP ? (void*)&k_propagate_rows<M, S, P, 512, RES> : (void*)&k_step_rows<M, S, P, 512, RES>;
  }
  return nullptr;
}
template <class M, int S, bool PROP>
void* rows_ptr_s(int parity, bool res, int block) {
  if (parity) return res ? rows_ptr_b<M, S, 1, PROP, true>(block) : rows_ptr_b<M, S, 1, PROP, false>(block);
  return res ? rows_ptr_b<M, S, 0, PROP, true>(block) : rows_ptr_b<M, S, 0, PROP, false>(block);
}
template <class M, bool PROP>
void* rows_ptr_m(int storage, int parity, bool res, int block) {
  switch (storage) {
    case LB_F32: return rows_ptr_s<M, ST_F32, PROP>(parity, res, block);
    case LB_F16: return rows_ptr_s<M, ST_F16, PROP>(parity, res, block);
    case LB_BF16: return rows_ptr_s<M, ST_BF16, PROP>(parity, res, block);
  }
  return nullptr;
}
void* rows_ptr(int lattice, int storage, int parity, bool res, int block, bool prop) {
  if (prop)
    return lattice == LB_D2Q9 ? rows_ptr_m<D2Q9, true>(storage, parity, res, block)
                              : rows_ptr_m<D3Q19, true>(storage, parity, res, block);
  return lattice == LB_D2Q9 ? rows_ptr_m<D2Q9, false>(storage, parity, res, block)
                            : rows_ptr_m<D3Q19, false>(storage, parity, res, block);
}

// Fused two-step passes (D3Q19 and D2Q9): step kernels and their
// propagation-only twins; wide: planes of 4 GiB or more, addressed one
// z-plane (row) at a time.
template <int S, bool W>
void* step2_ptr_s(int lattice, bool prop) {
  if (lattice == LB_D2Q9) return prop ? (void*)&k_step2_2d<S, true, W> : (void*)&k_step2_2d<S, false, W>;
  return prop ? (void*)&k_step2<S, true, W> : (void*)&k_step2<S, false, W>;
}
template <bool W>
void* step2_ptr_w(int lattice, int storage, bool prop) {
  switch (storage) {
    case LB_F32: return step2_ptr_s<ST_F32, W>(lattice, prop);
    case LB_F16: return step2_ptr_s<ST_F16, W>(lattice, prop);
    case LB_BF16: return step2_ptr_s<ST_BF16, W>(lattice, prop);
  }
  return nullptr;
}
void* step2_ptr(int lattice, int storage, bool wide, bool prop) {
  return wide ? step2_ptr_w<true>(lattice, storage, prop) : step2_ptr_w<false>(lattice, storage, prop);
}

// Initial states (rest, thermal, fields), gathers (populations, moments,
// modes) and the health check; init and gather kinds are template
// parameters of their kernels.
enum KernelKind {
  KK_INIT_REST, KK_INIT_THERMAL, KK_INIT_FIELDS,
  KK_GATHER_POPULATIONS, KK_GATHER_MOMENTS, KK_GATHER_MODES,
  KK_CHECK
};
template <class M, int S, int P, bool W>
void* aux_ptr3(KernelKind kk) {
  switch (kk) {
    case KK_INIT_REST: return (void*)&k_init<M, S, P, W, 0>;
    case KK_INIT_THERMAL: return (void*)&k_init<M, S, P, W, 1>;
    case KK_INIT_FIELDS: return (void*)&k_init<M, S, P, W, 2>;
    case KK_GATHER_POPULATIONS: return (void*)&k_gather<M, S, P, W, 0>;
    case KK_GATHER_MOMENTS: return (void*)&k_gather<M, S, P, W, 1>;
    case KK_GATHER_MODES: return (void*)&k_gather<M, S, P, W, 2>;
    case KK_CHECK: return (void*)&k_check<M, S, P, W>;
  }
  return nullptr;
}
template <class M, int S>
void* aux_ptr_s(KernelKind kk, int parity, bool wide) {
  if (parity) return wide ? aux_ptr3<M, S, 1, true>(kk) : aux_ptr3<M, S, 1, false>(kk);
  return wide ? aux_ptr3<M, S, 0, true>(kk) : aux_ptr3<M, S, 0, false>(kk);
}
template <class M>
void* aux_ptr_m(KernelKind kk, int storage, int parity, bool wide) {
  switch (storage) {
    case LB_F32: return aux_ptr_s<M, ST_F32>(kk, parity, wide);
    case LB_F16: return aux_ptr_s<M, ST_F16>(kk, parity, wide);
    case LB_BF16: return aux_ptr_s<M, ST_BF16>(kk, parity, wide);
  }
  return nullptr;
}
void* aux_ptr(KernelKind kk, int lattice, int storage, int parity, bool wide) {
  return lattice == LB_D2Q9 ? aux_ptr_m<D2Q9>(kk, storage, parity, wide)
                            : aux_ptr_m<D3Q19>(kk, storage, parity, wide);
}

}  // namespace

// ---------------------------------------------------------------- context
struct lb_ctx {
  bool owner = true;            // false for views
  lb_ctx* parent = nullptr;     // batch of a view
  int replica = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int storage = LB_F32;
  int lattice = LB_D3Q19;
  bool wide = false;
  std::vector<lb_params> reps;  // one per lattice (1 for a single lattice)
  std::vector<uint64_t> offsets;
  int64_t t = 0;                // host mirror of *d_t

  // device metadata: [d_t (8 B) | result (5 doubles) | pad] [partials] [lats] [lats in tile order] [blk]
  char* d_meta = nullptr;
  uint64_t* d_t = nullptr;
  double* d_result = nullptr;
  double* d_partial = nullptr;
  LatDesc* d_lats = nullptr;
  LatDesc* d_tile_lats = nullptr;
  uint32_t* d_blk = nullptr;
  uint32_t* d_blk_rows = nullptr;   // tile prefix of the row tiling
  double* h_result = nullptr;   // pinned
  std::vector<LatDesc> lats;

  lb_schedule sched{256, 0, 16, {0, 0}, {1, 0}, 0, 0, 0};
  // Lattices in tile order are split into groups of consecutive lattices
  // (one group unless sched.group_mb is set); every step is one launch per
  // group, and a graph chunk runs all its steps on one group before the next.
  struct Group {
    uint32_t first, count;      // lattices [first, first + count) in tile order
    uint32_t grid, grid_rows;   // workgroups per launch, flat and row tiling
  };
  std::vector<Group> groups;

  // graph of sched.graph_chunk steps starting at even t, plus the counter advance
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  struct StepArgs {
    const LatDesc* lats;
    const uint32_t* blk;
    uint32_t nlat;
    uint32_t remap;
    const uint64_t* d_t;
    uint32_t t_off;
  };
  std::vector<StepArgs> graph_args;
  struct AdvArgs {
    uint64_t* d_t;
    uint64_t n;
  } adv_args;

  // fused schedule: the second state buffer (library-owned), the descriptors
  // of both buffers (d_f2[0] the state, d_f2[1] the second buffer), the tile
  // grid of k_step2 (D3Q19) or k_step2_2d (D2Q9), the planes (rows) a tile
  // walks and the workgroup size
  char* d_state_b = nullptr;
  LatDesc* d_f2 = nullptr;
  uint32_t f2_ntx = 0, f2_nty = 0, f2_ntz = 0, f2_len = 0;
  int f2_threads = 0;
  struct F2Args {
    const LatDesc* src;
    uint64_t dst;
    const uint64_t* d_t;
    uint32_t t_off, ntx, nty, zlen;
  };
  std::vector<F2Args> graph_f2_args;

  lb_ctx* root() { return parent ? parent : this; }
};

namespace {

void drop_graph(lb_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

// Planes (D3Q19: z-planes; D2Q9: rows) per tile column of the fused pass,
// for `across` tiles per plane, `extent` planes and `slots` tiles resident
// on the device at a time (CUs times tiles per CU).  A pass runs in rounds
// of `slots` tiles, each round taking one tile's chunk + 3 phases plus about
// one of set-up.  Lattices with many rounds take 32 planes (the fastest at
// 512^3 and 16384^2); with few, a last round that leaves many CUs idle costs
// a large part of the pass, and the chunk length from 8 to 32 that
// minimises the estimate is taken instead (256^3 on 256 CUs: 22 planes, 5
// rounds of 26 phases instead of 4 of 36).  The result does not depend on it.
uint32_t fused_chunk(uint64_t across, uint32_t extent, uint32_t slots) {
  constexpr uint32_t LONG = 32;
  auto tiles = [&](uint32_t z) { return across * ((extent + z - 1u) / z); };
  auto cost = [&](uint32_t z) { return ((tiles(z) + slots - 1u) / slots) * (uint64_t)(z + 4u); };
  if (tiles(LONG) >= 16ull * slots) return LONG;
  uint32_t best = LONG;
  for (uint32_t z = 8; z < LONG; ++z)
    if (cost(z) < cost(best)) best = z;
  return best;
}

// Tile order, replica groups and the per-lattice block prefixes (relative to
// the first tile of the lattice's group) for the current schedule.
int upload_schedule(lb_ctx* c) {
  const int nlat = (int)c->lats.size();
  std::vector<int> order(nlat);
  for (int i = 0; i < nlat; ++i) order[i] = i;
  if (c->sched.order == 1)
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return c->lats[a].nsites > c->lats[b].nsites; });
  else if (c->sched.order == 2)
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return c->lats[a].nsites < c->lats[b].nsites; });
  std::vector<LatDesc> tl(nlat);
  std::vector<uint32_t> blk(nlat + 1), blk_rows(nlat + 1);
  std::vector<lb_ctx::Group> groups;
  const uint64_t cap = (uint64_t)c->sched.group_mb << 20;  // state bytes per group; 0: one group
  const uint64_t per_site = (uint64_t)q_of(c->lattice) * elem_size(c->storage);
  uint64_t acc = 0, acc_rows = 0, bytes = 0;
  uint32_t first = 0;
  auto close_group = [&](uint32_t end) {
    groups.push_back({first, end - first, (uint32_t)acc, (uint32_t)acc_rows});
    return acc < (1ull << 31) && acc_rows < (1ull << 31);
  };
  for (int i = 0; i < nlat; ++i) {
    tl[i] = c->lats[order[i]];
    const uint64_t b = (per_site * tl[i].nsites + 255) & ~255ull;
    if (cap && (uint32_t)i > first && bytes + b > cap) {  // a lattice above the cap is a group of its own
      if (!close_group((uint32_t)i)) return fail(LB_EUNSUPPORTED, "too many workgroups for one launch");
      first = (uint32_t)i;
      acc = acc_rows = bytes = 0;
    }
    bytes += b;
    tl[i].segs = (tl[i].nx + c->sched.block - 1) / c->sched.block;
    div_magic(tl[i].segs, tl[i].ds_m, tl[i].ds_s1, tl[i].ds_s2);
    blk[i] = (uint32_t)acc;
    blk_rows[i] = (uint32_t)acc_rows;
    acc += (tl[i].nsites + c->sched.block - 1) / c->sched.block;
    acc_rows += (uint64_t)tl[i].ny * tl[i].nz * tl[i].segs;
  }
  if (!close_group((uint32_t)nlat)) return fail(LB_EUNSUPPORTED, "too many workgroups for one launch");
  blk[nlat] = (uint32_t)acc;
  blk_rows[nlat] = (uint32_t)acc_rows;
  c->groups = groups;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(c->d_tile_lats, tl.data(), sizeof(LatDesc) * nlat, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->d_blk, blk.data(), sizeof(uint32_t) * (nlat + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->d_blk_rows, blk_rows.data(), sizeof(uint32_t) * (nlat + 1), hipMemcpyHostToDevice));
  if (c->sched.fused) {
    // descriptors of the state buffer and of the second buffer (same geometry)
    LatDesc f2[2] = {c->lats[0], c->lats[0]};
    f2[1].base = (uint64_t)(uintptr_t)c->d_state_b;
    HIP_TRY(hipMemcpy(c->d_f2, f2, sizeof(f2), hipMemcpyHostToDevice));
    const bool d2 = c->lattice == LB_D2Q9;
    c->f2_threads = d2 ? F2D_THREADS : F2_THREADS;
    int cus = 0, per_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, step2_ptr(c->lattice, c->storage, c->wide, false),
                                                         c->f2_threads, 0));
    const uint32_t slots = (uint32_t)std::max(1, cus * per_cu);
    if (d2) {
      c->f2_ntx = (f2[0].nx + (uint32_t)F2D_W - 1u) / (uint32_t)F2D_W;
      c->f2_len = fused_chunk(c->f2_ntx, f2[0].ny, slots);
      c->f2_nty = (f2[0].ny + c->f2_len - 1u) / c->f2_len;
      c->f2_ntz = 1;
    } else {
      c->f2_ntx = (f2[0].nx + 63u) / 64u;
      c->f2_nty = (f2[0].ny + (uint32_t)F2_TY - 1u) / (uint32_t)F2_TY;
      c->f2_len = fused_chunk((uint64_t)c->f2_ntx * c->f2_nty, f2[0].nz, slots);
      c->f2_ntz = (f2[0].nz + c->f2_len - 1u) / c->f2_len;
    }
  }
  drop_graph(c);
  return LB_OK;
}

// The fused passes take one lattice and address its planes one z-plane
// (D3Q19) or one row (D2Q9) at a time, so a plane may exceed 4 GiB but such
// a slice may not.
bool fused_eligible(const lb_ctx* c) {
  if (c->reps.size() != 1 || (c->lattice != LB_D3Q19 && c->lattice != LB_D2Q9)) return false;
  const lb_params& p = c->reps[0];
  const uint64_t slice = (uint64_t)p.nx * (c->lattice == LB_D2Q9 ? 1u : (uint64_t)p.ny) * elem_size(c->storage);
  return slice < (1ull << 32);
}

// The fused schedule's second buffer: allocated once, the size of the state,
// if the device has room for it beside a margin of 1 GiB.
int ensure_state_b(lb_ctx* c) {
  if (c->d_state_b) return LB_OK;
  const size_t bytes = (size_t)q_of(c->lattice) * sites_of(c->reps[0]) * elem_size(c->storage);
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  if (free_b < bytes + (1ull << 30))
    return fail(LB_EUNSUPPORTED, "not enough free device memory for the fused schedule's second state buffer");
  const hipError_t e = hipMalloc(&c->d_state_b, bytes);
  if (e != hipSuccess) {
    c->d_state_b = nullptr;
    (void)hipGetLastError();
    return fail(LB_EUNSUPPORTED, std::string("second state buffer of the fused schedule: ") + hipGetErrorString(e));
  }
  return LB_OK;
}

void release_state_b(lb_ctx* c) {
  if (!c->d_state_b) return;
  drop_graph(c);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->d_state_b);
  c->d_state_b = nullptr;
}

// Kernel, grid, workgroup size, lattices and tile prefix of the launch of
// group g in a step of the given parity.
struct StepLaunch {
  void* fn;
  uint32_t grid;
  int block;
  const LatDesc* lats;
  const uint32_t* blk;
  uint32_t nlat;
};
StepLaunch step_launch(const lb_ctx* c, int parity, size_t g, bool prop = false) {
  const lb_ctx::Group& G = c->groups[g];
  const bool res = c->sched.resident != 0;
  if (c->sched.tiling[parity])
    return {rows_ptr(c->lattice, c->storage, parity, res, c->sched.block, prop), G.grid_rows, c->sched.block,
            c->d_tile_lats + G.first, c->d_blk_rows + G.first, G.count};
  return {step_ptr(c->lattice, c->storage, parity, c->wide, res, c->sched.block, prop), G.grid, c->sched.block,
          c->d_tile_lats + G.first, c->d_blk + G.first, G.count};
}

// One step of every group.  prop: the propagation-only kernels of the same
// schedule instead.
int launch_step(lb_ctx* c, uint32_t t_off, int parity, bool prop = false) {
  for (size_t g = 0; g < c->groups.size(); ++g) {
    const StepLaunch sl = step_launch(c, parity, g, prop);
    if (!sl.fn) return fail(LB_EINVAL, "no step kernel for this schedule");
    lb_ctx::StepArgs a{sl.lats, sl.blk, sl.nlat, (uint32_t)c->sched.xcd_remap[parity], c->d_t, t_off};
    void* args[] = {&a.lats, &a.blk, &a.nlat, &a.remap, &a.d_t, &a.t_off};
    HIP_TRY(hipLaunchKernel(sl.fn, dim3(sl.grid), dim3(sl.block), args, 0, c->stream));
  }
  return LB_OK;
}

// One fused pass (two steps from even t + t_off): state buffer -> second
// buffer (to_b) or back.
lb_ctx::F2Args pass_args(const lb_ctx* c, uint32_t t_off, bool to_b) {
  return {to_b ? c->d_f2 : c->d_f2 + 1,
          to_b ? (uint64_t)(uintptr_t)c->d_state_b : c->lats[0].base,
          c->d_t, t_off, c->f2_ntx, c->f2_nty, c->f2_len};
}

int launch_pass(lb_ctx* c, uint32_t t_off, bool to_b, bool prop = false) {
  lb_ctx::F2Args a = pass_args(c, t_off, to_b);
  void* args[] = {&a.src, &a.dst, &a.d_t, &a.t_off, &a.ntx, &a.nty, &a.zlen};
  HIP_TRY(hipLaunchKernel(step2_ptr(c->lattice, c->storage, c->wide, prop), dim3(c->f2_ntx * c->f2_nty * c->f2_ntz),
                          dim3(c->f2_threads), args, 0, c->stream));
  return LB_OK;
}

int launch_advance(lb_ctx* c, uint64_t n) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, c->stream, c->d_t, n);
  HIP_TRY(hipGetLastError());
  return LB_OK;
}

// A chain of graph_chunk steps of each group in turn (all steps of one group
// before the next, so a group whose state fits in the Infinity Cache stays
// there), then the counter advance.  Under the fused schedule (one lattice)
// the chain is fused passes, out to the second buffer and back, for every
// four steps, and AA steps for the rest of the chunk.
int build_graph(lb_ctx* c) {
  drop_graph(c);
  const int K = c->sched.graph_chunk;
  const int units = c->sched.fused ? K / 4 : 0;  // pairs of fused passes
  HIP_TRY(hipGraphCreate(&c->graph, 0));
  c->graph_args.assign((K - 4 * units) * c->groups.size(), {});
  c->graph_f2_args.assign(2 * units, {});
  hipGraphNode_t prev = nullptr;
  auto add_node = [&](void* fn, uint32_t grid, int block, void** args) -> int {
    hipKernelNodeParams kp{};
    kp.func = fn;
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(block);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    HIP_TRY(hipGraphAddKernelNode(&node, c->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
    prev = node;
    return LB_OK;
  };
  for (int p = 0; p < 2 * units; ++p) {
    c->graph_f2_args[p] = pass_args(c, (uint32_t)(2 * p), (p & 1) == 0);
    lb_ctx::F2Args& a = c->graph_f2_args[p];
    void* args[] = {&a.src, &a.dst, &a.d_t, &a.t_off, &a.ntx, &a.nty, &a.zlen};
    int rc = add_node(step2_ptr(c->lattice, c->storage, c->wide, false), c->f2_ntx * c->f2_nty * c->f2_ntz, c->f2_threads,
                      args);
    if (rc) return rc;
  }
  const int K1 = K - 4 * units;  // AA steps per group, from step 4 * units of the chunk
  for (size_t n = 0; n < c->graph_args.size(); ++n) {
    const size_t g = n / K1;
    const int s = 4 * units + (int)(n % K1);
    const StepLaunch sl = step_launch(c, s & 1, g);
    if (!sl.fn) return fail(LB_EINVAL, "no step kernel for this schedule");
    c->graph_args[n] = {sl.lats, sl.blk, sl.nlat, (uint32_t)c->sched.xcd_remap[s & 1], c->d_t, (uint32_t)s};
    lb_ctx::StepArgs& a = c->graph_args[n];
    void* args[] = {&a.lats, &a.blk, &a.nlat, &a.remap, &a.d_t, &a.t_off};
    int rc = add_node(sl.fn, sl.grid, sl.block, args);
    if (rc) return rc;
  }
  c->adv_args = {c->d_t, (uint64_t)K};
  void* aargs[] = {&c->adv_args.d_t, &c->adv_args.n};
  int rc = add_node((void*)&k_advance, 1, 64, aargs);
  if (rc) return rc;
  HIP_TRY(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
  return LB_OK;
}

// m steps launched one by one (prop: the propagation-only kernels), then the
// counter advance.  Under the fused schedule, from even t, every four steps
// run as two fused passes (out to the second buffer and back).
int direct_steps(lb_ctx* c, int64_t m, bool prop = false) {
  int64_t s = 0;
  if (c->sched.fused && !(c->t & 1)) {
    for (; s + 4 <= m; s += 4) {
      int rc = launch_pass(c, (uint32_t)s, true, prop);
      if (!rc) rc = launch_pass(c, (uint32_t)s + 2u, false, prop);
      if (rc) return rc;
    }
  }
  for (; s < m; ++s) {
    int rc = launch_step(c, (uint32_t)s, (int)((c->t + s) & 1), prop);
    if (rc) return rc;
  }
  int rc = launch_advance(c, (uint64_t)m);
  if (rc) return rc;
  c->t += m;
  return LB_OK;
}

int advance(lb_ctx* c, int64_t n) {
  if (n < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  HIP_TRY(hipSetDevice(c->device));
  const int K = c->sched.graph_chunk;
  if (n > 0 && (c->t & 1)) {
    int rc = direct_steps(c, 1);
    if (rc) return rc;
    --n;
  }
  // a replay holds K launches per replica group; past 2^16 kernel nodes the
  // steps are launched directly instead (same work, more host launches)
  const bool graphable = (uint64_t)K * c->groups.size() <= (1u << 16);
  if (n >= K && graphable) {
    if (!c->graph_exec) {
      int rc = build_graph(c);
      if (rc) return rc;
    }
    while (n >= K) {
      HIP_TRY(hipGraphLaunch(c->graph_exec, c->stream));
      c->t += K;
      n -= K;
    }
  }
  while (n > 0) {  // the device counter advances every K steps, as in a replay
    const int64_t m = std::min<int64_t>(n, K);
    int rc = direct_steps(c, m);
    if (rc) return rc;
    n -= m;
  }
  return LB_OK;
}

int alloc_meta(lb_ctx* c) {
  const int nlat = (int)c->lats.size();
  const size_t head = 256;
  const size_t part = sizeof(double) * 5 * CHECK_BLOCKS;
  const size_t lats = sizeof(LatDesc) * nlat;
  const size_t blk = sizeof(uint32_t) * (nlat + 1);
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t f2 = up(2 * sizeof(LatDesc));
  const size_t total = head + up(part) + 2 * up(lats) + 2 * up(blk) + f2;
  HIP_TRY(hipMalloc(&c->d_meta, total));
  c->d_t = reinterpret_cast<uint64_t*>(c->d_meta);
  c->d_result = reinterpret_cast<double*>(c->d_meta + 64);
  c->d_partial = reinterpret_cast<double*>(c->d_meta + head);
  c->d_lats = reinterpret_cast<LatDesc*>(c->d_meta + head + up(part));
  c->d_tile_lats = reinterpret_cast<LatDesc*>(c->d_meta + head + up(part) + up(lats));
  c->d_blk = reinterpret_cast<uint32_t*>(c->d_meta + head + up(part) + 2 * up(lats));
  c->d_blk_rows = reinterpret_cast<uint32_t*>(c->d_meta + head + up(part) + 2 * up(lats) + up(blk));
  c->d_f2 = reinterpret_cast<LatDesc*>(c->d_meta + head + up(part) + 2 * up(lats) + 2 * up(blk));
  HIP_TRY(hipHostMalloc((void**)&c->h_result, sizeof(double) * 5, hipHostMallocDefault));
  HIP_TRY(hipMemcpy(c->d_lats, c->lats.data(), lats, hipMemcpyHostToDevice));
  return LB_OK;
}

void free_ctx(lb_ctx* c) {
  if (!c) return;
  if (c->owner) {
    drop_graph(c);
    release_state_b(c);
    if (c->d_meta) (void)hipFree(c->d_meta);
    if (c->h_result) (void)hipHostFree(c->h_result);
  }
  delete c;
}

int init_lattice(lb_ctx* c, int idx, int kind, const float* d_fields, int parity) {
  const lb_params& p = c->reps[idx];
  const uint32_t n = (uint32_t)sites_of(p);
  const KernelKind kk = kind == LB_INIT_REST ? KK_INIT_REST : kind == LB_INIT_THERMAL ? KK_INIT_THERMAL : KK_INIT_FIELDS;
  void* fn = aux_ptr(kk, c->lattice, c->storage, parity, c->wide);
  const LatDesc* L = c->d_lats + idx;
  const float* f = d_fields;
  void* args[] = {&L, &f};
  HIP_TRY(hipLaunchKernel(fn, dim3((uint32_t)(((uint64_t)n + 255) / 256)), dim3(256), args, 0, c->stream));
  return LB_OK;
}

// Default schedule, from measurements on MI355X (512^3 D3Q19 and 16384^2
// D2Q9 boxes): fp32 runs the even step row-tiled and the odd step flat, both
// without XCD remapping; the 16-bit forms run the even step flat and the odd
// step row-tiled, with XCD groups of 8 consecutive tiles on D3Q19 and no
// remapping on D2Q9 (groups of 8 made the D2Q9 bf16 step 10% slower).
// State of 32 MB to 320 MB on one lattice runs resident in the Infinity
// Cache (4-14% faster from 96^3 to 160^3), unless fp32 state above 256 MiB
// (D2Q9: 32 MiB) takes the fused pass (below); a batch whose replicas each
// fit in 224 MiB runs resident groups of 224 MiB once it holds 32 MB or more
// (the 96-replica fp32 ensemble: 11% faster).  Below 32 MB the streaming
// policy measured as fast or faster.  lb_autotune refines it for a given
// workload.
int default_schedule(lb_ctx* c) {
  if (c->storage == LB_F32) c->sched = lb_schedule{256, 0, 16, {0, 0}, {1, 0}, 0, 0, 0};
  else if (c->lattice == LB_D2Q9) c->sched = lb_schedule{256, 0, 16, {0, 0}, {0, 1}, 0, 0, 0};
  else c->sched = lb_schedule{256, 0, 16, {8, 8}, {0, 1}, 0, 0, 0};
  if (c->wide) c->sched.tiling[0] = c->sched.tiling[1] = 0;
  uint64_t total = 0, largest = 0;
  for (const lb_params& p : c->reps) {
    const uint64_t b = (uint64_t)q_of(p.lattice) * sites_of(p) * elem_size(p.storage);
    total += b;
    largest = std::max(largest, b);
  }
  constexpr uint64_t MB = 1000000, MIB = 1ull << 20;
  if (!c->wide) {
    if (c->reps.size() == 1) {
      if (total >= 32 * MB && total <= 320 * MB) c->sched.resident = 1;
    } else if (total >= 32 * MB && largest <= 224 * MIB) {
      c->sched.resident = 1;
      c->sched.group_mb = 224;
    }
  }
  // fp32 state beyond the cache streams through HBM: two fused steps per
  // launch move about half the bytes (512^3 D3Q19: 5.2-5.4 against 7.2 ms
  // per two steps; 16384^2 D2Q9: 4.35 against 6.84 ms), when the second
  // buffer fits on the device; planes of 4 GiB or more included.  Measured
  // crossovers against the resident AA steps: D3Q19 between 152^3 (267 MB,
  // AA 8% faster) and 156^3 (289 MB, fused 13% faster), D2Q9 between 724^2
  // (19 MB, AA 6% faster) and 1024^2 (38 MB, fused 11% faster).  The 16-bit
  // forms keep one step per launch: their collision already keeps the VALU
  // busy enough that the fused pass is slower.
  const uint64_t fused_above = c->lattice == LB_D2Q9 ? 32 * MIB : 256 * MIB;
  if (c->storage == LB_F32 && fused_eligible(c) && total > fused_above) {
    const std::string keep = g_last_error;
    if (ensure_state_b(c) == LB_OK) c->sched.fused = 1;
    else g_last_error = keep;  // no room: one step per launch, not an error
  }
  return upload_schedule(c);
}

// Local view of one lattice for gathers: (ctx owning the metadata, index).
struct View {
  lb_ctx* root;
  int idx;
};
View view_of(lb_ctx* c) { return c->parent ? View{c->parent, c->replica} : View{c, 0}; }

int gather(lb_ctx* c, int what, float* d_out) {
  if (!c) return fail(LB_EINVAL, "ctx is NULL");
  if (!d_out) return fail(LB_EINVAL, "output pointer is NULL");
  View v = view_of(c);
  lb_ctx* r = v.root;
  if (r->reps.size() > 1 && !c->parent) return fail(LB_EINVAL, "gathers on a batch need a view (lb_batch_view)");
  HIP_TRY(hipSetDevice(r->device));
  const uint32_t n = (uint32_t)sites_of(r->reps[v.idx]);
  const KernelKind kk = what == 0 ? KK_GATHER_POPULATIONS : what == 1 ? KK_GATHER_MOMENTS : KK_GATHER_MODES;
  void* fn = aux_ptr(kk, r->lattice, r->storage, (int)(r->t & 1), r->wide);
  const LatDesc* L = r->d_lats + v.idx;
  float* o = d_out;
  void* args[] = {&L, &o};
  HIP_TRY(hipLaunchKernel(fn, dim3((uint32_t)(((uint64_t)n + 255) / 256)), dim3(256), args, 0, r->stream));
  return LB_OK;
}

}  // namespace

// ---------------------------------------------------------------- steps without allocation
// lb_step_noalloc keeps what a context would hold in device memory (lattice
// descriptors, tile prefixes, the step counter) in one file-scope device
// array instead.  Host code never uses the array's name as an address: its
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t NA_OFF_T = 0;                                          // uint64 step counter
constexpr size_t NA_OFF_BLK = 256;                                      // flat tile prefix
constexpr size_t NA_OFF_BLKR = NA_OFF_BLK + 4 * (LB_NOALLOC_MAX_REPLICAS + 1 + 63);  // row tile prefix
constexpr size_t NA_OFF_DESC = (NA_OFF_BLKR + 4 * (LB_NOALLOC_MAX_REPLICAS + 1) + 255) & ~(size_t)255;
constexpr size_t NA_BYTES = NA_OFF_DESC + sizeof(LatDesc) * LB_NOALLOC_MAX_REPLICAS;
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_CHUNK = 8;  // descriptors per setup launch (passed by value: under 4 KB of arguments)
struct NaDescs {
  LatDesc d[NA_CHUNK];
  uint32_t n;
};
struct NaMeta {
  uint32_t blk[LB_NOALLOC_MAX_REPLICAS + 1];
  uint32_t blk_rows[LB_NOALLOC_MAX_REPLICAS + 1];
  uint64_t t;
  uint32_t n;
};
static_assert(sizeof(NaDescs) < 4000 && sizeof(NaMeta) < 4000, "setup kernel arguments must stay below 4 KB");

__global__ void __launch_bounds__(64) k_noalloc_descs(NaDescs c, LatDesc* __restrict__ dst) {
  constexpr uint32_t W = sizeof(LatDesc) / 4;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&c.d[0]);
  uint32_t* out = reinterpret_cast<uint32_t*>(dst);
  for (uint32_t i = threadIdx.x; i < c.n * W; i += 64) out[i] = src[i];
}

__global__ void __launch_bounds__(64) k_noalloc_meta(NaMeta m, uint32_t* __restrict__ blk,
                                                     uint32_t* __restrict__ blk_rows, uint64_t* __restrict__ d_t) {
  for (uint32_t i = threadIdx.x; i <= m.n; i += 64) {
    blk[i] = m.blk[i];
    blk_rows[i] = m.blk_rows[i];
  }
  if (threadIdx.x == 0) *d_t = m.t;
}

// Device address of `scratch` on the current device, looked up once per device.
int noalloc_scratch(int device, unsigned char** out) {
  constexpr int MAXDEV = 64;
  static std::mutex mu;
  static unsigned char* addr[MAXDEV] = {};
  if (device < 0 || device >= MAXDEV) return fail(LB_EUNSUPPORTED, "lb_step_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[device] = static_cast<unsigned char*>(p);
  }
  *out = addr[device];
  return LB_OK;
}

// ================================================================ C ABI
extern "C" {

size_t lb_state_bytes(const lb_params* p) {
  if (validate(p) != LB_OK) return 0;
  return (size_t)(q_of(p->lattice) * sites_of(*p) * elem_size(p->storage));
}

const char* lb_strerror(int code) {
  switch (code) {
    case LB_OK: return "success";
    case LB_EINVAL: return "invalid argument";
    case LB_EDEVICE: return "HIP device or launch failure";
    case LB_ESTATE: return "state holds non-finite populations or rho <= 0";
    case LB_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char* lb_last_error(void) { return g_last_error.c_str(); }

int lb_init(const lb_params* p, void* d_state, void* hip_stream, int32_t init_kind, const float* d_fields,
            int64_t t0, lb_ctx** out) {
  if (!out) return fail(LB_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (!d_state) return fail(LB_EINVAL, "d_state is NULL");
  if (((uintptr_t)d_state & 255) != 0) return fail(LB_EINVAL, "d_state must be 256-byte aligned");
  if (init_kind < LB_INIT_REST || init_kind > LB_INIT_KEEP) return fail(LB_EINVAL, "unknown init_kind");
  if (init_kind == LB_INIT_FIELDS && !d_fields) return fail(LB_EINVAL, "LB_INIT_FIELDS needs d_fields");
  if (t0 < 0) return fail(LB_EINVAL, "t0 must be >= 0");

  lb_ctx* c = new lb_ctx();
  c->stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return fail(LB_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  c->storage = p->storage;
  c->lattice = p->lattice;
  c->wide = is_wide(*p);
  c->reps.push_back(*p);
  c->offsets.push_back(0);
  c->lats.push_back(make_desc(*p, (uint64_t)(uintptr_t)d_state));
  c->t = t0;
  if ((rc = alloc_meta(c)) || (rc = default_schedule(c))) {
    free_ctx(c);
    return rc;
  }
  hipLaunchKernelGGL(k_set_t, dim3(1), dim3(64), 0, c->stream, c->d_t, (uint64_t)t0);
  e = hipGetLastError();
  if (e != hipSuccess) {
    free_ctx(c);
    return fail(LB_EDEVICE, std::string("k_set_t: ") + hipGetErrorString(e));
  }
  if (init_kind != LB_INIT_KEEP && (rc = init_lattice(c, 0, init_kind, d_fields, (int)(t0 & 1)))) {
    free_ctx(c);
    return rc;
  }
  if (p->storage == LB_BF16 && p->kT == 0.0)
    g_last_error = "warning: bf16 storage without thermal noise is biased (its rounding of slowly varying "
                   "fields does not average out: a shear wave decays about 2% too slowly); use fp16 or fp32 "
                   "for deterministic runs";
  *out = c;
  return LB_OK;
}

int lb_step(lb_ctx* ctx, int64_t nsteps) {
  if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
  if (ctx->parent) return fail(LB_EINVAL, "a view cannot step; step its batch");
  return advance(ctx, nsteps);
}

int lb_propagate(lb_ctx* ctx, int64_t nsteps) {
  if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
  if (ctx->parent) return fail(LB_EINVAL, "a view cannot step; step its batch");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return LB_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  // the same launches as lb_step's direct path (fused passes under the fused
  // schedule), with the propagation-only kernels
  if (ctx->t & 1) {
    int rc = direct_steps(ctx, 1, true);
    if (rc) return rc;
    --nsteps;
  }
  while (nsteps > 0) {
    const int64_t m = std::min<int64_t>(nsteps, 1024);
    int rc = direct_steps(ctx, m, true);
    if (rc) return rc;
    nsteps -= m;
  }
  return LB_OK;
}

int lb_populations(lb_ctx* ctx, float* d_out) { return gather(ctx, 0, d_out); }
int lb_moments(lb_ctx* ctx, float* d_out) { return gather(ctx, 1, d_out); }
int lb_modes(lb_ctx* ctx, float* d_out) { return gather(ctx, 2, d_out); }

int lb_check(lb_ctx* ctx, int64_t* n_bad, double* sums_out) {
  if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
  View v = view_of(ctx);
  lb_ctx* r = v.root;
  if (r->reps.size() > 1 && !ctx->parent) return fail(LB_EINVAL, "lb_check on a batch needs a view");
  HIP_TRY(hipSetDevice(r->device));
  void* fn = aux_ptr(KK_CHECK, r->lattice, r->storage, (int)(r->t & 1), r->wide);
  const LatDesc* L = r->d_lats + v.idx;
  double* part = r->d_partial;
  void* args[] = {&L, &part};
  HIP_TRY(hipLaunchKernel(fn, dim3(CHECK_BLOCKS), dim3(256), args, 0, r->stream));
  hipLaunchKernelGGL(k_check_final, dim3(1), dim3(64), 0, r->stream, r->d_partial, CHECK_BLOCKS, r->d_result);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(r->h_result, r->d_result, sizeof(double) * 5, hipMemcpyDeviceToHost, r->stream));
  HIP_TRY(hipStreamSynchronize(r->stream));
  const lb_params& p = r->reps[v.idx];
  const int64_t bad = (int64_t)r->h_result[0];
  if (n_bad) *n_bad = bad;
  if (sums_out) {
    sums_out[0] = r->h_result[1] + p.rho0 * (double)sites_of(p);
    for (int a = 0; a < 3; ++a) sums_out[a + 1] = r->h_result[a + 2];
  }
  return bad > 0 ? fail(LB_ESTATE, "non-finite populations or rho <= 0 found") : LB_OK;
}

int64_t lb_step_count(const lb_ctx* ctx) {
  if (!ctx) return -1;
  return ctx->parent ? ctx->parent->t : ctx->t;
}

void lb_destroy(lb_ctx* ctx) {
  if (!ctx) return;
  if (ctx->owner) (void)hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
}

int lb_copy_rate(const void* d_src, void* d_dst, size_t bytes, int32_t reps, void* hip_stream, double* gbs_out) {
  if (!d_src || !d_dst || !gbs_out) return fail(LB_EINVAL, "NULL argument");
  if (((uintptr_t)d_src & 255) || ((uintptr_t)d_dst & 255)) return fail(LB_EINVAL, "buffers must be 256-byte aligned");
  if (bytes == 0 || bytes % 16) return fail(LB_EINVAL, "bytes must be a positive multiple of 16");
  const uint64_t n4 = bytes / 16;
  if ((n4 + 255) / 256 > 0x7FFFFFFFull) return fail(LB_EUNSUPPORTED, "copy too large for one launch");
  if (reps < 1) return fail(LB_EINVAL, "reps must be >= 1");
  const char* s = (const char*)d_src;
  const char* d = (const char*)d_dst;
  if (s < d + bytes && d < s + bytes) return fail(LB_EINVAL, "source and destination overlap");
  hipStream_t st = (hipStream_t)hip_stream;
  const dim3 grid((uint32_t)((n4 + 255) / 256));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_copy4, grid, dim3(256), 0, st, (const f32x4*)d_src, (f32x4*)d_dst, n4);  // warm-up
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    hipLaunchKernelGGL(k_copy4, grid, dim3(256), 0, st, (const f32x4*)d_src, (f32x4*)d_dst, n4);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(LB_EDEVICE, std::string("lb_copy_rate: ") + hipGetErrorString(e));
  *gbs_out = 2.0 * (double)bytes * reps / ((double)ms * 1e6);
  return LB_OK;
}

int lb_params_from_physical(double b, double h, double rho, double eta, double zeta, double kBT,
                            lb_params* p) {
  if (!p) return fail(LB_EINVAL, "params is NULL");
  const double v[5] = {b, h, rho, eta, zeta};
  for (double x : v)
    if (!(x > 0.0) || !std::isfinite(x)) return fail(LB_EINVAL, "b, h, rho, eta and zeta must be finite and > 0");
  if (!(kBT >= 0.0) || !std::isfinite(kBT)) return fail(LB_EINVAL, "k_B T must be finite and >= 0");
  if (p->lattice != LB_D3Q19 && p->lattice != LB_D2Q9) return fail(LB_EINVAL, "unknown lattice");
  const double cs2_hat = 1.0 / 3.0;  // both lattices, Sec. II
  const double d = p->lattice == LB_D2Q9 ? 2.0 : 3.0;
  const double eta_hat = eta * h / (rho * b * b * cs2_hat);
  const double zeta_hat = zeta * h / (rho * b * b * cs2_hat);
  const double mu = kBT * h * h / (cs2_hat * std::pow(b, d + 2.0));  // Sec. VI
  p->rho0 = 1.0;
  p->kT = cs2_hat * mu / rho;  // lattice units: mass unit rho b^d, mu_lattice = mu / rho
  p->gamma_shear = (2.0 * eta_hat - 1.0) / (2.0 * eta_hat + 1.0);
  p->gamma_bulk = (d * zeta_hat - 1.0) / (d * zeta_hat + 1.0);
  return LB_OK;
}

size_t lb_batch_pool_bytes(const lb_params* reps, int32_t nrep) {
  if (!reps || nrep < 1) return 0;
  size_t total = 0;
  for (int r = 0; r < nrep; ++r) {
    size_t b = lb_state_bytes(&reps[r]);
    if (!b) return 0;
    total += (b + 255) & ~(size_t)255;
  }
  return total;
}

size_t lb_batch_offset(const lb_params* reps, int32_t nrep, int32_t r) {
  if (!reps || r < 0 || r >= nrep) return 0;
  size_t off = 0;
  for (int i = 0; i < r; ++i) off += (lb_state_bytes(&reps[i]) + 255) & ~(size_t)255;
  return off;
}

int lb_batch_init(const lb_params* reps, int32_t nrep, void* d_pool, void* hip_stream, int32_t init_kind,
                  int64_t t0, lb_ctx** out) {
  if (!out) return fail(LB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!reps || nrep < 1) return fail(LB_EINVAL, "need at least one replica");
  for (int r = 0; r < nrep; ++r) {
    int rc = validate(&reps[r]);
    if (rc) return rc;
    if (reps[r].storage != reps[0].storage) return fail(LB_EINVAL, "all replicas need the same storage type");
    if (reps[r].lattice != reps[0].lattice) return fail(LB_EINVAL, "all replicas need the same lattice");
    if (is_wide(reps[r])) return fail(LB_EUNSUPPORTED, "replicas must hold < 4 GiB per population plane");
  }
  if (!d_pool || ((uintptr_t)d_pool & 255)) return fail(LB_EINVAL, "d_pool must be non-NULL and 256-byte aligned");
  if (init_kind == LB_INIT_FIELDS) return fail(LB_EUNSUPPORTED, "LB_INIT_FIELDS is not available for ensembles");
  if (init_kind < LB_INIT_REST || init_kind > LB_INIT_KEEP) return fail(LB_EINVAL, "unknown init_kind");
  if (t0 < 0) return fail(LB_EINVAL, "t0 must be >= 0");

  lb_ctx* c = new lb_ctx();
  c->stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return fail(LB_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  c->storage = reps[0].storage;
  c->lattice = reps[0].lattice;
  c->wide = false;
  uint64_t off = 0;  // running lb_batch_offset
  for (int r = 0; r < nrep; ++r) {
    c->reps.push_back(reps[r]);
    c->offsets.push_back(off);
    c->lats.push_back(make_desc(reps[r], (uint64_t)(uintptr_t)d_pool + off));
    off += (lb_state_bytes(&reps[r]) + 255) & ~(size_t)255;
  }
  c->t = t0;
  int rc;
  if ((rc = alloc_meta(c)) || (rc = default_schedule(c))) {
    free_ctx(c);
    return rc;
  }
  hipLaunchKernelGGL(k_set_t, dim3(1), dim3(64), 0, c->stream, c->d_t, (uint64_t)t0);
  e = hipGetLastError();
  if (e != hipSuccess) {
    free_ctx(c);
    return fail(LB_EDEVICE, std::string("k_set_t: ") + hipGetErrorString(e));
  }
  if (init_kind != LB_INIT_KEEP)
    for (int r = 0; r < nrep; ++r)
      if ((rc = init_lattice(c, r, init_kind, nullptr, (int)(t0 & 1)))) {
        free_ctx(c);
        return rc;
      }
  *out = c;
  return LB_OK;
}

int lb_batch_step(lb_ctx* batch, int64_t nsteps) {
  if (!batch) return fail(LB_EINVAL, "batch is NULL");
  if (batch->parent) return fail(LB_EINVAL, "a view cannot step; step its batch");
  return advance(batch, nsteps);
}

int lb_batch_view(lb_ctx* batch, int32_t replica, lb_ctx** view) {
  if (!batch || !view) return fail(LB_EINVAL, "NULL argument");
  *view = nullptr;
  if (batch->parent) return fail(LB_EINVAL, "cannot take a view of a view");
  if (replica < 0 || replica >= (int)batch->reps.size()) return fail(LB_EINVAL, "replica out of range");
  lb_ctx* v = new lb_ctx();
  v->owner = false;
  v->parent = batch;
  v->replica = replica;
  v->stream = batch->stream;
  v->device = batch->device;
  v->storage = batch->storage;
  v->lattice = batch->lattice;
  *view = v;
  return LB_OK;
}

int lb_get_schedule(const lb_ctx* ctx, lb_schedule* out) {
  if (!ctx || !out) return fail(LB_EINVAL, "NULL argument");
  *out = (ctx->parent ? ctx->parent : ctx)->sched;
  return LB_OK;
}

int lb_set_schedule(lb_ctx* ctx, const lb_schedule* s) {
  if (!ctx || !s) return fail(LB_EINVAL, "NULL argument");
  if (ctx->parent) return fail(LB_EINVAL, "set the schedule on the batch, not a view");
  if (s->block != 64 && s->block != 128 && s->block != 256 && s->block != 512)
    return fail(LB_EINVAL, "block must be 64, 128, 256 or 512");
  if (s->order < 0 || s->order > 2) return fail(LB_EINVAL, "order must be 0, 1 or 2");
  for (int q = 0; q < 2; ++q) {
    if (s->xcd_remap[q] < 0 || s->xcd_remap[q] > 64)
      return fail(LB_EINVAL, "xcd_remap entries must be 0 (off), 1 (contiguous) or a group size 2..64");
    if (s->tiling[q] != 0 && s->tiling[q] != 1) return fail(LB_EINVAL, "tiling entries must be 0 or 1");
    if (s->tiling[q] && ctx->wide) return fail(LB_EUNSUPPORTED, "the row tiling needs planes below 4 GiB");
  }
  if (s->graph_chunk < 2 || (s->graph_chunk & 1) || s->graph_chunk > 1024)
    return fail(LB_EINVAL, "graph_chunk must be even and in [2, 1024]");
  if (s->resident != 0 && s->resident != 1) return fail(LB_EINVAL, "resident must be 0 or 1");
  if (s->resident && ctx->wide) return fail(LB_EUNSUPPORTED, "the resident cache policy needs planes below 4 GiB");
  if (s->group_mb < 0 || s->group_mb > (1 << 20)) return fail(LB_EINVAL, "group_mb must be in [0, 2^20]");
  if (s->fused != 0 && s->fused != 1) return fail(LB_EINVAL, "fused must be 0 or 1");
  if (s->fused && !fused_eligible(ctx))
    return fail(LB_EUNSUPPORTED, "the fused schedule needs a single lattice whose z-planes (D3Q19) or rows (D2Q9) stay below 4 GiB");

  HIP_TRY(hipSetDevice(ctx->device));
  if (s->fused) {
    int rc = ensure_state_b(ctx);
    if (rc) return rc;
  }
  ctx->sched = *s;
  int rc = upload_schedule(ctx);
  if (!s->fused) release_state_b(ctx);
  return rc;
}

}  // extern "C"

namespace {

// Autotune cache (LBF_TUNE_CACHE): one line per tuned workload, its key and
// the schedule fields, appended after each timed tuning; the last line with
// a matching key wins.  The key names the device (architecture and CU
// count), this build of the library, the lattice and storage, and every
// replica's box and noise flag in the order given, so a schedule is reused
// only for the workload and kernels it was timed on.
std::string tune_key(const lb_ctx* c) {
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess)
    dev = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the replica boxes and noise flags
  auto mix = [&](uint64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (v >> (8 * b)) & 0xFF;
      h *= 1099511628211ull;
    }
  };
  for (const lb_params& p : c->reps) {
    mix(((uint64_t)p.nx << 32) | (uint32_t)p.ny);
    mix(((uint64_t)p.nz << 1) | (p.kT > 0.0 ? 1u : 0u));
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s|%s %s|lattice%d|storage%d|n%zu|%dx%dx%d|%016llx", dev.c_str(), __DATE__,
                __TIME__, c->lattice, c->storage, c->reps.size(), c->reps[0].nx, c->reps[0].ny, c->reps[0].nz,
                (unsigned long long)h);
  return buf;
}

bool tune_cache_find(const char* path, const std::string& key, lb_schedule* out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    const char* tab = std::strchr(line, '\t');
    if (!tab || (size_t)(tab - line) != key.size() || std::strncmp(line, key.data(), key.size()) != 0) continue;
    lb_schedule s{};
    if (std::sscanf(tab + 1, "%d %d %d %d %d %d %d %d %d %d", &s.block, &s.order, &s.graph_chunk, &s.xcd_remap[0],
                    &s.xcd_remap[1], &s.tiling[0], &s.tiling[1], &s.resident, &s.group_mb, &s.fused) == 10) {
      *out = s;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_add(const char* path, const std::string& key, const lb_schedule& s) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;  // the tuned schedule is applied either way
  std::fprintf(f, "%s\t%d %d %d %d %d %d %d %d %d %d\n", key.c_str(), s.block, s.order, s.graph_chunk, s.xcd_remap[0],
               s.xcd_remap[1], s.tiling[0], s.tiling[1], s.resident, s.group_mb, s.fused);
  std::fclose(f);
}

int autotune_timed(lb_ctx* ctx, int32_t steps, char* report, size_t report_len);

}  // namespace

extern "C" {

int lb_autotune(lb_ctx* ctx, int32_t steps, char* report, size_t report_len) {
  if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
  if (ctx->parent) return fail(LB_EINVAL, "tune the batch, not a view");
  if (steps < 2) return fail(LB_EINVAL, "steps must be >= 2");
  HIP_TRY(hipSetDevice(ctx->device));
  const char* path = std::getenv("LBF_TUNE_CACHE");
  const bool cache = path && *path;
  const std::string key = cache ? tune_key(ctx) : std::string();
  lb_schedule s{};
  if (cache && tune_cache_find(path, key, &s)) {
    const std::string keep = g_last_error;
    if (lb_set_schedule(ctx, &s) == LB_OK) {
      if (report && report_len) {
        const std::string rep = "[{\"cached\":true,\"key\":\"" + key + "\"}]";
        std::strncpy(report, rep.c_str(), report_len - 1);
        report[report_len - 1] = 0;
      }
      return LB_OK;
    }
    g_last_error = keep;  // e.g. no room for the fused pass's buffer now: tune afresh
  }
  const int rc = autotune_timed(ctx, steps, report, report_len);
  if (rc == LB_OK && cache) tune_cache_add(path, key, ctx->sched);
  return rc;
}

}  // extern "C"

namespace {

int autotune_timed(lb_ctx* ctx, int32_t steps, char* report, size_t report_len) {
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));

  // scratch copy of the whole state and of the step counter
  size_t bytes = 0;
  for (size_t r = 0; r < ctx->reps.size(); ++r)
    bytes = std::max<size_t>(bytes, ctx->offsets[r] + ((lb_state_bytes(&ctx->reps[r]) + 255) & ~(size_t)255));
  {
    // a predictable failure is reported as such, before anything changes
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    if (free_b < bytes + (256ull << 20))
      return fail(LB_EUNSUPPORTED, "not enough free device memory for the autotuner's scratch copy of the state");
  }
  char* scratch = nullptr;
  HIP_TRY(hipMalloc(&scratch, bytes));
  const uint64_t base0 = ctx->lats[0].base - ctx->offsets[0];
  const hipError_t ce = hipMemcpyAsync(scratch, (void*)(uintptr_t)base0, bytes, hipMemcpyDeviceToDevice, ctx->stream);
  if (ce != hipSuccess) {
    (void)hipFree(scratch);
    return fail(LB_EDEVICE, std::string("hipMemcpyAsync (autotune scratch copy): ") + hipGetErrorString(ce));
  }

  const std::vector<LatDesc> saved_lats = ctx->lats;
  const lb_schedule saved = ctx->sched;
  const int64_t saved_t = ctx->t;
  for (size_t r = 0; r < ctx->lats.size(); ++r) ctx->lats[r].base = (uint64_t)(uintptr_t)scratch + ctx->offsets[r];

  struct Cand {
    int block, ord, remap, til;
    double ms[2];   // first pass: mean even / odd step time
    double ref[2];  // second pass (shortlisted candidates only), else -1
  };
  std::vector<Cand> cands;
  int rc = LB_OK;
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (auto& e : ev)
    if (rc == LB_OK && hipEventCreate(&e) != hipSuccess) rc = fail(LB_EDEVICE, "hipEventCreate");

  // Mean even and odd step time of one schedule over `steps` launches of
  // each parity, after one warm-up launch of each.
  auto time_schedule = [&](const Cand& cd, double out[2]) -> int {
    ctx->sched = lb_schedule{cd.block, cd.ord, saved.graph_chunk, {cd.remap, cd.remap}, {cd.til, cd.til}, 0, 0};
    int r = upload_schedule(ctx);
    if (r == LB_OK) r = direct_steps(ctx, 2);
    out[0] = out[1] = 0.0;
    for (int k = 0; k < 2 * steps && r == LB_OK; ++k) {
      const int parity = (int)(ctx->t & 1);
      if (hipEventRecord(ev[0], ctx->stream) != hipSuccess) return fail(LB_EDEVICE, "hipEventRecord");
      if ((r = launch_step(ctx, 0, parity))) break;
      if (hipEventRecord(ev[1], ctx->stream) != hipSuccess) return fail(LB_EDEVICE, "hipEventRecord");
      if ((r = launch_advance(ctx, 1))) break;
      ctx->t += 1;
      if (hipEventSynchronize(ev[1]) != hipSuccess) return fail(LB_EDEVICE, "hipEventSynchronize");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
      out[parity] += ms;
    }
    out[0] /= steps;
    out[1] /= steps;
    return r;
  };

  // First pass: every block size and tile order with every (remap, tiling)
  // pair, even and odd steps timed separately (the state layout does not
  // depend on the schedule, so the parities can be chosen independently).
  const int blocks[] = {64, 128, 256, 512};
  const int remaps[] = {0, 1, 2, 4, 8};
  const int norders = ctx->lats.size() > 1 ? 3 : 1;
  const int ntiling = ctx->wide ? 1 : 2;
  for (int bi = 0; bi < 4 && rc == LB_OK; ++bi)
    for (int ord = 0; ord < norders && rc == LB_OK; ++ord)
      for (int ri = 0; ri < 5 && rc == LB_OK; ++ri)
        for (int til = 0; til < ntiling && rc == LB_OK; ++til) {
          Cand cd{blocks[bi], ord, remaps[ri], til, {0.0, 0.0}, {-1.0, -1.0}};
          rc = time_schedule(cd, cd.ms);
          cands.push_back(cd);
        }

  // Second pass: a mean over `steps` launches differs by a percent or two
  // between repeats, about as much as the candidates differ, so the minimum
  // of the first pass favours lucky draws.  The fastest few per parity are
  // timed again, in several interleaved rounds, and the choice is made on
  // those times alone.
  constexpr int SHORT = 6, ROUNDS = 3;
  std::vector<size_t> shortlist;
  for (int q = 0; q < 2 && rc == LB_OK; ++q) {
    std::vector<size_t> idx(cands.size());
    for (size_t k = 0; k < idx.size(); ++k) idx[k] = k;
    const size_t m = std::min<size_t>(SHORT, idx.size());
    std::partial_sort(idx.begin(), idx.begin() + m, idx.end(),
                      [&](size_t a, size_t b) { return cands[a].ms[q] < cands[b].ms[q]; });
    for (size_t k = 0; k < m; ++k)
      if (std::find(shortlist.begin(), shortlist.end(), idx[k]) == shortlist.end()) shortlist.push_back(idx[k]);
  }
  for (size_t k : shortlist) cands[k].ref[0] = cands[k].ref[1] = 0.0;
  for (int round = 0; round < ROUNDS && rc == LB_OK; ++round)
    for (size_t k : shortlist) {
      double ms[2];
      if ((rc = time_schedule(cands[k], ms))) break;
      cands[k].ref[0] += ms[0] / ROUNDS;
      cands[k].ref[1] += ms[1] / ROUNDS;
    }

  // Best (block, order): the sum of its fastest shortlisted even and odd
  // (remap, tiling) choices.
  lb_schedule best = saved;
  double best_ms = 1e300;
  for (size_t a : shortlist) {
    const Cand& g = cands[a];
    int pick[2] = {-1, -1};
    for (size_t b : shortlist) {
      const Cand& h = cands[b];
      if (h.block != g.block || h.ord != g.ord) continue;
      for (int q = 0; q < 2; ++q)
        if (pick[q] < 0 || h.ref[q] < cands[pick[q]].ref[q]) pick[q] = (int)b;
    }
    const double tot = cands[pick[0]].ref[0] + cands[pick[1]].ref[1];
    if (tot < best_ms) {
      best_ms = tot;
      best = lb_schedule{g.block, g.ord, saved.graph_chunk, {cands[pick[0]].remap, cands[pick[1]].remap},
                         {cands[pick[0]].til, cands[pick[1]].til}, 0, 0};
    }
  }

  // Second stage: the cache policy and the replica groups of that schedule.
  // Both pay only through reuse of cached state across the steps of a graph
  // replay, so each variant is timed on whole replays (the path lb_step
  // takes): one warm-up replay, then at least 2 * steps steps, in interleaved
  // rounds.  A variant replaces the first stage's choice (streaming, one
  // group) only when it is at least 1% faster.
  struct Var {
    int res, gmb, fused;
    double ms;
  };
  std::vector<Var> vars;
  {
    const int gmbs[] = {0, 64, 128, 160, 192, 224, 256};
    const int ngmb = ctx->lats.size() > 1 ? 7 : 1;
    for (int res = 0; res < (ctx->wide ? 1 : 2); ++res)
      for (int gi = 0; gi < ngmb; ++gi) vars.push_back({res, gmbs[gi], 0, 0.0});
    // the fused two-step schedule, when its second buffer fits
    if (rc == LB_OK && fused_eligible(ctx)) {
      const std::string keep = g_last_error;
      if (ensure_state_b(ctx) == LB_OK) vars.push_back({0, 0, 1, 0.0});
      else g_last_error = keep;
    }
  }
  const int K2 = best.graph_chunk;
  const int64_t chunks = std::max<int64_t>(1, (2 * (int64_t)steps + K2 - 1) / K2);
  auto time_variant = [&](const Var& v, double& ms_out) -> int {
    ctx->sched = best;
    ctx->sched.resident = v.res;
    ctx->sched.group_mb = v.gmb;
    ctx->sched.fused = v.fused;
    int r = upload_schedule(ctx);
    if (r == LB_OK && (ctx->t & 1)) r = direct_steps(ctx, 1);
    if (r == LB_OK) r = advance(ctx, K2);  // warm-up replay (builds the graph)
    if (r != LB_OK) return r;
    if (hipEventRecord(ev[0], ctx->stream) != hipSuccess) return fail(LB_EDEVICE, "hipEventRecord");
    if ((r = advance(ctx, chunks * K2))) return r;
    if (hipEventRecord(ev[1], ctx->stream) != hipSuccess) return fail(LB_EDEVICE, "hipEventRecord");
    if (hipEventSynchronize(ev[1]) != hipSuccess) return fail(LB_EDEVICE, "hipEventSynchronize");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    ms_out = ms / (double)(chunks * K2);
    return LB_OK;
  };
  constexpr int ROUNDS2 = 3;
  for (int round = 0; round < ROUNDS2 && rc == LB_OK && vars.size() > 1; ++round)
    for (auto& v : vars) {
      double ms = 0.0;
      if ((rc = time_variant(v, ms))) break;
      v.ms += ms / ROUNDS2;
    }
  if (rc == LB_OK && vars.size() > 1) {
    const Var* pick = &vars[0];
    for (const auto& v : vars)
      if (v.ms < pick->ms && v.ms < 0.99 * vars[0].ms) pick = &v;
    best.resident = pick->res;
    best.group_mb = pick->gmb;
    best.fused = pick->fused;
  }

  std::string rep = "[";
  for (size_t k = 0; k < cands.size(); ++k) {
    const Cand& cd = cands[k];
    char buf[256];
    int n = std::snprintf(buf, sizeof(buf), "%s{\"block\":%d,\"order\":%d,\"xcd_remap\":%d,\"tiling\":%d,"
                          "\"even_ms\":%.6f,\"odd_ms\":%.6f", k ? "," : "", cd.block, cd.ord, cd.remap, cd.til,
                          cd.ms[0], cd.ms[1]);
    if (cd.ref[0] >= 0.0)
      std::snprintf(buf + n, sizeof(buf) - n, ",\"refined_even_ms\":%.6f,\"refined_odd_ms\":%.6f}", cd.ref[0],
                    cd.ref[1]);
    else
      std::snprintf(buf + n, sizeof(buf) - n, "}");
    rep += buf;
  }
  for (const auto& v : vars) {
    if (vars.size() < 2 || rc != LB_OK) break;
    char buf[160];
    std::snprintf(buf, sizeof(buf), ",{\"stage\":2,\"resident\":%d,\"group_mb\":%d,\"fused\":%d,\"ms_per_step\":%.6f}",
                  v.res, v.gmb, v.fused, v.ms);
    rep += buf;
  }
  rep += "]";
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);

  // restore the state pointers, step counter and device counter; apply the best schedule
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(scratch);
  ctx->lats = saved_lats;
  ctx->t = saved_t;
  (void)hipMemcpy(ctx->d_lats, ctx->lats.data(), sizeof(LatDesc) * ctx->lats.size(), hipMemcpyHostToDevice);
  hipLaunchKernelGGL(k_set_t, dim3(1), dim3(64), 0, ctx->stream, ctx->d_t, (uint64_t)saved_t);
  ctx->sched = (rc == LB_OK) ? best : saved;
  int rc2 = upload_schedule(ctx);
  if (!ctx->sched.fused) release_state_b(ctx);
  if (report && report_len) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return rc ? rc : rc2;
}

}  // namespace

extern "C" {

int lb_step_noalloc(const lb_params* reps, int32_t nrep, void* d_pool, void* hip_stream, int64_t t0,
                    int64_t nsteps) {
  if (!reps || nrep < 1) return fail(LB_EINVAL, "lb_step_noalloc needs at least one lattice");
  if (nrep > LB_NOALLOC_MAX_REPLICAS)
    return fail(LB_EUNSUPPORTED, "lb_step_noalloc takes at most LB_NOALLOC_MAX_REPLICAS (64) lattices: its "
                                 "device scratch holds 64 descriptors; use lb_batch_init / lb_batch_step");
  for (int r = 0; r < nrep; ++r) {
    int rc = validate(&reps[r]);
    if (rc) return rc;
    if (reps[r].storage != reps[0].storage) return fail(LB_EINVAL, "all lattices need the same storage type");
    if (reps[r].lattice != reps[0].lattice) return fail(LB_EINVAL, "all lattices need the same lattice model");
    if (nrep > 1 && is_wide(reps[r])) return fail(LB_EUNSUPPORTED, "batched lattices must hold < 4 GiB per plane");
  }
  if (!d_pool || ((uintptr_t)d_pool & 255)) return fail(LB_EINVAL, "d_pool must be non-NULL and 256-byte aligned");
  if (t0 < 0) return fail(LB_EINVAL, "t0 must be >= 0");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return LB_OK;

  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  unsigned char* base = nullptr;
  int rc = noalloc_scratch(device, &base);
  if (rc) return rc;
  LatDesc* d_lats = reinterpret_cast<LatDesc*>(base + NA_OFF_DESC);
  uint32_t* d_blk = reinterpret_cast<uint32_t*>(base + NA_OFF_BLK);
  uint32_t* d_blk_rows = reinterpret_cast<uint32_t*>(base + NA_OFF_BLKR);
  uint64_t* d_t = reinterpret_cast<uint64_t*>(base + NA_OFF_T);
  hipStream_t st = (hipStream_t)hip_stream;

  // the library's default launch shape, streaming cache policy, one launch per step
  constexpr int BLOCK = 256;
  const int storage = reps[0].storage, lattice = reps[0].lattice;
  const bool wide = is_wide(reps[0]);
  int tiling[2] = {1, 0}, remap[2] = {0, 0};
  if (storage != LB_F32) {
    tiling[0] = 0;
    tiling[1] = 1;
    if (lattice == LB_D3Q19) remap[0] = remap[1] = 8;
  }
  if (wide) tiling[0] = tiling[1] = 0;

  // descriptors, in chunks passed by value, then the tile prefixes and the step counter
  NaMeta meta{};
  uint64_t off = 0, acc = 0, acc_rows = 0;
  for (int r0 = 0; r0 < nrep; r0 += NA_CHUNK) {
    NaDescs chunk{};
    chunk.n = (uint32_t)std::min(NA_CHUNK, nrep - r0);
    for (uint32_t k = 0; k < chunk.n; ++k) {
      const lb_params& p = reps[r0 + k];
      LatDesc L = make_desc(p, (uint64_t)(uintptr_t)d_pool + off);
      L.segs = (L.nx + BLOCK - 1) / BLOCK;
      div_magic(L.segs, L.ds_m, L.ds_s1, L.ds_s2);
      meta.blk[r0 + k] = (uint32_t)acc;
      meta.blk_rows[r0 + k] = (uint32_t)acc_rows;
      acc += (L.nsites + BLOCK - 1) / BLOCK;
      acc_rows += (uint64_t)L.ny * L.nz * L.segs;
      off += (lb_state_bytes(&p) + 255) & ~(size_t)255;
      chunk.d[k] = L;
    }
    hipLaunchKernelGGL(k_noalloc_descs, dim3(1), dim3(64), 0, st, chunk, d_lats + r0);
    HIP_TRY(hipGetLastError());
  }
  if (acc >= (1ull << 31) || acc_rows >= (1ull << 31)) return fail(LB_EUNSUPPORTED, "too many workgroups for one launch");
  meta.blk[nrep] = (uint32_t)acc;
  meta.blk_rows[nrep] = (uint32_t)acc_rows;
  meta.t = (uint64_t)t0;
  meta.n = (uint32_t)nrep;
  hipLaunchKernelGGL(k_noalloc_meta, dim3(1), dim3(64), 0, st, meta, d_blk, d_blk_rows, d_t);
  HIP_TRY(hipGetLastError());

  // the steps, in runs of 16 launches between counter advances
  const uint32_t nlat = (uint32_t)nrep;
  for (int64_t s0 = 0; s0 < nsteps; s0 += 16) {
    const int64_t m = std::min<int64_t>(16, nsteps - s0);
    for (int64_t s = 0; s < m; ++s) {
      const int parity = (int)((t0 + s0 + s) & 1);
      const bool rows = tiling[parity] != 0;
      void* fn = rows ? rows_ptr(lattice, storage, parity, false, BLOCK, false)
                      : step_ptr(lattice, storage, parity, wide, false, BLOCK, false);
      const LatDesc* lats = d_lats;
      const uint32_t* blk = rows ? d_blk_rows : d_blk;
      uint32_t rm = (uint32_t)remap[parity];
      const uint64_t* dt = d_t;
      uint32_t t_off = (uint32_t)s;
      uint32_t nl = nlat;
      void* args[] = {&lats, &blk, &nl, &rm, &dt, &t_off};
      HIP_TRY(hipLaunchKernel(fn, dim3((uint32_t)(rows ? acc_rows : acc)), dim3(BLOCK), args, 0, st));
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, d_t, (uint64_t)m);
    HIP_TRY(hipGetLastError());
  }
  return LB_OK;
}

}  // extern "C"
