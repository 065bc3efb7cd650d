// lbf_kernels.h -- gfx950 kernels of the fluctuating lattice Boltzmann update
// (Duenweg, Schiller & Ladd, arXiv:0707.1581): the fused in-place
// collide-and-stream step, initial states, parity-resolved gathers and the
// health-check reduction, templated on the lattice model (D3Q19 or D2Q9,
// see lbf_math.h).
//
// One thread per lattice site; all q populations of a site are loaded
// before anything is stored, the mode transform, relaxation and noise stay in
// VGPRs, and nothing goes through LDS.  The in-place update uses the AA access
// pattern: a step at even t reads plane i at site r and writes the
// post-collision population i to plane opp(i) at r; a step at odd t reads
// plane j at r + c_j (which holds n_opp(j)(r)) and writes population j to
// plane j at r + c_j.  Each thread therefore reads and writes the same q
// locations, and no two threads touch the same location, so one buffer
// suffices and no synchronisation is needed inside a step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbf_math.h"

namespace lbf {

enum { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

// ---------------------------------------------------------------- storage
// The stored value is d_i = (n_i - a_i rho0) / (a_i rho0); 16-bit forms round
// to nearest even on store, all arithmetic is fp32.
template <int S> struct Codec;
template <> struct Codec<ST_F32> {
  using T = float;
  static __device__ __forceinline__ float dec(T v) { return v; }
  static __device__ __forceinline__ T enc(float x) { return x; }
};
template <> struct Codec<ST_F16> {
  using T = _Float16;
  static __device__ __forceinline__ float dec(T v) { return (float)v; }
  static __device__ __forceinline__ T enc(float x) { return (_Float16)x; }
};
template <> struct Codec<ST_BF16> {
  using T = uint16_t;
  static __device__ __forceinline__ float dec(T v) { return __uint_as_float((uint32_t)v << 16); }
  static __device__ __forceinline__ T enc(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
};

// ---------------------------------------------------------------- lattice descriptor
// One per lattice (a single lattice, or one replica of an ensemble); read by
// every workgroup through scalar loads.
struct alignas(16) LatDesc {
  uint64_t base;      // device address of plane 0
  uint64_t plane;     // elements per plane = nx * ny * nz
  uint32_t nsites;    // = plane (< 2^32)
  uint32_t nx, ny, nz;
  uint32_t nxy;
  uint32_t wx, wy, wz;              // nx - 1, (ny - 1) nx, (nz - 1) nx ny
  uint32_t dx_m, dx_s1, dx_s2;      // division by nx: (t + ((n - t) >> s1)) >> s2, t = mulhi(n, m)
  uint32_t dy_m, dy_s1, dy_s2;      // division by ny
  uint32_t key0, key1;              // Philox key = seed
  uint32_t thermal;                 // 1 when kT > 0
  uint32_t segs;                    // row tiling: workgroups per x-row (ceil(nx / block))
  uint32_t ds_m, ds_s1, ds_s2;      // division by segs
  float rho0;
  // per-mode coefficients, indexed from the first non-conserved mode K0 = d + 1
  // (D3Q19 uses all entries, D2Q9 the first 6, 3, 6 and 9)
  float ca[15];   // gamma_k / (36 w_k), k = K0..q-1
  float cb[6];    // (1 - gamma_k) / (36 w_k), stress modes k = K0..K0+NSTRESS-1
  float cc[15];   // sqrt(mu (1 - gamma_k^2) / (w_k rho0)), k = K0..q-1; 0 if unthermalised
  float ci[19];   // sqrt(mu / (rho0 w_k)), k = 0..q-1: thermal initial state
};
static_assert(sizeof(LatDesc) % 16 == 0, "LatDesc alignment");

__device__ __forceinline__ uint32_t fastdiv(uint32_t n, uint32_t m, uint32_t s1, uint32_t s2) {
  const uint32_t t = __umulhi(n, m);
  return (t + ((n - t) >> s1)) >> s2;
}

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror & Shaw (SC'11): ten rounds of two 32x32->64 products
// of counter words 0 and 2 with the published multipliers, feeding the high
// halves through the key and the other two words; the key advances by the
// published Weyl constants between rounds.
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0, n2;
    if (r == 0) {
      // counter words 1..3 are uniform here: plain xors stay on the scalar unit
      n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
      n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    } else {
      // three-input xor (truth table 0x96) in one gfx950 bitop3
      n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
      n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    }
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Four 24-bit uniforms from three words taken as one 96-bit big-endian number.
__device__ __forceinline__ void chunks4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t ch[4]) {
  ch[0] = w0 >> 8;
  ch[1] = ((w0 << 16) | (w1 >> 16)) & 0xFFFFFFu;
  ch[2] = ((w1 << 8) | (w2 >> 24)) & 0xFFFFFFu;
  ch[3] = w2 & 0xFFFFFFu;
}

// Box-Muller pair from chunks (a, b): u1 = (a + 1) 2^-24 in (0, 1],
// u2 = b 2^-24; returns s * sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2) with
// s = sqrt(scale2): the caller passes -2 ln(2) s^2 as k2, folding the scale
// into the log multiplier.  v_log_f32 is log2 and v_sin/v_cos take
// revolutions.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float k2, float& z0, float& z1) {
  const float u1 = __builtin_fmaf((float)a, 0x1p-24f, 0x1p-24f);
  const float u2 = (float)b * 0x1p-24f;
  const float r = __builtin_amdgcn_sqrtf(k2 * __builtin_amdgcn_logf(u1));
  z0 = r * __builtin_amdgcn_cosf(u2);
  z1 = r * __builtin_amdgcn_sinf(u2);
}
constexpr float NEG_2LN2 = -1.3862943611198906f;  // -2 ln 2: sqrt(-2 ln u) = sqrt(-2 ln2 log2 u)

// ---------------------------------------------------------------- addressing
// Element offsets o_j of site r + c_j (periodic), j = 0..q-1.
template <class M, class Off>
__device__ __forceinline__ void neighbour_offsets(const LatDesc& L, uint32_t site, Off o[M::Q]) {
  const uint32_t zy = fastdiv(site, L.dx_m, L.dx_s1, L.dx_s2);
  const uint32_t x = site - zy * L.nx;
  uint32_t z = 0, y = zy;  // a 2D lattice has nz = 1
  if constexpr (M::D == 3) {
    z = fastdiv(zy, L.dy_m, L.dy_s1, L.dy_s2);
    y = zy - z * L.ny;
  }
  // signed steps in 32-bit wrap-around arithmetic; the sums land in [0, N)
  const uint32_t xm = (x == 0) ? L.wx : 0xFFFFFFFFu;
  const uint32_t xp = (x == L.wx) ? 0u - L.wx : 1u;
  const uint32_t ym = (y == 0) ? L.wy : 0u - L.nx;
  const uint32_t yp = (y * L.nx == L.wy) ? 0u - L.wy : L.nx;
  const uint32_t zm = (z == 0) ? L.wz : 0u - L.nxy;
  const uint32_t zp = (z * L.nxy == L.wz) ? 0u - L.wz : L.nxy;
#pragma unroll
  for (int j = 0; j < M::Q; ++j) {
    uint32_t s = site;
    if (M::CY[j] > 0) s += yp;
    if (M::CY[j] < 0) s += ym;
    if (M::CZ[j] > 0) s += zp;
    if (M::CZ[j] < 0) s += zm;
    if (M::CX[j] > 0) s += xp;
    if (M::CX[j] < 0) s += xm;
    o[j] = (Off)s;
  }
}

// State access.  Lattices whose population planes are below 4 GiB use buffer
// instructions: the plane's resource descriptor lives in SGPRs (base, size in
// bytes, the gfx9 raw-buffer format word) and each lane supplies only a
// 32-bit byte offset, so no per-lane 64-bit address arithmetic is needed; the
// hardware range check also drops any access outside the plane.  Larger
// planes use global (address space 1) loads and stores with 64-bit offsets.
//
// Cache policy per storage type and step parity, chosen by measurement on
// MI355X (512^3 box): the even step reads and writes whole aligned rows once,
// so non-temporal (streaming) loads and stores bring it close to the bandwidth
// of pure data movement; the odd step's x-shifted accesses share cache lines
// between neighbouring waves, which non-temporal loads would evict early, so
// it keeps those planes cached and streams the others.  The same policy
// measured fastest for all three storage types.  The resident policy (RES)
// caches every access: it pays when the state a run of launches touches fits
// in the 256 MB Infinity Cache (a small lattice, or one group of replicas
// stepped several times before the next group), where streaming hints would
// send every step back to HBM.
#define LBF_GLOBAL __attribute__((address_space(1)))
constexpr int CPOL_NT = 2;              // cache policy bit: non-temporal
constexpr int RAW_BUFFER_WORD3 = 0x00020000;

template <class M, int S, int P, bool RES = false> struct CachePolicy {
  // plane j of the odd step is accessed at r + c_j: shifted along x iff c_jx != 0
  static constexpr bool nt_load(int j) { return !RES && (P == 0 || M::CX[j] == 0); }
  static constexpr bool nt_store(int j) { return !RES && (P == 0 || M::CX[j] == 0); }
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const LatDesc& L, int plane, uint32_t esize) {
  const uint64_t bytes = L.plane * esize;
  return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)(L.base + (uint64_t)plane * bytes), 0,
                                           (int)(uint32_t)bytes, RAW_BUFFER_WORD3);
}

template <class T> struct Raw;
// b: per-lane byte offset; so: uniform byte offset (the instruction's SGPR
// offset field).
template <> struct Raw<float> {
  template <int POL> static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t b, uint32_t so = 0) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, b, so, POL));
  }
  template <int POL> static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t b, float v, uint32_t so = 0) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, b, so, POL);
  }
};
template <> struct Raw<_Float16> {
  template <int POL> static __device__ __forceinline__ _Float16 ld(__amdgpu_buffer_rsrc_t r, uint32_t b, uint32_t so = 0) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, b, so, POL));
  }
  template <int POL> static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t b, _Float16 v, uint32_t so = 0) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, b, so, POL);
  }
};
template <> struct Raw<uint16_t> {
  template <int POL> static __device__ __forceinline__ uint16_t ld(__amdgpu_buffer_rsrc_t r, uint32_t b, uint32_t so = 0) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, b, so, POL);
  }
  template <int POL> static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t b, uint16_t v, uint32_t so = 0) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, b, so, POL);
  }
};

// Register form of a loaded value that is carried across loop iterations (the
// fused passes' prefetched planes).  16-bit values travel zero-extended in a
// 32-bit register each: an array of 16-bit values is otherwise kept as packed
// pairs, and packing a pair waits for both loads right after they are issued.
template <class T> struct Carry {
  using U = T;
  static __device__ __forceinline__ U wrap(T v) { return v; }
  static __device__ __forceinline__ T unwrap(U u) { return u; }
};
template <> struct Carry<_Float16> {
  using U = uint32_t;
  static __device__ __forceinline__ U wrap(_Float16 v) { return (uint32_t)__builtin_bit_cast(uint16_t, v); }
  static __device__ __forceinline__ _Float16 unwrap(U u) { return __builtin_bit_cast(_Float16, (uint16_t)u); }
};
template <> struct Carry<uint16_t> {
  using U = uint32_t;
  static __device__ __forceinline__ U wrap(uint16_t v) { return (uint32_t)v; }
  static __device__ __forceinline__ uint16_t unwrap(U u) { return (uint16_t)u; }
};

template <class T, int POL, class Off>
__device__ __forceinline__ T ld(const LatDesc& L, int plane, Off o) {
  if constexpr (sizeof(Off) == 4) {
    return Raw<T>::template ld<POL>(plane_rsrc(L, plane, sizeof(T)), o * (uint32_t)sizeof(T));
  } else {
    const LBF_GLOBAL T* p = (const LBF_GLOBAL T*)(uintptr_t)L.base + (uint64_t)plane * L.plane;
    if constexpr (POL == CPOL_NT) return __builtin_nontemporal_load(p + o);
    else return p[o];
  }
}
template <class T, int POL, class Off>
__device__ __forceinline__ void st(const LatDesc& L, int plane, Off o, T v) {
  if constexpr (sizeof(Off) == 4) {
    Raw<T>::template st<POL>(plane_rsrc(L, plane, sizeof(T)), o * (uint32_t)sizeof(T), v);
  } else {
    LBF_GLOBAL T* p = (LBF_GLOBAL T*)(uintptr_t)L.base + (uint64_t)plane * L.plane;
    if constexpr (POL == CPOL_NT) __builtin_nontemporal_store(v, p + o);
    else p[o] = v;
  }
}

// Policy chosen per plane; `nt` is a constant once the plane loops unroll.
// Buffer accesses only: the policy is an immediate operand of the buffer
// intrinsic, so the two branches stay distinct.  Two global accesses of the
// same address that differ only in the non-temporal hint are merged by the
// optimiser into one access without it, so the 64-bit-offset path loops with
// the plane index as a compile-time constant instead (static_for) and passes
// the policy as a template argument.
template <class T>
__device__ __forceinline__ T ld_sel(const LatDesc& L, int plane, uint32_t o, bool nt) {
  return nt ? ld<T, CPOL_NT>(L, plane, o) : ld<T, 0>(L, plane, o);
}
template <class T>
__device__ __forceinline__ void st_sel(const LatDesc& L, int plane, uint32_t o, T v, bool nt) {
  if (nt) st<T, CPOL_NT>(L, plane, o, v); else st<T, 0>(L, plane, o, v);
}

constexpr int pol(bool nt) { return nt ? CPOL_NT : 0; }
template <int N> struct Idx { static constexpr int value = N; };
template <int B, int E, int STEP = 1, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(Idx<B>{});
    static_for<B + STEP, E, STEP>(f);
  }
}

// 16-bit storage, planes below 4 GiB: the two members of an opposite pair are
// converted together (one packed conversion) and stored through global
// stores with a uniform plane address and a 32-bit lane byte offset; the
// second value leaves from the high half of the register (a d16_hi store), so
// a pair costs one conversion instruction and no shift.  Bits are the same as
// Codec<S>::enc (round to nearest even).
template <int S> struct Half2;
template <> struct Half2<ST_F16> {
  using E = _Float16;
  using V = _Float16 __attribute__((ext_vector_type(2)));
};
template <> struct Half2<ST_BF16> {
  using E = __bf16;
  using V = __bf16 __attribute__((ext_vector_type(2)));
};
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ LBF_GLOBAL char* plane_ptr(const LatDesc& L, int plane, uint32_t esize) {
  return (LBF_GLOBAL char*)(uintptr_t)(L.base + (uint64_t)plane * L.plane * esize);
}

// pa + ba <- a, pb + bb <- b, both with cache policy POL (the two members of
// an opposite pair have the same one).
template <int S, int POL>
__device__ __forceinline__ void st_pair16(LBF_GLOBAL char* pa, uint32_t ba, float a, LBF_GLOBAL char* pb,
                                          uint32_t bb, float b) {
  using H = Half2<S>;
  const typename H::V v = __builtin_convertvector((f32x2){a, b}, typename H::V);
  LBF_GLOBAL typename H::E* qa = (LBF_GLOBAL typename H::E*)(pa + ba);
  LBF_GLOBAL typename H::E* qb = (LBF_GLOBAL typename H::E*)(pb + bb);
  if constexpr (POL == CPOL_NT) {
    __builtin_nontemporal_store(v.x, qa);
    __builtin_nontemporal_store(v.y, qb);
  } else {
    *qa = v.x;
    *qb = v.y;
  }
}

// Load the q populations (as d_i) of site r of the state at parity P.
template <class M, int S, int P, bool RES = false, class Off>
__device__ __forceinline__ void load_site(const LatDesc& L, uint32_t site, float d[M::Q], Off o[M::Q]) {
  using C = Codec<S>;
  using CP = CachePolicy<M, S, P, RES>;
  using T = typename C::T;
  if (P == 0) {
#pragma unroll
    for (int j = 0; j < M::Q; ++j) o[j] = (Off)site;
  } else {
    neighbour_offsets<M>(L, site, o);
  }
  // at the odd step plane j at r + c_j holds population opp(j) of site r
  if constexpr (sizeof(Off) == 4) {
#pragma unroll
    for (int j = 0; j < M::Q; ++j) d[P == 0 ? j : M::OPP[j]] = C::dec(ld_sel<T>(L, j, o[j], CP::nt_load(j)));
  } else {
    static_for<0, M::Q>([&](auto J) {
      constexpr int j = decltype(J)::value;
      d[P == 0 ? j : M::OPP[j]] = C::dec(ld<T, pol(CP::nt_load(j))>(L, j, o[j]));
    });
  }
}

// ---------------------------------------------------------------- collision
// Post-collision d*_i of one site from its pre-collision d_i, in place:
// forward transform, equilibrium stress modes (the model's stress_eq),
// relaxation m* = m^eq + gamma_k (m - m^eq) of every non-conserved mode and,
// when kT > 0, noise sqrt(mu rho w_k (1 - gamma_k^2)) r_k (Sec. IV), then the
// back-transform.  Noise: the q - d - 1 non-conserved modes take, in table
// order, the unit normals of stream 0 of (seed, site, t) (Philox words ->
// 24-bit chunks -> Box-Muller pairs).
template <class M>
__device__ __forceinline__ void collide(const LatDesc& L, float d[M::Q], uint32_t site, uint32_t tlo,
                                        uint32_t thi) {
  constexpr int Q = M::Q, K0 = M::D + 1, NS = M::NSTRESS;
  float mu[Q];
  M::forward(d, mu);

  const float R = 36.0f + mu[0];
  const float iR = __builtin_amdgcn_rcpf(R);
  float eq[NS];
  M::stress_eq(mu, iR, eq);

  float nu[Q];
  nu[0] = mu[0] * (1.0f / 36.0f);
#pragma unroll
  for (int k = 1; k < K0; ++k) nu[k] = mu[k] * (1.0f / 12.0f);
  if (L.thermal) {
    constexpr int NP = (Q - K0 + 1) / 2;    // Box-Muller pairs
    constexpr int NT = (2 * NP + 3) / 4;    // word triples, four chunks each
    constexpr int NC = (3 * NT + 3) / 4;    // Philox calls
    // every noise amplitude scales with sqrt(rho / rho0) = sqrt(R / 36)
    const float k2 = (NEG_2LN2 / 36.0f) * R;
    uint32_t w[4 * NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) philox10(site, tlo, (uint32_t)c, thi, L.key0, L.key1, w + 4 * c);
    uint32_t ch[4 * NT];
#pragma unroll
    for (int g = 0; g < NT; ++g) chunks4(w[3 * g], w[3 * g + 1], w[3 * g + 2], ch + 4 * g);
    float z[2 * NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) box_muller(ch[2 * p], ch[2 * p + 1], k2, z[2 * p], z[2 * p + 1]);
#pragma unroll
    for (int k = K0; k < K0 + NS; ++k)
      nu[k] = __builtin_fmaf(L.ca[k - K0], mu[k], __builtin_fmaf(L.cb[k - K0], eq[k - K0], L.cc[k - K0] * z[k - K0]));
#pragma unroll
    for (int k = K0 + NS; k < Q; ++k) nu[k] = __builtin_fmaf(L.ca[k - K0], mu[k], L.cc[k - K0] * z[k - K0]);
  } else {
#pragma unroll
    for (int k = K0; k < K0 + NS; ++k) nu[k] = __builtin_fmaf(L.ca[k - K0], mu[k], L.cb[k - K0] * eq[k - K0]);
#pragma unroll
    for (int k = K0 + NS; k < Q; ++k) nu[k] = L.ca[k - K0] * mu[k];
  }

  M::back(nu, d);
}

// ---------------------------------------------------------------- tile lookup
// Blocks are dealt to the eight XCDs round-robin (block i runs on XCD i % 8),
// and each XCD has its own L2.  The remap decides which logical tile block i
// takes: mode 0 keeps tile i (consecutive tiles on different XCDs); mode 1
// gives each XCD one contiguous eighth of the tiles; mode g >= 2 gives each
// XCD g consecutive tiles at a time, so tiles that share cache lines (the two
// halves of an x-row, say) share an L2 while the XCDs still walk the lattice
// together.  Every mode is a bijection on [0, G).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t i, uint32_t G, uint32_t mode) {
  if (mode == 0) return i;
  if (mode == 1) {
    const uint32_t q = G >> 3, r = G & 7u, x = i & 7u, k = i >> 3;
    return x * q + (x < r ? x : r) + k;
  }
  const uint32_t S = 8u * mode;                 // one super-group: g tiles on each XCD
  const uint32_t full = (G / S) * S;
  if (i >= full) return i;                      // ragged tail keeps its order
  const uint32_t base = i - i % S, r = i % S;
  return base + (r & 7u) * mode + (r >> 3);
}

// Lattice of logical block b: blk[l] <= b < blk[l + 1] (uniform search).
__device__ __forceinline__ uint32_t find_lattice(const uint32_t* __restrict__ blk, uint32_t nlat, uint32_t b) {
  uint32_t lo = 0, hi = nlat;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (blk[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- step kernel
// One fused collide-and-stream step at step count t = *d_t + t_off with
// parity P = t & 1, for every site of every lattice in lats[0..nlat), with
// the streaming or (RES) the resident cache policy.
template <class M, int S, int P, bool WIDE, int BLOCK, bool RES>
__global__ void __launch_bounds__(BLOCK)
k_step(const LatDesc* __restrict__ lats, const uint32_t* __restrict__ blk, uint32_t nlat,
       uint32_t remap, const uint64_t* __restrict__ d_t, uint32_t t_off) {
  using Off = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  using C = Codec<S>;
  constexpr int Q = M::Q;
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x, remap);
  uint32_t l = 0;
  if (nlat > 1) l = find_lattice(blk, nlat, b);
  const LatDesc& L = lats[l];
  const uint32_t b0 = (nlat > 1) ? blk[l] : 0u;
  const uint32_t site = (b - b0) * BLOCK + threadIdx.x;
  if (site >= L.nsites) return;
  const uint64_t t = *d_t + t_off;

  float d[Q];
  Off o[Q];
  load_site<M, S, P, RES>(L, site, d, o);
  collide<M>(L, d, site, (uint32_t)t, (uint32_t)(t >> 32));
  using CP = CachePolicy<M, S, P, RES>;
  using T = typename C::T;
  if constexpr (S != ST_F32 && !WIDE && P == 1) {
    // rest population alone, then the opposite pairs (i, i + 1), i odd, packed;
    // population j goes to plane j at r + c_j.  (At the even step, where every
    // store of the site has the same offset, plain buffer stores measure a
    // little faster.)
    st<T, pol(CP::nt_store(0))>(L, 0, o[0], C::enc(d[0]));
    static_for<1, Q, 2>([&](auto I) {
      constexpr int i = decltype(I)::value;
      static_assert(CP::nt_store(i) == CP::nt_store(i + 1), "pair members share a policy");
      st_pair16<S, pol(CP::nt_store(i))>(plane_ptr(L, i, 2), (uint32_t)o[i] * 2u, d[i], plane_ptr(L, i + 1, 2),
                                         (uint32_t)o[i + 1] * 2u, d[i + 1]);
    });
  } else if constexpr (!WIDE) {
    // population i goes to plane opp(i) at r (even) or to plane i at r + c_i (odd)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      constexpr bool even = P == 0;
      const int plane = even ? M::OPP[i] : i;
      st_sel(L, plane, o[i], C::enc(d[i]), CP::nt_store(plane));
    }
  } else {
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int plane = P == 0 ? M::OPP[i] : i;
      st<T, pol(CP::nt_store(plane))>(L, plane, o[i], C::enc(d[i]));
    });
  }
}

// ---------------------------------------------------------------- step kernel, row tiling
// The same update with a different work split: each workgroup covers one
// segment of BLOCK consecutive sites of one x-row (L.segs segments per row).
// Then y, z, the periodic y/z neighbour rows and every plane's row offset are
// uniform across the workgroup and live in SGPRs (they enter the buffer
// instruction as its scalar offset); each lane only computes x and its two
// periodic x-neighbours.  Lanes past the end of the row stay idle, so this
// suits rows of at least a few workgroups' worth of sites.
template <class M, int S, int P, int BLOCK, bool RES>
__global__ void __launch_bounds__(BLOCK)
k_step_rows(const LatDesc* __restrict__ lats, const uint32_t* __restrict__ blk, uint32_t nlat,
            uint32_t remap, const uint64_t* __restrict__ d_t, uint32_t t_off) {
  using C = Codec<S>;
  using T = typename C::T;
  using CP = CachePolicy<M, S, P, RES>;
  constexpr int EP = pol(CP::nt_load(0));  // the even step's one policy for every plane
  constexpr int Q = M::Q;
  constexpr uint32_t ES = sizeof(T);
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x, remap);
  uint32_t l = 0;
  if (nlat > 1) l = find_lattice(blk, nlat, b);
  const LatDesc& L = lats[l];
  const uint32_t bl = b - ((nlat > 1) ? blk[l] : 0u);
  // uniform: row (y + ny z) and segment of this workgroup
  const uint32_t row = fastdiv(bl, L.ds_m, L.ds_s1, L.ds_s2);
  const uint32_t x = (bl - row * L.segs) * BLOCK + threadIdx.x;
  if (x >= L.nx) return;
  uint32_t z = 0, y = row;  // a 2D lattice has nz = 1
  if constexpr (M::D == 3) {
    z = fastdiv(row, L.dy_m, L.dy_s1, L.dy_s2);
    y = row - z * L.ny;
  }
  const uint64_t t = *d_t + t_off;
  const uint32_t site = x + row * L.nx;

  // uniform row offsets (elements) of the y/z neighbours, periodic
  const uint32_t r0 = row * L.nx;
  const uint32_t ym = (y == 0) ? L.wy : 0u - L.nx;
  const uint32_t yp = (y * L.nx == L.wy) ? 0u - L.wy : L.nx;
  const uint32_t zm = (z == 0) ? L.wz : 0u - L.nxy;
  const uint32_t zp = (z * L.nxy == L.wz) ? 0u - L.wz : L.nxy;
  // per-lane x offsets in bytes: x - 1, x, x + 1 (periodic)
  const uint32_t bx = x * ES;
  const uint32_t bxm = (x == 0 ? L.wx : x - 1u) * ES;
  const uint32_t bxp = (x == L.wx ? 0u : x + 1u) * ES;

  float d[Q];
  if (P == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      d[i] = C::dec(Raw<T>::template ld<EP>(plane_rsrc(L, i, ES), bx, r0 * ES));
  } else {
    // plane j at r + c_j holds population opp(j) of site r
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      uint32_t ro = r0;
      if (M::CY[j] > 0) ro += yp;
      if (M::CY[j] < 0) ro += ym;
      if (M::CZ[j] > 0) ro += zp;
      if (M::CZ[j] < 0) ro += zm;
      const uint32_t vx = M::CX[j] > 0 ? bxp : (M::CX[j] < 0 ? bxm : bx);
      const T v = CP::nt_load(j) ? Raw<T>::template ld<CPOL_NT>(plane_rsrc(L, j, ES), vx, ro * ES)
                                 : Raw<T>::template ld<0>(plane_rsrc(L, j, ES), vx, ro * ES);
      d[M::OPP[j]] = C::dec(v);
    }
  }
  collide<M>(L, d, site, (uint32_t)t, (uint32_t)(t >> 32));
  // uniform row offset (elements) and lane byte offset of plane j at r + c_j
  auto row_of = [&](int j) {
    uint32_t ro = r0;
    if (M::CY[j] > 0) ro += yp;
    if (M::CY[j] < 0) ro += ym;
    if (M::CZ[j] > 0) ro += zp;
    if (M::CZ[j] < 0) ro += zm;
    return ro;
  };
  auto lane_of = [&](int j) { return M::CX[j] > 0 ? bxp : (M::CX[j] < 0 ? bxm : bx); };
  if constexpr (S != ST_F32) {
    // rest population alone, then the opposite pairs (i, i + 1), i odd, packed
    if (P == 0) {
      Raw<T>::template st<EP>(plane_rsrc(L, 0, ES), bx, C::enc(d[0]), r0 * ES);
#pragma unroll
      for (int i = 1; i < Q; i += 2)
        st_pair16<S, EP>(plane_ptr(L, i + 1, ES) + r0 * ES, bx, d[i], plane_ptr(L, i, ES) + r0 * ES, bx, d[i + 1]);
    } else {
      Raw<T>::template st<pol(CP::nt_store(0))>(plane_rsrc(L, 0, ES), bx, C::enc(d[0]), r0 * ES);
      static_for<1, Q, 2>([&](auto I) {
        constexpr int i = decltype(I)::value;
        static_assert(CP::nt_store(i) == CP::nt_store(i + 1), "pair members share a policy");
        st_pair16<S, pol(CP::nt_store(i))>(plane_ptr(L, i, ES) + row_of(i) * ES, lane_of(i), d[i],
                                           plane_ptr(L, i + 1, ES) + row_of(i + 1) * ES, lane_of(i + 1), d[i + 1]);
      });
    }
  } else if (P == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      Raw<T>::template st<EP>(plane_rsrc(L, M::OPP[i], ES), bx, C::enc(d[i]), r0 * ES);
  } else {
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const uint32_t ro = row_of(j), vx = lane_of(j);
      if (CP::nt_store(j)) Raw<T>::template st<CPOL_NT>(plane_rsrc(L, j, ES), vx, C::enc(d[j]), ro * ES);
      else Raw<T>::template st<0>(plane_rsrc(L, j, ES), vx, C::enc(d[j]), ro * ES);
    }
  }
}

// ---------------------------------------------------------------- propagation only
// One AA step with the identity collision: every population moves from r to
// r + c_i (periodic) and nothing else happens.  The stored values move
// unchanged, without decoding, so the result is an exact permutation of the
// state.  k_propagate and k_propagate_rows take the tiles, accesses and cache
// policy of k_step and k_step_rows, so their duration is the data-movement
// floor of the step of the same schedule.  (Their set-up code repeats that of
// the step kernels on purpose: routing both through one shared device
// function changed the step kernels' register allocation, with SGPR spills.)
template <class M, int S, int P, bool WIDE, int BLOCK, bool RES>
__global__ void __launch_bounds__(BLOCK)
k_propagate(const LatDesc* __restrict__ lats, const uint32_t* __restrict__ blk, uint32_t nlat,
            uint32_t remap, const uint64_t* __restrict__ d_t, uint32_t t_off) {
  using Off = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  using T = typename Codec<S>::T;
  using CP = CachePolicy<M, S, P, RES>;
  constexpr int Q = M::Q;
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x, remap);
  uint32_t l = 0;
  if (nlat > 1) l = find_lattice(blk, nlat, b);
  const LatDesc& L = lats[l];
  const uint32_t b0 = (nlat > 1) ? blk[l] : 0u;
  const uint32_t site = (b - b0) * BLOCK + threadIdx.x;
  if (site >= L.nsites) return;
  Off o[Q];
  T h[Q];
  if (P == 0) {
#pragma unroll
    for (int j = 0; j < Q; ++j) o[j] = (Off)site;
  } else {
    neighbour_offsets<M>(L, site, o);
  }
  // even: population i of r is plane i at r and goes to plane opp(i) at r;
  // odd: plane j at r + c_j holds population opp(j) of r, and population j
  // of r goes to plane j at r + c_j
  static_for<0, Q>([&](auto J) {
    constexpr int j = decltype(J)::value;
    h[P == 0 ? j : M::OPP[j]] = ld<T, pol(CP::nt_load(j))>(L, j, o[j]);
  });
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int plane = P == 0 ? M::OPP[i] : i;
    st<T, pol(CP::nt_store(plane))>(L, plane, o[i], h[i]);
  });
}

template <class M, int S, int P, int BLOCK, bool RES>
__global__ void __launch_bounds__(BLOCK)
k_propagate_rows(const LatDesc* __restrict__ lats, const uint32_t* __restrict__ blk, uint32_t nlat,
                 uint32_t remap, const uint64_t* __restrict__ d_t, uint32_t t_off) {
  using T = typename Codec<S>::T;
  using CP = CachePolicy<M, S, P, RES>;
  constexpr int EP = pol(CP::nt_load(0));  // the even step's one policy for every plane
  constexpr int Q = M::Q;
  constexpr uint32_t ES = sizeof(T);
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x, remap);
  uint32_t l = 0;
  if (nlat > 1) l = find_lattice(blk, nlat, b);
  const LatDesc& L = lats[l];
  const uint32_t bl = b - ((nlat > 1) ? blk[l] : 0u);
  const uint32_t row = fastdiv(bl, L.ds_m, L.ds_s1, L.ds_s2);
  const uint32_t x = (bl - row * L.segs) * BLOCK + threadIdx.x;
  if (x >= L.nx) return;
  uint32_t z = 0, y = row;
  if constexpr (M::D == 3) {
    z = fastdiv(row, L.dy_m, L.dy_s1, L.dy_s2);
    y = row - z * L.ny;
  }
  const uint32_t r0 = row * L.nx;
  const uint32_t bx = x * ES;
  T h[Q];
  if (P == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = Raw<T>::template ld<EP>(plane_rsrc(L, i, ES), bx, r0 * ES);
#pragma unroll
    for (int i = 0; i < Q; ++i) Raw<T>::template st<EP>(plane_rsrc(L, M::OPP[i], ES), bx, h[i], r0 * ES);
    return;
  }
  const uint32_t ym = (y == 0) ? L.wy : 0u - L.nx;
  const uint32_t yp = (y * L.nx == L.wy) ? 0u - L.wy : L.nx;
  const uint32_t zm = (z == 0) ? L.wz : 0u - L.nxy;
  const uint32_t zp = (z * L.nxy == L.wz) ? 0u - L.wz : L.nxy;
  const uint32_t bxm = (x == 0 ? L.wx : x - 1u) * ES;
  const uint32_t bxp = (x == L.wx ? 0u : x + 1u) * ES;
  uint32_t ro[Q], vx[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    ro[j] = r0;
    if (M::CY[j] > 0) ro[j] += yp;
    if (M::CY[j] < 0) ro[j] += ym;
    if (M::CZ[j] > 0) ro[j] += zp;
    if (M::CZ[j] < 0) ro[j] += zm;
    vx[j] = M::CX[j] > 0 ? bxp : (M::CX[j] < 0 ? bxm : bx);
    h[M::OPP[j]] = CP::nt_load(j) ? Raw<T>::template ld<CPOL_NT>(plane_rsrc(L, j, ES), vx[j], ro[j] * ES)
                                  : Raw<T>::template ld<0>(plane_rsrc(L, j, ES), vx[j], ro[j] * ES);
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (CP::nt_store(j)) Raw<T>::template st<CPOL_NT>(plane_rsrc(L, j, ES), vx[j], h[j], ro[j] * ES);
    else Raw<T>::template st<0>(plane_rsrc(L, j, ES), vx[j], h[j], ro[j] * ES);
  }
}

// ---------------------------------------------------------------- two fused steps
// k_step2 advances a D3Q19 lattice by two steps, t and t + 1 (t even), in one
// pass over HBM: it reads the state in the even AA layout (plane i at site r
// holds n_i(r)) from one buffer and writes the state at t + 2, in the same
// layout, to a second buffer.  Each population of the lattice is read once
// (plus a one-site halo) and written once per two steps instead of twice.
//
// Work split.  A workgroup owns a 64 x F2_TY column of x-y sites and walks a
// chunk of zlen planes along z.  Its waves 0..F2_TY-1 hold one x-row each;
// two more waves hold the halo rows y0 - 1 and y0 + F2_TY, and one the halo
// columns x0 - 1 and x0 + 64 (periodic).  For each plane the first step is
// collided on the tile and its halo, and every post-collision population
// that lands inside the tile is pushed into an LDS ring that accumulates the
// pre-collision populations of the second step: the c_z = -1 populations of
// plane u belong to plane u - 1, c_z = 0 to u, c_z = +1 to u + 1.  The second
// step of plane u - 2 is then collided from the ring (its last populations
// arrived one plane earlier) and pushed along c_j into the destination
// buffer.  Both steps of one plane share a phase, with one barrier per plane;
// the ring keeps flat populations for 3 planes, up-going for 4 and
// down-going for 2 (57 planes of 64 x F2_TY values).  The loads of the next
// plane but one are in flight while a plane is processed.
//
// The two steps compute exactly what two k_step launches compute (same
// collision code, same noise keys, 16-bit values rounded into the ring as
// they would be stored), so the result is bit-identical to the AA pair.
// WIDE (planes of 4 GiB or more): every access goes through the descriptor
// of one z-plane of one population plane, so no 64-bit offsets are needed;
// smaller planes take one descriptor per plane.  PROP: the identity
// collision (the data-movement floor of the pass).
constexpr int F2_TY = 10;                     // interior rows per tile
constexpr int F2_THREADS = (F2_TY + 3) * 64;  // interior + two halo-row + one halo-column waves

template <class M> struct ZClass {
  // index of population i among the populations with its c_z
  static constexpr int idx(int i) {
    int n = 0;
    for (int j = 0; j < i; ++j) n += (M::CZ[j] == M::CZ[i]) ? 1 : 0;
    return n;
  }
};

struct F2Ring {
  static constexpr int TP = 64 * F2_TY;          // interior sites of a tile
  static constexpr int NF = 9, NU = 5, ND = 5;   // D3Q19 populations with c_z = 0, +1, -1
  static constexpr int SF = 3, SU = 4, SD = 2;   // ring slots (planes in flight) per class
  static constexpr int BASE_U = SF * NF * TP;
  static constexpr int BASE_D = BASE_U + SU * NU * TP;
  static constexpr int TOTAL = BASE_D + SD * ND * TP;
  // element offset of population i's plane in the slots (fs, us, ds)
  static __device__ __forceinline__ uint32_t base(int i, uint32_t fs, uint32_t us, uint32_t ds) {
    const int c = D3Q19::CZ[i];
    const uint32_t k = (uint32_t)ZClass<D3Q19>::idx(i) * TP;
    if (c == 0) return fs * (NF * TP) + k;
    if (c > 0) return BASE_U + us * (NU * TP) + k;
    return BASE_D + ds * (ND * TP) + k;
  }
};

// Descriptor of population plane `plane` of the state at base (planes of
// plane_elems elements, below 4 GiB).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc_base(uint64_t base, uint64_t plane_elems, int plane,
                                                                  uint32_t esize) {
  const uint64_t bytes = plane_elems * esize;
  return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)(base + (uint64_t)plane * bytes), 0,
                                           (int)(uint32_t)bytes, RAW_BUFFER_WORD3);
}

// Descriptor of one slice of a population plane (a z-plane of a D3Q19 plane,
// a row of a D2Q9 plane) of slice_elems elements: slice `slice` of plane
// `plane` of the state at base.  Addressed slice by slice, a plane may
// exceed the 32-bit range of one descriptor; only the slice must stay below
// 4 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slice_rsrc(uint64_t base, uint64_t plane_elems, int plane,
                                                             uint32_t slice, uint32_t slice_elems, uint32_t esize) {
  const uint64_t off = ((uint64_t)plane * plane_elems + (uint64_t)slice * slice_elems) * esize;
  return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)(base + off), 0, (int)(slice_elems * esize),
                                           RAW_BUFFER_WORD3);
}

template <int S, bool PROP, bool WIDE>
__global__ void __launch_bounds__(F2_THREADS)
k_step2(const LatDesc* __restrict__ src, uint64_t dst_base, const uint64_t* __restrict__ d_t, uint32_t t_off,
        uint32_t ntx, uint32_t nty, uint32_t zlen) {
  using M = D3Q19;
  using C = Codec<S>;
  using T = typename C::T;
  using U = typename Carry<T>::U;  // register form of the prefetched values
  using R = F2Ring;
  constexpr int Q = M::Q;
  constexpr uint32_t ES = sizeof(T);
  __shared__ T ring[R::TOTAL];
  const LatDesc& L = *src;

  // tile: each XCD takes one contiguous eighth of the tiles (x fastest, then
  // y, then z chunk), so the tiles sharing halo lines run on one L2
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x, 1);
  const uint32_t txi = b % ntx, rest = b / ntx;
  const uint32_t tyi = rest % nty, tzi = rest / nty;
  const uint32_t nx = L.nx, ny = L.ny, nz = L.nz, nxy = L.nxy;
  const uint32_t x0 = txi * 64u, y0 = tyi * (uint32_t)F2_TY, z0 = tzi * zlen;
  const uint32_t TW = min(64u, nx - x0), TH = min((uint32_t)F2_TY, ny - y0), ZC = min(zlen, nz - z0);
  const uint32_t NIT = ZC + 3u;  // phase it: first step of plane z0 + it - 1, second of z0 + it - 3
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
  const uint64_t t = *d_t + t_off;

  // first-step site of this lane, in tile coordinates sx in [-1, TW], sy in [-1, TH]
  int sx, sy;
  bool act1;
  if (w < (uint32_t)F2_TY) {
    sx = (int)lane; sy = (int)w; act1 = lane < TW && w < TH;
  } else if (w == (uint32_t)F2_TY) {
    sx = (int)lane; sy = -1; act1 = lane < TW;
  } else if (w == (uint32_t)F2_TY + 1u) {
    sx = (int)lane; sy = (int)TH; act1 = lane < TW;
  } else {
    const uint32_t h = lane & 31u;
    sx = lane < 32u ? -1 : (int)TW; sy = (int)h - 1; act1 = h < TH + 2u;
  }
  const int gx = (int)x0 + sx, gy = (int)y0 + sy;
  const uint32_t x1 = gx < 0 ? nx - 1u : ((uint32_t)gx >= nx ? 0u : (uint32_t)gx);
  const uint32_t y1 = gy < 0 ? ny - 1u : ((uint32_t)gy >= ny ? 0u : (uint32_t)gy);
  const uint32_t sxy = x1 + nx * y1;
  const int s1idx = sy * 64 + sx;  // ring index of the first-step site (when inside the tile)

  // second-step site of this lane (interior waves); periodic neighbour offsets
  const bool act2 = w < TH && lane < TW;
  const uint32_t x2 = x0 + lane, y2 = y0 + w;
  const uint32_t bx = x2 * ES;
  const uint32_t bxm = (x2 == 0 ? nx - 1u : x2 - 1u) * ES;
  const uint32_t bxp = (x2 + 1u >= nx ? 0u : x2 + 1u) * ES;
  const uint32_t ry = y2 * nx;
  const uint32_t rym = (y2 == 0 ? ny - 1u : y2 - 1u) * nx;
  const uint32_t ryp = (y2 + 1u >= ny ? 0u : y2 + 1u) * nx;
  const uint32_t lidx = w * 64u + lane;

  auto zfirst = [&](uint32_t it) {  // lattice z of the first-step plane of phase it
    const int zz = (int)z0 + (int)it - 1;
    return zz < 0 ? nz - 1u : ((uint32_t)zz >= nz ? 0u : (uint32_t)zz);
  };
  auto load_plane = [&](uint32_t it, U (&v)[Q]) {
    if constexpr (WIDE) {  // one descriptor per z-plane of each population plane
      const uint32_t zf = zfirst(it);
#pragma unroll
      for (int i = 0; i < Q; ++i)
        v[i] = Carry<T>::wrap(Raw<T>::template ld<0>(slice_rsrc(L.base, L.plane, i, zf, nxy, ES), sxy * ES, 0u));
    } else {  // one descriptor per population plane, the z-plane in the uniform offset
      const uint32_t so = zfirst(it) * nxy * ES;
#pragma unroll
      for (int i = 0; i < Q; ++i) v[i] = Carry<T>::wrap(Raw<T>::template ld<0>(plane_rsrc(L, i, ES), sxy * ES, so));
    }
  };
  // first step of plane u = it - 1: collide, push into P(u - 1), P(u), P(u + 1)
  auto first = [&](uint32_t it, const U (&v)[Q]) {
    if (!act1 || it > ZC + 1u) return;
    float d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = C::dec(Carry<T>::unwrap(v[i]));
    if constexpr (!PROP) collide<M>(L, d, sxy + zfirst(it) * nxy, (uint32_t)t, (uint32_t)(t >> 32));
    const uint32_t fs = (it + 2u) % 3u, us = it % 4u, ds = it & 1u;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int tx = sx + M::CX[i], ty = sy + M::CY[i];
      if (tx >= 0 && tx < (int)TW && ty >= 0 && ty < (int)TH)
        ring[R::base(i, fs, us, ds) + (uint32_t)(s1idx + M::CY[i] * 64 + M::CX[i])] = PROP ? Carry<T>::unwrap(v[i]) : C::enc(d[i]);
    }
  };
  // second step of plane z0 + it - 3 from P(it - 3), pushed into the destination
  auto second = [&](uint32_t it) {
    if (it < 3u || !act2) return;
    const uint32_t z = z0 + it - 3u;
    const uint32_t fs = it % 3u, us = (it + 1u) % 4u, ds = (it + 1u) & 1u;
    T h[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = ring[R::base(i, fs, us, ds) + lidx];
    float d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = C::dec(h[i]);
    if constexpr (!PROP) {
      const uint64_t t1 = t + 1u;
      collide<M>(L, d, x2 + ry + z * nxy, (uint32_t)t1, (uint32_t)(t1 >> 32));
    }
    if constexpr (WIDE) {  // one descriptor per z-plane of each population plane
      const uint32_t zm = z == 0 ? nz - 1u : z - 1u;
      const uint32_t zp = z + 1u >= nz ? 0u : z + 1u;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const uint32_t zs = M::CZ[j] > 0 ? zp : (M::CZ[j] < 0 ? zm : z);
        const uint32_t ro = M::CY[j] > 0 ? ryp : (M::CY[j] < 0 ? rym : ry);
        const uint32_t vx = M::CX[j] > 0 ? bxp : (M::CX[j] < 0 ? bxm : bx);
        const T v = PROP ? h[j] : C::enc(d[j]);
        const __amdgpu_buffer_rsrc_t r = slice_rsrc(dst_base, L.plane, j, zs, nxy, ES);
        // x-shifted planes share lines with the neighbouring tiles: cached; the others stream
        if (M::CX[j] != 0) Raw<T>::template st<0>(r, vx, v, ro * ES);
        else Raw<T>::template st<CPOL_NT>(r, vx, v, ro * ES);
      }
    } else {  // one descriptor per population plane, the z-plane in the uniform offset
      const uint32_t rz = z * nxy;
      const uint32_t rzm = (z == 0 ? nz - 1u : z - 1u) * nxy;
      const uint32_t rzp = (z + 1u >= nz ? 0u : z + 1u) * nxy;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const uint32_t ro = (M::CY[j] > 0 ? ryp : (M::CY[j] < 0 ? rym : ry)) +
                            (M::CZ[j] > 0 ? rzp : (M::CZ[j] < 0 ? rzm : rz));
        const uint32_t vx = M::CX[j] > 0 ? bxp : (M::CX[j] < 0 ? bxm : bx);
        const T v = PROP ? h[j] : C::enc(d[j]);
        // x-shifted planes share lines with the neighbouring tiles: cached; the others stream
        if (M::CX[j] != 0) Raw<T>::template st<0>(plane_rsrc_base(dst_base, L.plane, j, ES), vx, v, ro * ES);
        else Raw<T>::template st<CPOL_NT>(plane_rsrc_base(dst_base, L.plane, j, ES), vx, v, ro * ES);
      }
    }
  };

  // two planes of loads in flight (register sets a and c, unrolled by two so
  // that both stay in registers); the first and second steps of a phase touch
  // different ring slots, so one barrier per phase suffices
  U a[Q], c[Q];
  if (act1) {
    load_plane(0u, a);
    load_plane(1u, c);
  }
  for (uint32_t it = 0; it < NIT; it += 2u) {
    first(it, a);
    if (act1 && it + 2u <= ZC + 1u) load_plane(it + 2u, a);
    second(it);
    __syncthreads();
    if (it + 1u >= NIT) break;
    first(it + 1u, c);
    if (act1 && it + 3u <= ZC + 1u) load_plane(it + 3u, c);
    second(it + 1u);
    __syncthreads();
  }
}

// Advance the device step counter after a run of step kernels.
__global__ void k_advance(uint64_t* d_t, uint64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d_t += n;
}
__global__ void k_set_t(uint64_t* d_t, uint64_t t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d_t = t;
}

// ---------------------------------------------------------------- initial states
// Store the q d_i of site r as the state at parity P.
template <class M, int S, int P, class Off>
__device__ __forceinline__ void store_site(const LatDesc& L, uint32_t site, const float d[M::Q]) {
  using C = Codec<S>;
  if (P == 0) {
#pragma unroll
    for (int i = 0; i < M::Q; ++i) st<typename C::T, 0>(L, i, (Off)site, C::enc(d[i]));
  } else {
    Off o[M::Q];
    neighbour_offsets<M>(L, site, o);
#pragma unroll
    for (int j = 0; j < M::Q; ++j) st<typename C::T, 0>(L, j, o[j], C::enc(d[M::OPP[j]]));
  }
}

// KIND 0: rest; KIND 1: thermal (stream 1, normal k -> mode k);
// KIND 2: n_i^eq(rho, u) from fields (1 + d, nz, ny, nx) = rho, ux, uy[, uz].
// The kind is a template parameter, so every init kernel is straight-line
// code: with 64-bit offsets, a run-time branch over the kinds merging into
// one shared store sequence compiled to stores whose offset register the
// fields branch never wrote.
template <class M, int S, int P, bool WIDE, int KIND>
__global__ void __launch_bounds__(256)
k_init(const LatDesc* __restrict__ Lp, const float* __restrict__ fields) {
  using Off = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  constexpr int Q = M::Q;
  const LatDesc& L = *Lp;
  const uint32_t site = blockIdx.x * 256u + threadIdx.x;
  if (site >= L.nsites) return;
  float d[Q];
  if constexpr (KIND == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = 0.0f;
  } else if constexpr (KIND == 1) {
    constexpr int NP = (Q + 1) / 2;         // Box-Muller pairs
    constexpr int NT = (2 * NP + 3) / 4;    // word triples
    constexpr int NC = (3 * NT + 3) / 4;    // Philox calls
    uint32_t w[4 * NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) philox10(site, 0u, (1u << 16) | (uint32_t)c, 0u, L.key0, L.key1, w + 4 * c);
    uint32_t ch[4 * NT];
#pragma unroll
    for (int g = 0; g < NT; ++g) chunks4(w[3 * g], w[3 * g + 1], w[3 * g + 2], ch + 4 * g);
    float z[2 * NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) box_muller(ch[2 * p], ch[2 * p + 1], NEG_2LN2, z[2 * p], z[2 * p + 1]);
    float nu[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) nu[k] = L.ci[k] * z[k];
    M::back(nu, d);
  } else {
    const uint64_t N = L.plane;
    const float rho = fields[site], ux = fields[N + site], uy = fields[2 * N + site];
    const float uz = (M::D == 3) ? fields[3 * N + site] : 0.0f;
    // d_i = rho/rho0 (1 + 3 u.c + 9/2 (u.c)^2 - 3/2 u^2) - 1
    const float dr = rho / L.rho0 - 1.0f;
    const float uu = (M::D == 3) ? 1.5f * (ux * ux + uy * uy + uz * uz) : 1.5f * (ux * ux + uy * uy);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float uc = (M::D == 3) ? M::CX[i] * ux + M::CY[i] * uy + M::CZ[i] * uz : M::CX[i] * ux + M::CY[i] * uy;
      const float poly = __builtin_fmaf(4.5f * uc, uc, 3.0f * uc) - uu;
      d[i] = __builtin_fmaf(1.0f + dr, poly, dr);
    }
  }
  store_site<M, S, P, Off>(L, site, d);
}

// ---------------------------------------------------------------- gathers
// WHAT: 0 populations n_i (q planes), 1 moments rho, j (1 + d planes), 2 modes
// m_k (q planes); a template parameter for the same reason as init's kind.
template <class M, int S, int P, bool WIDE, int WHAT>
__global__ void __launch_bounds__(256)
k_gather(const LatDesc* __restrict__ Lp, float* __restrict__ out) {
  using Off = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  constexpr int Q = M::Q;
  const LatDesc& L = *Lp;
  const uint32_t site = blockIdx.x * 256u + threadIdx.x;
  if (site >= L.nsites) return;
  const uint64_t N = L.plane;
  float d[Q];
  Off o[Q];
  load_site<M, S, P>(L, site, d, o);
  if constexpr (WHAT == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float ar = (M::A36[i] / 36.0f) * L.rho0;
      out[i * N + site] = __builtin_fmaf(ar, d[i], ar);
    }
  } else {
    float mu[Q];
    M::forward(d, mu);
    const float s = L.rho0 * (1.0f / 36.0f);
    if constexpr (WHAT == 1) {
      out[site] = __builtin_fmaf(s, mu[0], L.rho0);
#pragma unroll
      for (int a = 1; a <= M::D; ++a) out[a * N + site] = s * mu[a];
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) out[k * N + site] = s * mu[k];
    }
  }
}

// ---------------------------------------------------------------- health check
// Per-block partial sums (bad-site count, rho - rho0, jx, jy, jz) in fp64 over
// a grid-stride loop; a second one-block kernel reduces the partials in a
// fixed order, so the result is deterministic.
constexpr int CHECK_BLOCKS = 512;
template <class M, int S, int P, bool WIDE>
__global__ void __launch_bounds__(256)
k_check(const LatDesc* __restrict__ Lp, double* __restrict__ partial) {
  using Off = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  constexpr int Q = M::Q;
  const LatDesc& L = *Lp;
  double acc[5] = {0, 0, 0, 0, 0};  // bad sites, rho - rho0, jx, jy, jz (0 in 2D)
  // 64-bit loop counter: the stride would wrap a 32-bit site index near 2^32
  for (uint64_t i = blockIdx.x * 256u + threadIdx.x; i < L.nsites; i += (uint64_t)gridDim.x * 256u) {
    const uint32_t site = (uint32_t)i;
    float d[Q];
    Off o[Q];
    load_site<M, S, P>(L, site, d, o);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < Q; ++i) finite = finite && __builtin_isfinite(d[i]);
    float mu[Q];
    M::forward(d, mu);
    const float s = L.rho0 * (1.0f / 36.0f);
    const float rho = __builtin_fmaf(s, mu[0], L.rho0);
    if (!finite || !(rho > 0.0f)) acc[0] += 1.0;
    acc[1] += (double)(s * mu[0]);
#pragma unroll
    for (int a = 1; a <= M::D; ++a) acc[1 + a] += (double)(s * mu[a]);
  }
  __shared__ double red[5][256];
#pragma unroll
  for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < (unsigned)w)
#pragma unroll
      for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) partial[blockIdx.x * 5 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(64) k_check_final(const double* __restrict__ partial, int nblocks,
                                                    double* __restrict__ result) {
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[b * 5 + threadIdx.x];
    result[threadIdx.x] = s;
  }
}

}  // namespace lbf
