// Two fused steps of a D2Q9 lattice per launch: the 2D form of k_step2.
//
// k_step2_2d advances a D2Q9 lattice by two steps, t and t + 1 (t even), in
// one pass over HBM: it reads the state in the even AA layout (plane i at
// site r holds n_i(r)) from one buffer and writes the state at t + 2, in the
// same layout, to a second buffer, so each population is read once (plus a
// one-site halo) and written once per two steps.
//
// Work split.  A workgroup owns a segment of F2D_W x-sites and walks a chunk
// of ylen rows along y.  Its waves 0..F2D_NW-1 hold 64 sites of the segment
// each; one more wave holds the two halo columns x0 - 1 and x0 + F2D_W
// (periodic).  For each row the first step is collided on the segment and its
// halo, and every post-collision population that lands inside the segment is
// pushed into an LDS ring of the second step's pre-collision populations: the
// c_y = -1 populations of row u belong to row u - 1, c_y = 0 to u, c_y = +1 to
// u + 1.  The second step of row u - 2 is then collided from the ring and
// pushed along c_j into the destination buffer.  Both steps of one row share
// a phase, with one barrier per phase; the ring keeps flat populations for 3
// rows, up-going for 4 and down-going for 2, as in the 3D pass (27 rows of
// F2D_W values).  The loads of the next row but one are in flight while a
// row is processed.
//
// The two steps compute exactly what two AA launches compute (same collision
// code, same noise keys, 16-bit values rounded into the ring as they would be
// stored), so the result is bit-identical to the AA pair.  WIDE (planes of 4
// GiB or more): every access goes through the descriptor of one row of one
// population plane, so no 64-bit offsets are needed; smaller planes take one
// descriptor per plane.  PROP: the identity collision (the data-movement
// floor of the pass).
#pragma once

#include "lbf_kernels.h"

namespace lbf {

constexpr int F2D_NW = 4;                       // waves over the segment (measured: 4 beats 2 and 8)
constexpr int F2D_W = 64 * F2D_NW;              // x-sites of a segment
constexpr int F2D_THREADS = (F2D_NW + 1) * 64;  // segment waves + the halo-column wave

template <class M> struct YClass {
  // index of population i among the populations with its c_y
  static constexpr int idx(int i) {
    int n = 0;
    for (int j = 0; j < i; ++j) n += (M::CY[j] == M::CY[i]) ? 1 : 0;
    return n;
  }
};

struct F2DRing {
  static constexpr int TP = F2D_W;               // sites of a row segment
  static constexpr int NF = 3, NU = 3, ND = 3;   // D2Q9 populations with c_y = 0, +1, -1
  static constexpr int SF = 3, SU = 4, SD = 2;   // ring slots (rows in flight) per class
  static constexpr int BASE_U = SF * NF * TP;
  static constexpr int BASE_D = BASE_U + SU * NU * TP;
  static constexpr int TOTAL = BASE_D + SD * ND * TP;
  // element offset of population i's row in the slots (fs, us, ds)
  static __device__ __forceinline__ uint32_t base(int i, uint32_t fs, uint32_t us, uint32_t ds) {
    const int c = D2Q9::CY[i];
    const uint32_t k = (uint32_t)YClass<D2Q9>::idx(i) * TP;
    if (c == 0) return fs * (NF * TP) + k;
    if (c > 0) return BASE_U + us * (NU * TP) + k;
    return BASE_D + ds * (ND * TP) + k;
  }
};

template <int S, bool PROP, bool WIDE>
__global__ void __launch_bounds__(F2D_THREADS)
k_step2_2d(const LatDesc* __restrict__ src, uint64_t dst_base, const uint64_t* __restrict__ d_t, uint32_t t_off,
           uint32_t ntx, uint32_t nty, uint32_t ylen) {
  using M = D2Q9;
  using C = Codec<S>;
  using T = typename C::T;
  using U = typename Carry<T>::U;  // register form of the prefetched values
  using R = F2DRing;
  constexpr int Q = M::Q;
  constexpr uint32_t ES = sizeof(T);
  __shared__ T ring[R::TOTAL];
  const LatDesc& L = *src;
  (void)nty;

  // segment: each XCD takes one contiguous eighth of the segments (x fastest,
  // then the y chunk), so segments sharing halo lines run on one L2
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x, 1);
  const uint32_t txi = b % ntx, tyi = b / ntx;
  const uint32_t nx = L.nx, ny = L.ny;
  const uint32_t x0 = txi * (uint32_t)F2D_W, y0 = tyi * ylen;
  const uint32_t TW = min((uint32_t)F2D_W, nx - x0), YC = min(ylen, ny - y0);
  const uint32_t NIT = YC + 3u;  // phase it: first step of row y0 + it - 1, second of y0 + it - 3
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
  const uint64_t t = *d_t + t_off;

  // first-step site of this lane, in segment coordinates sx in [-1, TW]
  int sx;
  bool act1;
  if (w < (uint32_t)F2D_NW) {
    sx = (int)(w * 64u + lane);
    act1 = (uint32_t)sx < TW;
  } else {
    sx = lane == 0u ? -1 : (int)TW;
    act1 = lane < 2u;
  }
  const int gx = (int)x0 + sx;
  const uint32_t x1 = gx < 0 ? nx - 1u : ((uint32_t)gx >= nx ? 0u : (uint32_t)gx);

  // second-step site of this lane (segment waves); periodic x neighbours
  const uint32_t lidx = w * 64u + lane;
  const bool act2 = w < (uint32_t)F2D_NW && lidx < TW;
  const uint32_t x2 = x0 + lidx;
  const uint32_t bx = x2 * ES;
  const uint32_t bxm = (x2 == 0 ? nx - 1u : x2 - 1u) * ES;
  const uint32_t bxp = (x2 + 1u >= nx ? 0u : x2 + 1u) * ES;

  auto yfirst = [&](uint32_t it) {  // lattice y of the first-step row of phase it
    const int yy = (int)y0 + (int)it - 1;
    return yy < 0 ? ny - 1u : ((uint32_t)yy >= ny ? 0u : (uint32_t)yy);
  };
  auto load_row = [&](uint32_t it, U (&v)[Q]) {
    const uint32_t yf = yfirst(it);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if constexpr (WIDE) v[i] = Carry<T>::wrap(Raw<T>::template ld<0>(slice_rsrc(L.base, L.plane, i, yf, nx, ES), x1 * ES, 0u));
      else v[i] = Carry<T>::wrap(Raw<T>::template ld<0>(plane_rsrc(L, i, ES), x1 * ES, yf * nx * ES));
    }
  };
  // first step of row u = it - 1: collide, push into P(u - 1), P(u), P(u + 1)
  auto first = [&](uint32_t it, const U (&v)[Q]) {
    if (!act1 || it > YC + 1u) return;
    float d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = C::dec(Carry<T>::unwrap(v[i]));
    if constexpr (!PROP) collide<M>(L, d, x1 + yfirst(it) * nx, (uint32_t)t, (uint32_t)(t >> 32));
    const uint32_t fs = (it + 2u) % 3u, us = it % 4u, ds = it & 1u;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int tx = sx + M::CX[i];
      if (tx >= 0 && tx < (int)TW) ring[R::base(i, fs, us, ds) + (uint32_t)tx] = PROP ? Carry<T>::unwrap(v[i]) : C::enc(d[i]);
    }
  };
  // second step of row y0 + it - 3 from P(it - 3), pushed into the destination
  auto second = [&](uint32_t it) {
    if (it < 3u || !act2) return;
    const uint32_t y = y0 + it - 3u;
    const uint32_t fs = it % 3u, us = (it + 1u) % 4u, ds = (it + 1u) & 1u;
    T h[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = ring[R::base(i, fs, us, ds) + lidx];
    float d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = C::dec(h[i]);
    if constexpr (!PROP) {
      const uint64_t t1 = t + 1u;
      collide<M>(L, d, x2 + y * nx, (uint32_t)t1, (uint32_t)(t1 >> 32));
    }
    if constexpr (WIDE) {  // one descriptor per row of each population plane
      const uint32_t ym = y == 0 ? ny - 1u : y - 1u;
      const uint32_t yp = y + 1u >= ny ? 0u : y + 1u;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const uint32_t ys = M::CY[j] > 0 ? yp : (M::CY[j] < 0 ? ym : y);
        const uint32_t vx = M::CX[j] > 0 ? bxp : (M::CX[j] < 0 ? bxm : bx);
        const T v = PROP ? h[j] : C::enc(d[j]);
        const __amdgpu_buffer_rsrc_t r = slice_rsrc(dst_base, L.plane, j, ys, nx, ES);
        // x-shifted planes share lines with the neighbouring segments: cached; the others stream
        if (M::CX[j] != 0) Raw<T>::template st<0>(r, vx, v, 0u);
        else Raw<T>::template st<CPOL_NT>(r, vx, v, 0u);
      }
    } else {  // one descriptor per population plane, the row in the uniform offset
      const uint32_t ry = y * nx;
      const uint32_t rym = (y == 0 ? ny - 1u : y - 1u) * nx;
      const uint32_t ryp = (y + 1u >= ny ? 0u : y + 1u) * nx;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const uint32_t ro = M::CY[j] > 0 ? ryp : (M::CY[j] < 0 ? rym : ry);
        const uint32_t vx = M::CX[j] > 0 ? bxp : (M::CX[j] < 0 ? bxm : bx);
        const T v = PROP ? h[j] : C::enc(d[j]);
        if (M::CX[j] != 0) Raw<T>::template st<0>(plane_rsrc_base(dst_base, L.plane, j, ES), vx, v, ro * ES);
        else Raw<T>::template st<CPOL_NT>(plane_rsrc_base(dst_base, L.plane, j, ES), vx, v, ro * ES);
      }
    }
  };

  // two rows of loads in flight (register sets a and c, unrolled by two);
  // the first and second steps of a phase touch different ring slots, so one
  // barrier per phase suffices
  U a[Q], c[Q];
  if (act1) {
    load_row(0u, a);
    load_row(1u, c);
  }
  for (uint32_t it = 0; it < NIT; it += 2u) {
    first(it, a);
    if (act1 && it + 2u <= YC + 1u) load_row(it + 2u, a);
    second(it);
    __syncthreads();
    if (it + 1u >= NIT) break;
    first(it + 1u, c);
    if (act1 && it + 3u <= YC + 1u) load_row(it + 3u, c);
    second(it + 1u);
    __syncthreads();
  }
}

}  // namespace lbf
