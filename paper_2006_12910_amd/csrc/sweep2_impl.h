// sweep2_impl.h -- two time steps per pass over the population buffers, for
// periodic domains whose step is the plain or obstacle sweep (no particles,
// noise, power law or boundary faces).
//
// A workgroup owns an output tile of TS_COLS x H nodes.  Phase A computes the
// first step (stream + collide, Sec. 2) on the tile and a one-node rim --
// 64 columns, one wave row each -- from global memory, exactly as k_sweep
// does, and keeps the stored values (rounded to the storage format with the
// first step's rounding bits) in LDS.  Phase B computes the second step on
// the tile, pulling from LDS, and stores it.  Every node of both steps goes
// through the same pull, collision and encoding as in k_sweep, so the result
// is bit-identical to two single steps, while each step's populations cross
// HBM once per two steps (plus the rim, read again by neighbouring tiles).
//
// The launch reads the buffer that holds the state and writes the other one,
// so after one launch the state sits in the buffer of the opposite parity;
// launches come in pairs (`which` = 0 then 1) that return it to the buffer
// the single-step convention expects (state T in f[T & 1]).
#pragma once

#include "sweep_impl.h"

namespace lbk {

// Bitwise select of a stored 16-bit value (zero-extended), then the keep
// mask: b where m is all ones, a where it is zero, all-zero bits (+0) where
// keep is zero.  The select is one three-input bitwise instruction (truth
// table 0xCA: first operand ? second : third), written as the builtin so
// that the optimiser neither packs two 16-bit selects into one register nor
// turns them into compares.
__device__ __forceinline__ uint32_t sel_keep(uint32_t a, uint32_t b, uint32_t m, uint32_t keep) {
  return __builtin_amdgcn_bitop3_b32(m, b, a, 0xCA) & keep;
}

template <int ST, int FEAT, int H, int PLM = PL_GENERIC>
__global__ __launch_bounds__(256) void k_sweep2(const DevDomain *__restrict__ doms,
                                                const int *__restrict__ prefix, int ndom,
                                                int kstep, int which) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = CompT<ST, 0>;
  constexpr bool LABELS = (FEAT & F_LABELS) != 0;
  constexpr int RS = H + 2;  // rows of the first step
  constexpr uint32_t B = sizeof(T);
  __shared__ T lds[9][RS][64];
  __shared__ uint16_t lnw[LABELS ? RS : 1][64];  // node words of the first-step nodes

  const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int dix = ndom == 1 ? 0 : find_domain(prefix, ndom, b);
  const DevDomain &D = doms[dix];
  const int local = b - prefix[dix];
  const int nx = D.nx, ny = D.ny, pitch = D.pitch;
  const int ty = local / D.tiles2_x, tx = local - ty * D.tiles2_x;
  const int x0 = tx * TS_COLS, y0 = ty * H;
  const int lane = (int)threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);

  const uint64_t T0 = *gbl(D.tstep) + (uint64_t)kstep;  // state time at the launch
  const uint32_t step1 = (uint32_t)(T0 + 1), step2 = (uint32_t)(T0 + 2);
  const uint32_t pitchB = (uint32_t)pitch * B, planeB = (uint32_t)ny * pitchB;
  const uint32_t nbytes = 9u * planeB;
  const int sb = (int)((T0 + (uint64_t)which) & 1);
  const BufRes src = pop_buffer(D.f[sb], nbytes);
  const BufRes dst = pop_buffer(D.f[sb ^ 1], nbytes);
  const bool has_lab = LABELS && D.label != nullptr;
  const bool sr = (ST == ST_F16 || ST == ST_BF16) && (D.feat & F_STOCH);
  bool bad = false;

  auto wrap = [](int c, int n) {
    c %= n;
    return c < 0 ? c + n : c;
  };
  // first-step column of this lane (wrapped), and its source columns
  const int xs = wrap(x0 - 1 + lane, nx);
  uint32_t colv[3] = {(uint32_t)wrap(xs + 1, nx) * B, (uint32_t)xs * B,
                      (uint32_t)wrap(xs - 1, nx) * B};

  // phase A: first step on rows y0 - 1 + r, r = wave, wave + 4, ...
  constexpr int UA = (RS + 3) / 4;  // rows per wave at most
  uint32_t nwa[UA];
#pragma unroll
  for (int u = 0; u < UA; ++u) {
    const int r = wave + 4 * u;
    nwa[u] = 0u;
    if (has_lab && r < RS)  // wave-uniform
      nwa[u] = gbl(D.nodew)[(uint32_t)wrap(y0 - 1 + r, ny) * pitch + xs];
  }
  // all pulls of this wave's rows first, so they are in flight together (the
  // row slots past the tile, in some waves, pull a valid row and are
  // discarded: branching around them measured 10 % slower)
  int ya[UA];
  Pulled<T> raw[UA];
  {
    uint32_t col[3] = {colv[0], colv[1], colv[2]};
    __asm__ volatile("" : "+v"(col[0]), "+v"(col[1]), "+v"(col[2]));
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const int r = wave + 4 * u;
      ya[u] = wrap(y0 - 1 + r, ny);
      uint32_t row[3];
      src_rows(ya[u], ny, pitchB, planeB, true, row);
      // FP32 and FP64: a domain without a label plane skips the label
      // selects (uniform; FP32 stress batch 1.581 against 1.610 ms per
      // step).  The same branch made the 16-bit kernels 1.6 % slower (their
      // code generation changed), so they keep the selects with zero masks.
      if (sizeof(T) == 2 || has_lab)
        pull_node<T, LABELS>(src, planeB, row, col, nwa[u] & 0xffu, raw[u]);
      else
        pull_node<T, false>(src, planeB, row, col, 0u, raw[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < UA; ++u) {
    const int r = wave + 4 * u;
    if (r >= RS) break;  // wave-uniform
    const int y = ya[u];
    if constexpr (LABELS) lnw[r][lane] = (uint16_t)nwa[u];
    // A solid node's first-step values are never read: a fluid neighbour
    // whose pull would take them bounces back off its own slot instead, and
    // phase B sweeps the solid node itself with zero deviations.  So phase A
    // collides whatever a solid node pulled (finite values of its
    // neighbours) without zeroing it first, nine selects a node fewer.
    R e[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) e[i] = (R)S::raw_dec(raw[u].get(i));
    const uint32_t node = (uint32_t)y * (uint32_t)nx + (uint32_t)xs;
    bad = bad || !(fabs(scaled_drho<ST, R>(e)) < R(1e30));
    collide_node<ST, FEAT, PLM, R>(D, e, node, step1);
    // the rounding mode is uniform: each branch keeps its own writes, so no
    // merged (packed) copy of the encoded values is formed
    auto emit = [&](auto sr_tag) {
      T q[9];
      encode_node<ST, R, decltype(sr_tag)::value>(D, e, node, step1, q);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[i][r][lane] = q[i];
    };
    if (sr) emit(std::true_type{});
    else emit(std::false_type{});
  }
  __syncthreads();

  // phase B: second step on the output rows r = 1 .. H (lanes 1 .. 62),
  // pulling from LDS; a pull from a solid source bounces back off the node's
  // own opposite slot (halfway bounce-back), as in phase A.
  const int x = x0 + lane - 1;
  const bool col_ok = lane >= 1 && lane <= TS_COLS && x < nx;
  constexpr int PL = RS * 64;  // elements of one LDS plane
#pragma unroll
  for (int u = 0; u < (H + 3) / 4; ++u) {
    const int r = 1 + wave + 4 * u;
    if (r > H) break;  // wave-uniform
    const int y = y0 + r - 1;
    if (y >= ny || !col_ok) continue;
    // the active lanes (1 .. 62) read inside the array: rows r - 1 .. r + 1
    // of every plane, lanes lane - 1 .. lane + 1
    R e[9];
    if constexpr (sizeof(T) == 2) {
      // 16-bit values: read both candidates of a direction and select the
      // bits (eight more reads, three bitwise instructions a direction, no
      // lane branching around a read).  The active lanes (1 .. 62) read
      // inside the array: rows r - 1 .. r + 1 of every plane, lanes
      // lane - 1 .. lane + 1.
      const T *p = &lds[0][0][0] + r * 64 + lane;
      uint32_t v[9];  // zero-extended: one value per register
      v[0] = p[0];
#pragma unroll
      for (int i = 1; i < 9; ++i) v[i] = p[i * PL - cy(i) * 64 - cx(i)];
      if constexpr (LABELS) {
        if (has_lab) {  // wave-uniform
          const uint32_t w = lnw[r][lane];
          uint32_t o[9];
#pragma unroll
          for (int j = 1; j < 9; ++j) o[j] = p[j * PL];
          // all ones where the node is fluid (a solid node is swept with
          // zero deviations), else zero
          const uint32_t keep = (w & NODE_SOLID) ? 0u : ~0u;
#pragma unroll
          for (int i = 1; i < 9; ++i) {
            // all ones where the pull bounces back, else zero
            const uint32_t m = (uint32_t)(-(int32_t)((w >> (i - 1)) & 1u));
            v[i] = sel_keep(v[i], o[opp(i)], m, keep);
          }
          v[0] &= keep;
        }
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) e[i] = (R)S::raw_dec((T)v[i]);
    } else {
      // wider values: one read a direction, its address picked by the
      // label bit (reading both candidates measured 1.4 % slower in FP32)
      const uint32_t w = LABELS ? (uint32_t)lnw[r][lane] : 0u;
      const bool solid = LABELS && (w & NODE_SOLID);
      e[0] = solid ? R(0) : (R)S::raw_dec(lds[0][r][lane]);
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const bool bounce = LABELS && ((w >> (i - 1)) & 1u);
        const T v = bounce ? lds[opp(i)][r][lane] : lds[i][r - cy(i)][lane - cx(i)];
        e[i] = solid ? R(0) : (R)S::raw_dec(v);
      }
    }
    const uint32_t node = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
    bad = bad || !(fabs(scaled_drho<ST, R>(e)) < R(1e30));
    collide_node<ST, FEAT, PLM, R>(D, e, node, step2);
    // Ordinary (cached) stores: a tile row is 62 values, so most 128-byte
    // lines are written in two parts by neighbouring workgroups, and the
    // cache merges the parts into one line write.  Streaming stores sent the
    // parts out separately (37 % more bytes written; 8192^2 FP16 0.50 ms
    // against 0.37 ms per two steps).
    const uint32_t colB = (uint32_t)x * B, rowB = (uint32_t)y * pitchB;
    auto emit = [&](auto sr_tag) {
      T q[9];
      encode_node<ST, R, decltype(sr_tag)::value>(D, e, node, step2, q);
#pragma unroll
      for (int i = 0; i < 9; ++i) bstore<T, false>(dst, colB, (uint32_t)i * planeB + rowB, q[i]);
    };
    if (sr) emit(std::true_type{});
    else emit(std::false_type{});
  }
  if (bad) atomicOr(D.health, HEALTH_NONFINITE);
}

}  // namespace lbk
