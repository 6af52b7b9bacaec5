// sweep_pair_impl.h -- the fused stream-collide sweep for the 16-bit formats,
// two neighbouring nodes (x0, x0 + 1, x0 even) per thread.
//
// The step is the one of k_sweep (sweep_impl.h): pull with mirror-slot
// bounce-back, Zou-He faces, collision in the stored scaling, stores and
// mirror writes.  Two 16-bit nodes per lane make every pull and store a
// 4-byte access (256 bytes per wave instruction instead of 128), halve the
// address arithmetic per node, and share one node-word load.  The pull of a
// direction with cx = +1 or -1 reads the pair of source columns (x0 - cx,
// x0 + 1 - cx), a 4-byte access aligned to 2 bytes; the lanes of the first
// and last pair of a row, whose source columns wrap or are clamped, read
// their two halves separately.
#pragma once

#include "sweep_impl.h"

namespace lbk {

// 4-byte load of two 16-bit values at a 2-byte-aligned address (unaligned
// global access is enabled on the device)
typedef uint32_t lbk_u32_a2 __attribute__((aligned(2)));
__device__ __forceinline__ uint32_t ld_pair(const char LBK_GLOBAL *b, uint32_t off) {
  return *(const lbk_u32_a2 LBK_GLOBAL *)(b + off);
}

// Two nodes per lane hold twice the registers of k_sweep's lanes: the plain
// and obstacle variants are held to 4 waves per SIMD.
template <int FEAT, int WIDE> constexpr int pair_min_waves() {
  return (FEAT & (F_NOISE | F_POWER)) == 0 && WIDE == 0 ? 4 : 1;
}

template <int ST, int FEAT, int PLM, int WIDE>
__global__ __launch_bounds__(256, (pair_min_waves<FEAT, WIDE>())) void k_sweep_pair(
    const DevDomain *__restrict__ doms, const int *__restrict__ prefix, int ndom, int kstep) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = CompT<ST, WIDE>;
  static_assert(sizeof(T) == 2, "the pair sweep is for 16-bit storage");
  constexpr int U = 2;  // rows loaded before computing: 4 nodes per thread
  constexpr uint32_t B = 2;

  const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int dix = ndom == 1 ? 0 : find_domain(prefix, ndom, b);
  const DevDomain &D = doms[dix];
  const int local = b - prefix[dix];
  const int nx = D.nx, ny = D.ny, pitch = D.pitch;
  const int tw = D.tile_w, npt = D.rows_per_thread;
  const int rows_pass = 256 / tw;
  const int tyi = local / D.tiles_x, txi = local - tyi * D.tiles_x;
  const int x0 = 2 * (txi * tw + (int)threadIdx.x % tw);
  if (x0 >= nx) return;
  const bool two = x0 + 1 < nx;  // the second node exists
  const int ybase = tyi * rows_pass * npt + (int)threadIdx.x / tw;

  const uint64_t T0 = *gbl(D.tstep) + (uint64_t)kstep;  // state time of the source buffer
  const uint32_t step = (uint32_t)(T0 + 1);
  void *const f0 = D.f[0];
  void *const f1 = D.f[1];
  const char LBK_GLOBAL *src = (const char LBK_GLOBAL *)((T0 & 1) ? f1 : f0);
  char LBK_GLOBAL *dst = (char LBK_GLOBAL *)((T0 & 1) ? f0 : f1);
  const uint32_t pitchB = (uint32_t)pitch * B;
  const uint32_t planeB = (uint32_t)ny * pitchB;
  bool bad = false;  // non-finite density seen by this thread
  const bool perx = D.bc_x == BC_PERIODIC, wallx = D.bc_x == BC_WALL;
  const bool pery = D.bc_y == BC_PERIODIC, wally = D.bc_y == BC_WALL;
  const bool pressx = D.bc_x == BC_PRESSURE;
  const bool has_lab = (FEAT & F_LABELS) != 0 && D.label != nullptr;
  const bool walls = !has_lab && (wallx || wally);
  // every source column pair of this lane is two adjacent columns
  const bool fast = x0 >= 2 && x0 + 2 < nx;

  // per node v (x = x0 + v; a missing second node repeats the first): source
  // columns x+1, x, x-1 in bytes, wall-column and inside-column direction masks
  uint32_t col[2][3], wall_cols[2], cols_in[2];
  bool face[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int x = v && two ? x0 + 1 : x0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int c = x + 1 - k;
      col[v][k] = (uint32_t)(c < 0 ? (perx ? c + nx : x) : (c >= nx ? (perx ? c - nx : x) : c)) * B;
    }
    wall_cols[v] = wallx ? (x == 1 ? dirs_cx(1) : 0u) | (x == nx - 2 ? dirs_cx(-1) : 0u) : 0u;
    cols_in[v] = 0xffu & ~(!perx && x == 0 ? dirs_cx(1) : 0u) & ~(!perx && x == nx - 1 ? dirs_cx(-1) : 0u);
    face[v] = pressx && (x == 0 || x == nx - 1);
  }
  // byte offset of the pair pulled along a direction with x-component cx
  // (a safe aligned one for the edge lanes, which then read halves)
  const uint32_t pair_m = (uint32_t)(fast ? x0 + 1 : x0) * B;  // cx = -1: columns x0+1, x0+2
  const uint32_t pair_0 = (uint32_t)x0 * B;                     // cx =  0
  const uint32_t pair_p = (uint32_t)(fast ? x0 - 1 : x0) * B;  // cx = +1: columns x0-1, x0
  const uint32_t pairc[3] = {pair_m, pair_0, pair_p};           // index 1 + cx

#pragma unroll 1
  for (int r0 = 0; r0 < npt; r0 += U) {
    int yg = ybase + r0 * rows_pass;
    __asm__ volatile("" : "+v"(yg));
    uint32_t raw[U][9];
    uint32_t nw[U];
    uint32_t act[U];  // bit v: node v is computed
    // phase 1: every load of the row group (pairs), none depending on another
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int yr = yg + u * rows_pass;
      const bool valid = r0 + u < npt && yr < ny;
      const int y = valid ? yr : ny - 1;
      uint32_t row[3];
      src_rows(y, ny, pitchB, planeB, pery, row);
      // node words of the pair (the plane is as wide as the pitch, x0 even)
      uint32_t w = has_lab ? ldb<uint32_t>((const char LBK_GLOBAL *)D.nodew, row[1] + pair_0) : 0u;
      if (!two) w &= 0xffffu;
      nw[u] = valid ? w : 0u;
      uint32_t a = 0;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int x = x0 + v;
        const bool wall =
            walls && ((wally && (y == 0 || y == ny - 1)) || (wallx && (x == 0 || x == nx - 1)));
        a |= (valid && (v == 0 || two) && !wall) ? 1u << v : 0u;
      }
      act[u] = a;
#pragma unroll
      for (int i = 0; i < 9; ++i)
        raw[u][i] = ld_pair(src, (uint32_t)i * planeB + (row[1 + cy(i)] + pairc[1 + cx(i)]));
      if (!fast) {
        // first or last pair of the row: the two halves come from their own
        // (wrapped or clamped) columns
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          const uint32_t base = (uint32_t)i * planeB + row[1 + cy(i)];
          const uint32_t lo = ldb<T>(src, base + col[0][1 + cx(i)]);
          const uint32_t hi = ldb<T>(src, base + col[1][1 + cx(i)]);
          raw[u][i] = lo | (hi << 16);
        }
      }
    }
    // phase 2: per node boundary reconstruction, collision, stores
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int y = yg + u * rows_pass;
      uint32_t am = act[u] & ~((nw[u] & NODE_SOLID ? 1u : 0u) | ((nw[u] >> 16) & NODE_SOLID ? 2u : 0u));
      if (!am) continue;
      uint32_t row[3];  // rows y + 1, y, y - 1; inside the domain for a computed node
      src_rows(y, ny, pitchB, planeB, true, row);
      auto emit = [&](auto sr_tag) {
        constexpr bool SR = decltype(sr_tag)::value;
        uint32_t qq[9] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          if (!((am >> v) & 1u)) continue;
          R e[9];
#pragma unroll
          for (int i = 0; i < 9; ++i) e[i] = (R)S::raw_dec((T)(v ? raw[u][i] >> 16 : raw[u][i]));
          if (face[v]) {
            // 2/3 + 2 (1/6) = 1 exactly in the chosen constants; unscaled values
            const R half = R(0.5), third2 = R(2) / R(3), sixth = (R(1) - third2) * R(0.5);
#pragma unroll
            for (int i = 0; i < 9; ++i) e[i] *= R(1) / R(kscale<ST>(i));
            if (x0 + v == 0) {
              const R s = e[0] + e[2] + e[4] + R(2) * (e[3] + e[6] + e[7]);
              const R rux = (par<R>(D.rho_in, D.rho_in_f) - par<R>(D.rho0, D.rho0_f)) - s;
              e[1] = e[3] + third2 * rux;
              e[5] = e[7] - half * (e[2] - e[4]) + sixth * rux;
              e[8] = e[6] + half * (e[2] - e[4]) + sixth * rux;
            } else {
              const R s = e[0] + e[2] + e[4] + R(2) * (e[1] + e[5] + e[8]);
              const R rux = s - (par<R>(D.rho_out, D.rho_out_f) - par<R>(D.rho0, D.rho0_f));
              e[3] = e[1] - third2 * rux;
              e[7] = e[5] + half * (e[2] - e[4]) - sixth * rux;
              e[6] = e[8] - half * (e[2] - e[4]) - sixth * rux;
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) e[i] *= R(kscale<ST>(i));
          }
          const uint32_t node = (uint32_t)y * (uint32_t)nx + (uint32_t)(x0 + v);
          collide_node<ST, FEAT, PLM, R>(D, e, node, step);
          bad = bad || !(fabs(scaled_drho<ST, R>(e)) < R(1e30));
          T q[9];
          encode_node<ST, R, SR>(D, e, node, step, q);
#pragma unroll
          for (int i = 0; i < 9; ++i) qq[i] = v ? (qq[i] & 0xffffu) | ((uint32_t)q[i] << 16) : (uint32_t)q[i];
          // mirror writes of node v (see k_sweep)
          uint32_t mb = (v ? nw[u] >> 16 : nw[u]) & 0xffu;
          if (walls) {
            const uint32_t wall_rows =
                wally ? (y == 1 ? dirs_cy(1) : 0u) | (y == ny - 2 ? dirs_cy(-1) : 0u) : 0u;
            mb = (wall_cols[v] | wall_rows) & cols_in[v];
          }
          if (mb) {
#pragma unroll
            for (int i = 1; i < 9; ++i) {
              if (!((mb >> (i - 1)) & 1u)) continue;
              stb<T>(dst, (uint32_t)i * planeB + (row[1 + cy(i)] + col[v][1 + cx(i)]), q[opp(i)]);
            }
          }
        }
        const uint32_t hereB = row[1] + pair_0;
        if (am == 3u) {
#pragma unroll
          for (int i = 0; i < 9; ++i) stb<uint32_t>(dst, (uint32_t)i * planeB + hereB, qq[i]);
        } else if (am == 1u) {
#pragma unroll
          for (int i = 0; i < 9; ++i) stb<T>(dst, (uint32_t)i * planeB + hereB, (T)qq[i]);
        } else {
#pragma unroll
          for (int i = 0; i < 9; ++i) stb<T>(dst, (uint32_t)i * planeB + hereB + B, (T)(qq[i] >> 16));
        }
      };
      if (D.feat & F_STOCH) emit(std::true_type{});
      else emit(std::false_type{});
    }
  }
  if (bad) atomicOr(D.health, HEALTH_NONFINITE);
}

}  // namespace lbk
