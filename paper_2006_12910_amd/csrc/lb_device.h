// lb_device.h -- internal definitions shared by the library's HIP sources:
// the D2Q9 lattice, the per-domain device descriptor, storage formats and the
// thermal-noise generator.  gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbk {

// ---------------------------------------------------------------------------
// D2Q9 (Sec. 2): direction i has velocity (CX[i], CY[i]); rest, the four axis
// directions at angles (i-1) pi/2, the four diagonals at (2i-9) pi/4.
constexpr int Q = 9;
__host__ __device__ constexpr int cx(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5); }
// lattice weights 4/9, 1/9, 1/36
template <class R> __host__ __device__ constexpr R wgt(int i) {
  return i == 0 ? R(4) / R(9) : (i <= 4 ? R(1) / R(9) : R(1) / R(36));
}
// power-of-two scale of the 16-bit deviation formats: w_i * scale_i = 8/9
__host__ __device__ constexpr float dscale(int i) { return i == 0 ? 2.0f : (i <= 4 ? 8.0f : 32.0f); }

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "axis opposites");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "diagonal opposites");

// Table t1 basis polynomials of the lattice vector, for k = 3..8 (the modes
// that carry noise): 3e^2-2, 2ex^2-e^2, ex ey, (3e^2-4)ex, (3e^2-4)ey,
// 9e^4-15e^2+2; their lengths are 4, 4/9, 1/9, 2/3, 2/3, 16.
__host__ __device__ constexpr int basis_poly(int k, int i) {
  return k == 3 ? 3 * (cx(i) * cx(i) + cy(i) * cy(i)) - 2
       : k == 4 ? 2 * cx(i) * cx(i) - (cx(i) * cx(i) + cy(i) * cy(i))
       : k == 5 ? cx(i) * cy(i)
       : k == 6 ? (3 * (cx(i) * cx(i) + cy(i) * cy(i)) - 4) * cx(i)
       : k == 7 ? (3 * (cx(i) * cx(i) + cy(i) * cy(i)) - 4) * cy(i)
       : 9 * (cx(i) * cx(i) + cy(i) * cy(i)) * (cx(i) * cx(i) + cy(i) * cy(i)) -
             15 * (cx(i) * cx(i) + cy(i) * cy(i)) + 2;
}

// ---------------------------------------------------------------------------
enum : int { BC_PERIODIC = 0, BC_WALL = 1, BC_PRESSURE = 2 };
enum : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

// Feature bits of a sweep instantiation.
enum : int {
  F_LABELS = 1,    // label plane (obstacles and/or particles)
  F_NOISE = 2,     // thermal noise
  F_POWER = 4,     // power-law tau*
  F_PRESSURE = 8,  // Zou-He faces on x
  F_STOCH = 16,    // stochastic rounding of the stored values (FP32 or 16-bit)
  F_FAVG = 32,     // particle update with the mean of two steps' forces (runtime only)
  F_TRT = 64,      // two-relaxation-time collision (never with F_NOISE)
};
// Power-law exponent specialisations.
enum : int { PL_GENERIC = 0, PL_HALF = 1, PL_3Q = 2, PL_3H = 3 };

// Tiles of the two-step sweep (k_sweep2): TS_COLS output columns (the 64
// lanes of a wave less a one-node rim) by H output rows (its LDS holds H + 2
// rows of 64 columns x 9 values).  Three tile heights are instantiated per
// storage format; the default is the middle one (measured on the 185 M-site
// stress batch: 16-bit rows 13 / 14 / 15 / 16 took 1.059 / 1.037 / 1.078 /
// 1.056 ms per step, FP32 rows 9 / 10 / 11 / 12 1.625 / 1.603 / 1.648 /
// 1.644 ms, one run), and the autotuner picks among the three.
constexpr int TS_COLS = 62;
constexpr int two_step_rows_of(int storage, int k) {  // k = 0, 1, 2
  return storage == ST_F64 ? 4 + 2 * k : (storage == ST_F32 ? 6 + 4 * k : 10 + 4 * k);
}
constexpr int two_step_rows(int storage) { return two_step_rows_of(storage, 1); }

// Labels: 0 fluid, 1 solid, 2 + p inside particle p.
constexpr uint8_t LBL_FLUID = 0, LBL_SOLID = 1, LBL_PART0 = 2;
// particles per domain: labels 2 .. 2 + 249 fit the uint8 label plane
constexpr int MAX_PARTICLES = 250;

// Particle state, FP64 (double-buffered by step parity).
struct PState {
  double x, y, ux, uy, omega;
  double radius, mass, inertia, rho_ratio;
  double fx, fy, torque;  // total force/torque used in the last update
  int32_t flags, pad;
  double pad2[3];
};
static_assert(sizeof(PState) == 128, "PState layout");

// Per-particle force accumulators produced each step.
struct PForce {
  double fx, fy, torque;  // exterior link momentum exchange (Eq. MP1)
  double ljx, ljy;        // repulsion from solid nodes (Eq. MP2)
  double cx_, cy_, ctorque;  // covered/uncovered nodes (Eq. MP3), for the next step
};

// Device-side descriptor of one domain (lives in the domain's workspace).
struct alignas(256) DevDomain {
  void *f[2];          // population buffers (deviations), [9][ny][pitch]
  uint8_t *label;      // [ny][pitch] or null
  uint16_t *nodew;     // [ny][pitch] with the label plane, static: bit 8 = node
                       // is solid, bit i-1 = the source x - e_i is solid
  uint64_t *tstep;     // completed steps
  uint32_t *health;    // latched error bits
  // FP64 density check: per-block partial sums (mass_blocks of them), the
  // total, and the drift control {reference, relative tolerance} (tolerance
  // 0: no drift check)
  double *partials;
  double *mass_out;
  const double *mass_ctl;
  int mass_blocks;
  PState *pstate[2];
  PForce *pforce;
  // per sweep tile: 1 where the particle coupling of the step from state T
  // touches the tile or its halo, in near_tiles[T & 1] (null without
  // particles; written by k_near_tiles)
  uint8_t *near_tiles[2];
  int nx, ny, pitch;   // pitch in elements, a multiple of 64
  int bc_x, bc_y;
  int np;              // particles
  int tile_w, rows_per_thread, tiles_x, tiles_y;
  int tiles2_x, tiles2_y;  // tiles of the two-step sweep (k_sweep2)
  int rows2;               // their output rows (one of two_step_rows_of)
  uint32_t key0, key1; // noise generator key
  int storage, feat;
  int stream_stores;   // 1: the sweep's stores bypass the caches (see k_sweep)
  // FP64 parameters; the face densities as deviations rho_in - rho0 and
  // rho_out - rho0, formed in FP64 so that the FP32 copies carry them to
  // FP32 precision (a difference of two FP32-rounded densities near 1 would
  // err by ~5e-8, i.e. 5e-5 of a 1e-3 pressure difference)
  double rho0, tau, omega, gx, gy, drho_in, drho_out, kT;
  double pl_n, pl_K, tau_min, tau_max;
  double lj_psi, lj_rit, lj_floor;
  // omega times the equilibrium's class coefficients in the stored scaling:
  // K_1 w_1, K_5 w_5 (even parts) and K_1 l_1, K_5 l_5 (linear terms), with
  // w_1 = 1/9, w_5 = w_1/4, l_1 = 1/3, l_5 = (1 - 2 l_1)/4 (see collide_node),
  // and 9/2 times the even-part ones (the second-order term's factor);
  // set by set_collision_coefficients for a fixed relaxation time
  double cw1, cw5, cl1, cl5, cq1, cq5;
  // two relaxation times: tau_m = 1/2 + magic / (tau - 1/2) and its rate
  // (with the power law, from the local tau* on the device)
  double tau_m, omega_m, magic;
  // FP32 copies
  float rho0_f, tau_f, omega_f, gx_f, gy_f, drho_in_f, drho_out_f, kT_f;
  float pl_n_f, pl_K_f, tau_min_f, tau_max_f;
  float cw1_f, cw5_f, cl1_f, cl5_f, cq1_f, cq5_f;
  float tau_m_f, omega_m_f, magic_f;
};

// omega-scaled equilibrium coefficients of a domain with a fixed relaxation
// time, in each arithmetic's own rounding (the collision's formula with its
// constants rounded to R).
template <class R> inline void collision_coefficients(R omega, R K1, R K5, R c[6]) {
  const R W1 = R(1) / R(9), W5 = R(0.25) * W1;
  const R L1 = R(1) / R(3), L5 = (R(1) - R(2) * L1) * R(0.25);
  c[0] = omega * (K1 * W1);
  c[1] = omega * (K5 * W5);
  c[2] = omega * (K1 * L1);
  c[3] = omega * (K5 * L5);
  c[4] = R(4.5) * c[0];
  c[5] = R(4.5) * c[1];
}
inline void set_collision_coefficients(DevDomain &h) {
  const bool k16 = h.storage == ST_F16 || h.storage == ST_BF16;
  double c[6];
  collision_coefficients<double>(h.omega, k16 ? dscale(1) : 1.0, k16 ? dscale(5) : 1.0, c);
  h.cw1 = c[0]; h.cw5 = c[1]; h.cl1 = c[2]; h.cl5 = c[3]; h.cq1 = c[4]; h.cq5 = c[5];
  float cf[6];
  collision_coefficients<float>(h.omega_f, k16 ? dscale(1) : 1.0f, k16 ? dscale(5) : 1.0f, cf);
  h.cw1_f = cf[0]; h.cw5_f = cf[1]; h.cl1_f = cf[2]; h.cl5_f = cf[3];
  h.cq1_f = cf[4]; h.cq5_f = cf[5];
}

// One particle of a batch: owning domain (index into the descriptor array) and
// particle index within it.
struct PItem {
  int dom, p;
};

constexpr uint32_t HEALTH_NONFINITE = 1u, HEALTH_FAST_PARTICLE = 2u, HEALTH_LINK_OVERFLOW = 4u,
                   HEALTH_MASS_DRIFT = 8u;

// ---------------------------------------------------------------------------
// Global-address-space views of device pointers: pointers read from the
// descriptor are generic to the compiler, which would otherwise emit flat
// memory instructions.
#define LBK_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ const LBK_GLOBAL T *gbl(const T *p) {
  return (const LBK_GLOBAL T *)p;
}
template <class T> __device__ __forceinline__ LBK_GLOBAL T *gbl(T *p) { return (LBK_GLOBAL T *)p; }

// ---------------------------------------------------------------------------
// Storage formats.  Value held = (f_i - w_i rho0) * scale.
// Scale of the stored deviations of direction i: the 16-bit formats store
// d_i times 2, 8, 32 (rest, axis, diagonal); the others store d_i.
template <int ST> constexpr float kscale(int i) {
  return (ST == ST_F16 || ST == ST_BF16) ? dscale(i) : 1.0f;
}

template <int ST> struct Store;
template <> struct Store<ST_F64> {
  using T = double;
  using R = double;
  static __device__ __forceinline__ R load(const T *p, size_t o, int) { return gbl(p)[o]; }
  static __device__ __forceinline__ R dec(T v, int) { return v; }
  static __device__ __forceinline__ T enc(R v, int, uint32_t) { return v; }
  static __device__ __forceinline__ R raw_dec(T v) { return v; }
  static __device__ __forceinline__ T raw_rn(R v) { return v; }
  static __device__ __forceinline__ T raw_sr(R v, uint32_t) { return v; }
  static __device__ __forceinline__ void put(T *p, size_t o, int, R v, uint32_t) { gbl(p)[o] = v; }
};
template <> struct Store<ST_F32> {
  using T = float;
  using R = float;
  static __device__ __forceinline__ R load(const T *p, size_t o, int) { return gbl(p)[o]; }
  static __device__ __forceinline__ R dec(T v, int) { return v; }
  static __device__ __forceinline__ T enc(R v, int, uint32_t) { return v; }
  static __device__ __forceinline__ R raw_dec(T v) { return v; }
  static __device__ __forceinline__ T raw_rn(R v) { return v; }
  static __device__ __forceinline__ T raw_sr(R v, uint32_t) { return v; }
  static __device__ __forceinline__ void put(T *p, size_t o, int, R v, uint32_t) { gbl(p)[o] = v; }
};

__device__ __forceinline__ uint16_t f32_to_bf16_rn(float v) {
  uint32_t b = __float_as_uint(v);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f32_to_f16_rn(float v) {
  _Float16 h = (_Float16)v;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) {
  return (float)__builtin_bit_cast(_Float16, h);
}
// Stochastic rounding with the CDNA4 conversion instructions
// (v_cvt_sr_f16_f32 / v_cvt_sr_bf16_f32): v rounds to the upper of its two
// neighbours with probability equal to its fractional position between them,
// drawing the comparison from the high bits of r.
typedef _Float16 lbk_half2 __attribute__((ext_vector_type(2)));
typedef __bf16 lbk_bf16x2 __attribute__((ext_vector_type(2)));
// The instruction writes the low half of its destination and keeps the high
// half.  Only the low half is used, so it is written as an ALU instruction
// with a fresh output register: the builtin's form ties the destination to a
// vector operand and costs a register copy or a zeroing move per value.
__device__ __forceinline__ uint16_t f32_to_f16_sr(float v, uint32_t r) {
  uint32_t o;
  __asm__("v_cvt_sr_f16_f32 %0, %1, %2" : "=v"(o) : "v"(v), "v"(r));
  return (uint16_t)o;
}
__device__ __forceinline__ uint16_t f32_to_bf16_sr(float v, uint32_t r) {
  uint32_t o;
  __asm__("v_cvt_sr_bf16_f32 %0, %1, %2" : "=v"(o) : "v"(v), "v"(r));
  return (uint16_t)o;
}

template <> struct Store<ST_F16> {
  using T = uint16_t;
  using R = float;
  static __device__ __forceinline__ R dec(T v, int i) { return f16_to_f32(v) * (1.0f / dscale(i)); }
  static __device__ __forceinline__ R raw_dec(T v) { return f16_to_f32(v); }
  static __device__ __forceinline__ T raw_rn(R v) { return f32_to_f16_rn(v); }
  static __device__ __forceinline__ T raw_sr(R v, uint32_t r) { return f32_to_f16_sr(v, r); }
  static __device__ __forceinline__ R load(const T *p, size_t o, int i) { return dec(gbl(p)[o], i); }
  static __device__ __forceinline__ T enc(R v, int i, uint32_t rbits) {
    return rbits ? f32_to_f16_sr(v * dscale(i), rbits) : f32_to_f16_rn(v * dscale(i));
  }
  static __device__ __forceinline__ void put(T *p, size_t o, int i, R v, uint32_t rbits) {
    gbl(p)[o] = enc(v, i, rbits);
  }
};
template <> struct Store<ST_BF16> {
  using T = uint16_t;
  using R = float;
  static __device__ __forceinline__ R dec(T v, int i) { return bf16_to_f32(v) * (1.0f / dscale(i)); }
  static __device__ __forceinline__ R raw_dec(T v) { return bf16_to_f32(v); }
  static __device__ __forceinline__ T raw_rn(R v) { return f32_to_bf16_rn(v); }
  static __device__ __forceinline__ T raw_sr(R v, uint32_t r) { return f32_to_bf16_sr(v, r); }
  static __device__ __forceinline__ R load(const T *p, size_t o, int i) { return dec(gbl(p)[o], i); }
  static __device__ __forceinline__ T enc(R v, int i, uint32_t rbits) {
    return rbits ? f32_to_bf16_sr(v * dscale(i), rbits) : f32_to_bf16_rn(v * dscale(i));
  }
  static __device__ __forceinline__ void put(T *p, size_t o, int i, R v, uint32_t rbits) {
    gbl(p)[o] = enc(v, i, rbits);
  }
};

// Random bits of direction i at a node with hash h: a multiplicative hash,
// whose high bits (those the rounding instructions use) are well mixed.
__device__ __forceinline__ uint32_t sr_bits(uint32_t h, int i) {
  return (h + (uint32_t)(i + 1) * 0x9E3779B9u) * 0x85EBCA6Bu;
}

// 32-bit integer hash (Wellons' "lowbias32" mixer) for stochastic-rounding bits.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// ---------------------------------------------------------------------------
// Thermal noise: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) with
// counter (node, step, 0, 0) and key (lo32(seed), hi32(seed) ^ domain_id).
// The 128 output bits give six 21-bit integers -- the top 21 bits of w0..w3
// and (w0 & 0x7ff) << 10 | (w2 & 0x3ff), (w1 & 0x7ff) << 10 | (w3 & 0x3ff) --
// turned into uniforms (2k+1) 2^-22 and paired (w0,w1), (w2,w3), (low words)
// into three Box-Muller transforms (radius, angle) giving Theta_3..Theta_8.
// Every floating-point operation below is a single correctly rounded IEEE
// float operation (the Horner steps fused multiply-adds, nothing else
// contracted) in a fixed order, so the host's independent implementation of
// the same definition reproduces it bit-exactly.

// a ^ b ^ k as one gfx950 v_bitop3_b32 (truth table 0x96, the parity of
// the three inputs); the compiler splits a three-input XOR into two.  k is
// the round key, the same for every lane of a wave at every call site (a
// kernel argument or the domain of the workgroup's tile), so it stays in a
// scalar register.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// ln u for u in (0,1]: u = m 2^e, m folded into [sqrt(1/2), sqrt(2)];
// ln m = 2 atanh(s), s = (m-1)/(m+1), power series through s^11 (Horner with
// fused multiply-adds); ln 2 in two parts (Cody-Waite) so that e * hi is exact.
__device__ __forceinline__ float noise_log(float u) {
#pragma clang fp contract(off)
  uint32_t b = __float_as_uint(u);
  int e = (int)((b >> 23) & 0xffu) - 127;
  float m = __uint_as_float((b & 0x007fffffu) | 0x3f800000u);
  if (m > 1.41421354f) {
    m = m * 0.5f;
    e = e + 1;
  }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float s2 = s * s;
  float p = 1.0f / 11.0f;
  p = __builtin_fmaf(p, s2, 1.0f / 9.0f);
  p = __builtin_fmaf(p, s2, 1.0f / 7.0f);
  p = __builtin_fmaf(p, s2, 1.0f / 5.0f);
  p = __builtin_fmaf(p, s2, 1.0f / 3.0f);
  p = __builtin_fmaf(p, s2, 1.0f);
  const float lnm = (s + s) * p;
  const float fe = (float)e;
  return __builtin_fmaf(fe, 0.693145751953125f, __builtin_fmaf(fe, 1.42860682030941723e-6f, lnm));
}

// sin and cos of 2 pi u, u a multiple of 2^-22 in (0,1): exact reduction to a
// quadrant and r in [-1/8, 1/8]; Taylor series at a = 2 pi r through a^9 (sin)
// and a^10 (cos), Horner with fused multiply-adds.
__device__ __forceinline__ void noise_sincos2pi(float u, float &sn, float &cs) {
#pragma clang fp contract(off)
  int q = (int)(u * 4.0f);
  float r = u - 0.25f * (float)q;
  if (r > 0.125f) {
    r = r - 0.25f;
    q = q + 1;
  }
  const float a = r * 6.28318530717958647692f;
  const float a2 = a * a;
  float ps = 1.0f / 362880.0f;
  ps = __builtin_fmaf(ps, a2, -1.0f / 5040.0f);
  ps = __builtin_fmaf(ps, a2, 1.0f / 120.0f);
  ps = __builtin_fmaf(ps, a2, -1.0f / 6.0f);
  const float sa = __builtin_fmaf(a * a2, ps, a);
  float pc = -1.0f / 3628800.0f;
  pc = __builtin_fmaf(pc, a2, 1.0f / 40320.0f);
  pc = __builtin_fmaf(pc, a2, -1.0f / 720.0f);
  pc = __builtin_fmaf(pc, a2, 1.0f / 24.0f);
  pc = __builtin_fmaf(pc, a2, -0.5f);
  const float ca = __builtin_fmaf(a2, pc, 1.0f);
  switch (q & 3) {
    case 0: sn = sa; cs = ca; break;
    case 1: sn = ca; cs = -sa; break;
    case 2: sn = -sa; cs = -ca; break;
    default: sn = -ca; cs = sa; break;
  }
}

__device__ __forceinline__ void noise_pair(uint32_t kr, uint32_t ka, float &z0, float &z1) {
#pragma clang fp contract(off)
  const float ur = (float)(2u * kr + 1u) * (1.0f / 4194304.0f);
  const float ua = (float)(2u * ka + 1u) * (1.0f / 4194304.0f);
  const float rad = sqrtf(-2.0f * noise_log(ur));
  float sn, cs;
  noise_sincos2pi(ua, sn, cs);
  z0 = rad * cs;
  z1 = rad * sn;
}

// The same pair through the hardware's transcendental instructions, for
// collisions in FP32 arithmetic: v_log_f32 (log2), v_sqrt_f32, and
// v_sin_f32 / v_cos_f32, whose argument is in turns, so sin(2 pi u) needs no
// range reduction.  Six instructions a pair instead of about seventy.  On
// every uniform of the form (2k+1) 2^-22 they were measured within 1 ulp
// (log2), 1.3e-7 absolute (sin, cos) and 1.4e-7 relative (radius) of the
// exact functions, so a deviate differs from the correctly rounded
// definition above by at most ~1e-6 absolute, below what FP32 arithmetic
// resolves in the collision.  FP64 arithmetic keeps the exact definition.
__device__ __forceinline__ void noise_pair_hw(uint32_t kr, uint32_t ka, float &z0, float &z1) {
  const float ur = (float)(2u * kr + 1u) * (1.0f / 4194304.0f);
  const float ua = (float)(2u * ka + 1u) * (1.0f / 4194304.0f);
  // -2 ln u = -2 ln 2 log2 u
  const float rad = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(ur));
  z0 = rad * __builtin_amdgcn_cosf(ua);
  z1 = rad * __builtin_amdgcn_sinf(ua);
}

// Theta_3..Theta_8 of one node and step (HW: the hardware transform above).
template <bool HW = false>
__device__ __forceinline__ void noise_normals(uint32_t k0, uint32_t k1, uint32_t node,
                                              uint32_t step, float th[6]) {
  uint32_t w[4];
  philox4x32_10(node, step, 0u, 0u, k0, k1, w);
  const uint32_t b0 = ((w[0] & 0x7ffu) << 10) | (w[2] & 0x3ffu);
  const uint32_t b1 = ((w[1] & 0x7ffu) << 10) | (w[3] & 0x3ffu);
  if constexpr (HW) {
    noise_pair_hw(w[0] >> 11, w[1] >> 11, th[0], th[1]);
    noise_pair_hw(w[2] >> 11, w[3] >> 11, th[2], th[3]);
    noise_pair_hw(b0, b1, th[4], th[5]);
  } else {
    noise_pair(w[0] >> 11, w[1] >> 11, th[0], th[1]);
    noise_pair(w[2] >> 11, w[3] >> 11, th[2], th[3]);
    noise_pair(b0, b1, th[4], th[5]);
  }
}

constexpr uint16_t NODE_SOLID = 0x100;

__device__ __forceinline__ bool source_of(int nx, int ny, bool perx, bool pery, int x, int y, int i,
                                          int &sx, int &sy) {
  sx = x - cx(i);
  sy = y - cy(i);
  if (sx < 0 || sx >= nx) { if (!perx) return false; sx = sx < 0 ? sx + nx : sx - nx; }
  if (sy < 0 || sy >= ny) { if (!pery) return false; sy = sy < 0 ? sy + ny : sy - ny; }
  return true;
}

// Static node word from the label plane: NODE_SOLID for a stationary solid
// node, else bit i-1 set when the source x - e_i of the pull along i is solid
// (that pull bounces back on the node's own slot).  Sources outside a
// non-periodic edge are left clear (pressure faces reconstruct them).
__device__ __forceinline__ uint16_t node_word(const uint8_t *lab, int nx, int ny, int pitch,
                                              bool perx, bool pery, int x, int y) {
  if (lab[(size_t)y * pitch + x] == LBL_SOLID) return NODE_SOLID;
  uint16_t m = 0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    int sx, sy;
    if (!source_of(nx, ny, perx, pery, x, y, i, sx, sy)) continue;
    if (lab[(size_t)sy * pitch + sx] == LBL_SOLID) m |= (uint16_t)(1u << (i - 1));
  }
  return m;
}

// ---------------------------------------------------------------------------
// XCD-aware block order: consecutive hardware block ids are dealt round-robin
// to the 8 XCDs; remap so that each XCD walks a contiguous run of tiles and
// the halo rows it pulls stay in its own L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int NX = 8;
  if (nblocks < 2 * NX) return bid;
  const int xcd = bid % NX, local = bid / NX;
  const int per = nblocks / NX, rem = nblocks % NX;
  return xcd * per + min(xcd, rem) + local;
}

// Which domain of a batch owns block b: largest d with prefix[d] <= b.
__device__ __forceinline__ int find_domain(const int *__restrict__ prefix, int ndom, int b) {
  int lo = 0, hi = ndom - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ double min_image(double d, double len, bool periodic) {
  return periodic ? d - len * floor(d / len + 0.5) : d;
}

}  // namespace lbk
