// pipe.hpp - software-pipelined fused step for FP32 and the 16-bit storage
// forms (included by lbm.hip inside its anonymous namespace).
//
// Same step as k_fused (eqs. (HYDRO), (FORCE), (LBEQ)/(LBEQ2) with the
// velocity shift, the f/g coupling and the counter-term), organised for
// gfx950's memory system:
//
//  * A work-group owns a TX x TY x-y tile and marches up a chunk of z planes.
//    The own node's stored words of plane k+2 are loaded while plane k is
//    collided, so every wave keeps one plane of loads in flight during its
//    arithmetic; the words of k+1 (loaded one plane earlier) give the
//    moments of k+1 and are kept in registers for its collision.  Three word
//    sets rotate through the roles (collide, next, in flight) by unrolling the
//    z loop three times, so no register copies are made.  The words of the
//    one-node ring around the tile (one ring node per thread, by the waves
//    that hold ring nodes) are loaded with those of the own node and only
//    their moments are kept.
//  * Every load and store is a raw buffer access: the descriptor's base is
//    the population row (wave-uniform, scalar registers), the scalar offset
//    the plane, and the vector offset a per-thread byte offset within the
//    plane that is fixed for the whole kernel (nine of them: the node and its
//    eight x-y neighbours, periodic wrap included), so streaming costs no
//    vector address arithmetic.
//  * rho, psi, E and Phi = E - T_lat rho of a plane and its ring sit in one
//    float4 per node in an LDS ring of four plane slots (one barrier per
//    plane); the force uses grad Phi = grad E - T_lat grad rho.
//  * Equilibria are evaluated per pair of opposite directions (shared even
//    part, odd part of opposite sign).  The 16-bit forms compute in deviation
//    space: x = pop - pop_ref with pop_ref the rest equilibrium of
//    (rho_ref, T_ref) (f_ref,l = 3 w_l rho_ref T_lat, g_ref,l = w_l rho_kappa
//    T_ref for l >= 1), so decoding is a conversion and the equilibria carry
//    the reference in their node constants.  The rest pair is FP32 and is
//    updated in remainder form: old value plus what the moving pairs lost.
//    In the 16-bit forms that is the sum over the 18 words of old decoded
//    value minus stored value (collision change and store rounding at once,
//    each difference of two halves exact), plus the wall's change to g.

namespace pipe {

// Scalars of the pipelined kernel (compute precision FP32).
struct PParams {
  int nx, ny, nz, periodic_z;
  float omega_f, omega_g, tau_nu, G, gravity, inv_cv, gamma, rho_kappa;
  float T_d, T_u, T_lat;
  float rho_ref0, T_ref0;   // deviation reference (0 for FP32 storage: absolute values)
  float Fref, Gref;         // sum over l >= 1 of the reference populations (0 for FP32)
  int wet_d, wet_u;
  float psi_wd, psi_wu;
  int psi_form;
  float one;                // 1.0 (an opaque multiplier: a fused a * one + c of a half
                            // operand becomes one mixed-precision FMA)
};

// Stored words: kMove bytes per moving pair; x values are absolute (FP32) or
// deviations (16-bit forms).
template <typename C> struct Word;
template <> struct Word<F32> {
  using S = float2;
  static constexpr uint32_t kMove = 8;
  static constexpr uint32_t kRowOff = 0;   // direction l >= 1 at rows l (in rows of N words)
  static constexpr bool kDev = false;
  static __device__ __forceinline__ void dec(S w, float& a, float& b) {
    a = w.x;
    b = w.y;
  }
  static __device__ __forceinline__ void acc(S w, float, float& sa, float& sb) {
    sa += w.x;
    sb += w.y;
  }
};
template <> struct Word<H16> {
  using S = uint32_t;
  static constexpr uint32_t kMove = 4;
  static constexpr uint32_t kRowOff = 1;   // rows l + 1 (the FP32 rest pair takes rows 0, 1)
  static constexpr bool kDev = true;
  static __device__ __forceinline__ void dec(S w, float& a, float& b) {
    a = (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu));
    b = (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
  }
  // sa += lo, sb += hi of a stored word (the conversions fused into the adds)
  static __device__ __forceinline__ void acc(S w, float one, float& sa, float& sb) {
    sa = __builtin_fmaf((float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu)), one, sa);
    sb = __builtin_fmaf((float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)), one, sb);
  }
  // encode (a, b) with one packed round-to-nearest-even conversion; da, db
  // receive xa - stored and xb - stored, each stored half read back by a
  // mixed-precision FMA (the difference of two halves is exact in FP32 unless
  // their exponents lie more than 13 apart)
  static __device__ __forceinline__ S enc_diff(float a, float b, float one, float xa, float xb,
                                               float& da, float& db) {
    typedef float f32x2v __attribute__((ext_vector_type(2)));
    typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
    f32x2v f;
    f.x = a;
    f.y = b;
    const f16x2 h = __builtin_convertvector(f, f16x2);
    da = __builtin_fmaf(-(float)h.x, one, xa);
    db = __builtin_fmaf(-(float)h.y, one, xb);
    return __builtin_bit_cast(uint32_t, h);
  }
};
template <> struct Word<B16> {
  using S = uint32_t;
  static constexpr uint32_t kMove = 4;
  static constexpr uint32_t kRowOff = 1;
  static constexpr bool kDev = true;
  static __device__ __forceinline__ void dec(S w, float& a, float& b) {
    a = __builtin_bit_cast(float, w << 16);
    b = __builtin_bit_cast(float, w & 0xFFFF0000u);
  }
  static __device__ __forceinline__ void acc(S w, float, float& sa, float& sb) {
    float a, b;
    dec(w, a, b);
    sa += a;
    sb += b;
  }
  // round to nearest even in hardware (the packed conversion of gfx950); da,
  // db as for H16
  static __device__ __forceinline__ S enc_diff(float a, float b, float, float xa, float xb,
                                               float& da, float& db) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    bf16x2 v;
    v.x = (__bf16)a;
    v.y = (__bf16)b;
    const uint32_t u = __builtin_bit_cast(uint32_t, v);
    da = xa - __builtin_bit_cast(float, u << 16);
    db = xb - __builtin_bit_cast(float, u & 0xFFFF0000u);
    return u;
  }
};

// 1/x within one rounding: the hardware reciprocal and one Newton step.
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(__builtin_fmaf(-x, r, 1.f), r, r);
}
// e^t from the hardware 2^x, with t log2(e) carried as an unevaluated sum
// h + l (the FMA gives the product's rounding error exactly) so that the
// argument adds no error beyond t's own rounding; 2^l = 1 + l ln 2 to far
// below float precision since |l| < 2^-22.
__device__ __forceinline__ float exp_f(float t) {
  const float L = 1.44269502e+00f;    // log2(e) rounded to float
  const float Ll = 1.92596303e-08f;   // log2(e) - L
  const float h = t * L;
  const float l = __builtin_fmaf(t, Ll, __builtin_fmaf(t, L, -h));
  return __builtin_amdgcn_exp2f(h) * __builtin_fmaf(l, 0.693147181f, 1.f);
}
// psi = exp(-1/rho) of eq. (FORCE) (form 0) or the original Shan-Chen 1 - e^-rho
__device__ __forceinline__ float psi_f(float rho, int form) {
  const float e = exp_f(form ? -rho : -recip(rho));
  return form ? 1.f - e : e;
}

// Index of the x-y offset of direction l among the nine per-thread offsets:
// 0 node, 1 (+x), 2 (-x), 3 (+y), 4 (-y), 5 (+x+y), 6 (-x-y), 7 (+x-y), 8 (-x+y).
__host__ __device__ constexpr int xy_slot(int l) {
  return CX[l] == 0 ? (CY[l] == 0 ? 0 : (CY[l] > 0 ? 3 : 4))
                    : (CY[l] == 0 ? (CX[l] > 0 ? 1 : 2)
                                  : (CX[l] > 0 ? (CY[l] > 0 ? 5 : 7) : (CY[l] > 0 ? 8 : 6)));
}

// Raw buffer access (gfx9 buffer descriptors): the descriptor holds a
// wave-uniform row start, soffset the wave-uniform plane offset and the
// VGPR the per-lane byte offset within the plane; no vector address
// arithmetic.  Rows stay below 4 GiB, so every offset fits in 32 bits and the
// range check (num_records = 2^32 - 1 bytes) never triggers.  The LLVM
// buffer intrinsics are declared directly (the clang builtins of this
// toolchain lower the 64-bit load to a single dword).
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ f32x2 buf_ld_v2f32(i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.load.v2f32");
__device__ uint32_t buf_ld_i32(i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.load.i32");
__device__ void buf_st_v2f32(f32x2 v, i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.store.v2f32");
__device__ void buf_st_i32(uint32_t v, i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.store.i32");

using rsrc_t = i32x4;
__device__ __forceinline__ rsrc_t mkrsrc(const char* row) {
  const uint64_t p = (uint64_t)row;
  rsrc_t r;
  r.x = (int)(uint32_t)p;
  r.y = (int)((uint32_t)(p >> 32) & 0xFFFFu);   // base bits 47:32, stride 0
  r.z = -1;                                    // num_records
  r.w = 0x00020000;                            // gfx9 raw-buffer word 3
  return r;
}
// Cache-policy bits of a buffer access (the aux operand): bit 1 marks it
// non-temporal, so its lines are the first to leave L2.
constexpr int kNonTemporal = 2;
// Stores to the x-y slots without an x shift (the node, +y, -y) cover whole
// 128-byte lines when a row of nx words and a wave's span are whole lines
// (nx a multiple of 32, tiles of 128 x 4); these are marked non-temporal.
// An x-shifted store covers part of the line at each end, which a
// neighbouring wave or tile completes, and stays normal.  The mark is a hint:
// results do not depend on it.
__host__ __device__ constexpr bool whole_lines(int xs) { return xs == 0 || xs == 3 || xs == 4; }

template <typename T> struct BufIO;
template <> struct BufIO<uint32_t> {
  static __device__ __forceinline__ uint32_t ld(rsrc_t r, uint32_t v, uint32_t s) {
    return buf_ld_i32(r, (int)v, (int)s, 0);
  }
  template <int AUX = 0>
  static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, uint32_t x) {
    buf_st_i32(x, r, (int)v, (int)s, AUX);
  }
};
template <> struct BufIO<float2> {
  static __device__ __forceinline__ float2 ld(rsrc_t r, uint32_t v, uint32_t s) {
    const f32x2 u = buf_ld_v2f32(r, (int)v, (int)s, 0);
    return make_float2(u.x, u.y);
  }
  template <int AUX = 0>
  static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, float2 x) {
    f32x2 u;
    u.x = x.x;
    u.y = x.y;
    buf_st_v2f32(u, r, (int)v, (int)s, AUX);
  }
};
// Start of row q (row_bytes apart) of a buffer; the empty asm keeps the
// compiler from hoisting all 19 row starts into scalar registers for the
// whole kernel (it recomputes them with two scalar adds instead).
__device__ __forceinline__ const char* row_start(const char* base, size_t row_bytes, int q) {
  const char* p = base;
  asm volatile("" : "+s"(p));
  return p + (size_t)q * row_bytes;
}

// The words of one node and one plane: the rest pair and the 18 moving words.
template <typename C>
struct NodeWords {
  float2 w0;
  typename Word<C>::S w[Q];   // [0] unused
};

template <typename C, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void k_pipe(const char* __restrict__ in,
                                                 char* __restrict__ out, PParams P, int ntx,
                                                 int nty, int kz) {
  using W = Word<C>;
  using S = typename W::S;
  constexpr int NT = TX * TY;
  constexpr int PW = TX + 2, PN = PW * (TY + 2);
  constexpr int NS = 4;
  __shared__ float4 sM[NS][PN];   // (psi, rho, E, Phi) of a plane and its ring

  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const uint32_t A = (uint32_t)nx * (uint32_t)ny;   // nodes per plane
  const size_t N = (size_t)A * (size_t)nz;
  // bytes of one plane of a moving row / of the rest row, and the row starts
  const size_t plane_m = (size_t)A * W::kMove, plane_0 = (size_t)A * 8u;
  const size_t row_m = row_pitch(N) * W::kMove;

  // XCD-aware tile order (work-groups are dealt round-robin over 8 XCDs)
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = bid % ntx;
  const int rem = bid / ntx;
  const int ty = rem % nty;
  const int zc = rem / nty;
  const int x0 = tx * TX, y0 = ty * TY;
  const int k0 = zc * kz;
  const int k1 = min(k0 + kz, nz);
  const int tw = min(TX, nx - x0), th = min(TY, ny - y0);

  const int t = threadIdx.x;
  const int lx = t % TX, ly = t / TX;
  const bool active = lx < tw && ly < th;
  const int i = active ? x0 + lx : x0, j = active ? y0 + ly : y0;
  const int im = wrap(i - 1, nx), ip = wrap(i + 1, nx), jm = wrap(j - 1, ny), jp = wrap(j + 1, ny);
  const int own_s = (ly + 1) * PW + (lx + 1);

  // node index within the plane of the node and its x-y neighbours
  uint32_t xyn[9];
  xyn[0] = (uint32_t)j * nx + i;
  xyn[1] = (uint32_t)j * nx + ip;
  xyn[2] = (uint32_t)j * nx + im;
  xyn[3] = (uint32_t)jp * nx + i;
  xyn[4] = (uint32_t)jm * nx + i;
  xyn[5] = (uint32_t)jp * nx + ip;
  xyn[6] = (uint32_t)jm * nx + im;
  xyn[7] = (uint32_t)jm * nx + ip;
  xyn[8] = (uint32_t)jp * nx + im;
  uint32_t xyb[9];   // the same in bytes of a moving row
#pragma unroll
  for (int q = 0; q < 9; ++q) xyb[q] = xyn[q] * W::kMove;

  // ring nodes of this thread: ring index r = t + m NT for m < NR (NR = 2
  // when the ring has more nodes than the tile threads, wide flat tiles)
  constexpr int NR = (2 * (TX + 2) + 2 * TY + NT - 1) / NT;
  const int nring = 2 * (tw + 2) + 2 * th;
  bool ringt[NR];
  uint32_t ring_n[NR];
  int ring_s[NR];
  bool ring_wave[NR];
#pragma unroll
  for (int m = 0; m < NR; ++m) {
    const int r = t + m * NT;
    ringt[m] = r < nring;
    int rx = 0, ry = 0;
    if (ringt[m]) {
      if (r < tw + 2) {
        rx = r - 1;
        ry = -1;
      } else if (r < 2 * (tw + 2)) {
        rx = r - (tw + 2) - 1;
        ry = th;
      } else {
        const int q = r - 2 * (tw + 2);
        rx = q < th ? -1 : tw;
        ry = q < th ? q : q - th;
      }
    }
    ring_n[m] = (uint32_t)wrap(y0 + ry, ny) * nx + (uint32_t)wrap(x0 + rx, nx);
    ring_s[m] = (ry + 1) * PW + (rx + 1);
    // ring loads are issued by the waves that hold ring nodes only
    ring_wave[m] = __builtin_amdgcn_readfirstlane(r) < nring;
  }

  const bool walls = !P.periodic_z;
  auto phys = [&](int kp) { return kp < 0 ? kp + nz : (kp >= nz ? kp - nz : kp); };
  auto slot = [&](int kp) { return (kp - k0 + NS) % NS; };
  auto exists = [&](int kp) { return walls ? (kp >= 0 && kp < nz) : true; };

  // load the words of node offsets (vm: moving rows, v0: rest row) of
  // physical plane kp.  Every lane of the wave loads (lanes without a node of
  // their own read a valid node of the tile), so there is no divergence.
  auto load = [&](int kp, uint32_t vm, uint32_t v0, NodeWords<C>& nw) {
    nw.w0 = BufIO<float2>::ld(mkrsrc(row_start(in, row_m, 0)), v0, (uint32_t)kp * (uint32_t)plane_0);
#pragma unroll
    for (int l = 1; l < Q; ++l)
      nw.w[l] = BufIO<S>::ld(mkrsrc(row_start(in, row_m, l + (int)W::kRowOff)), vm,
                             (uint32_t)kp * (uint32_t)plane_m);
  };
  auto load_all = [&](int kp, NodeWords<C>& nw, NodeWords<C>* nr) {
    load(kp, xyb[0], xyn[0] * 8u, nw);
#pragma unroll
    for (int m = 0; m < NR; ++m)
      if (ring_wave[m]) load(kp, ring_n[m] * W::kMove, ring_n[m] * 8u, nr[m]);
  };
  // moments (rho, E) of a node's words, in a fixed order
  auto node_moments = [&](const NodeWords<C>& nw, float& rho, float& E) {
    float sf = 0.f, sg = 0.f;
#pragma unroll
    for (int l = 1; l < Q; ++l) W::acc(nw.w[l], P.one, sf, sg);
    rho = nw.w0.x + (P.Fref + sf);
    E = nw.w0.y + (P.Gref + sg);
  };
  auto put = [&](int s, int q, float rho, float E) {
    sM[s][q] = make_float4(psi_f(rho, P.psi_form), rho, E, E - P.T_lat * rho);
  };
  // moments of a plane's own and ring nodes into its slot
  auto fill = [&](int s, const NodeWords<C>& own, const NodeWords<C>* ring) {
    if (active) {
      float rho, E;
      node_moments(own, rho, E);
      put(s, own_s, rho, E);
    }
#pragma unroll
    for (int m = 0; m < NR; ++m)
      if (ringt[m]) {
        float rho, E;
        node_moments(ring[m], rho, E);
        put(s, ring_s[m], rho, E);
      }
  };
  // wall ghost slot: psi mirrored (or of the prescribed wall density), rho,
  // E and Phi extrapolated linearly through the wall
  auto ghost = [&](int sg, int sw, int si, int wet, float psi_w) {
    for (int q = t; q < PN; q += NT) {
      const float4 a = sM[sw][q], b = sM[si][q];
      sM[sg][q] = make_float4(wet ? psi_w : a.x, 2.f * a.y - b.y, 2.f * a.z - b.z,
                              2.f * a.w - b.w);
    }
  };

  // collision of the own node of plane k (words nw) and push streaming
  auto collide = [&](int k, const NodeWords<C>& nw) {
    const int sm = slot(k - 1), s0 = slot(k), sp = slot(k + 1);
    float xf[Q], xg[Q];
#pragma unroll
    for (int l = 1; l < Q; ++l) W::dec(nw.w[l], xf[l], xg[l]);
    const float4 me = sM[s0][own_s];
    const float psi = me.x, rho = me.y, E = me.z;
    // W-stencil gradients of psi, E and Phi, accumulated over pairs of
    // opposite neighbours (the same sums as grad_w, in pair order)
    float gpx = 0.f, gpy = 0.f, gpz = 0.f, gEx = 0.f, gEy = 0.f, gEz = 0.f;
    float gFx = 0.f, gFy = 0.f, gFz = 0.f;
#pragma unroll
    for (int l = 1; l < Q; l += 2) {
      const int lb = l + 1;
      const int sa = CZ[l] < 0 ? sm : (CZ[l] > 0 ? sp : s0);
      const int sb = CZ[lb] < 0 ? sm : (CZ[lb] > 0 ? sp : s0);
      const float4 a = sM[sa][own_s + CY[l] * PW + CX[l]];
      const float4 b = sM[sb][own_s + CY[lb] * PW + CX[lb]];
      const float wq = l < 7 ? (1.f / 6.f) : (1.f / 12.f);
      const float dp = wq * (a.x - b.x), dE = wq * (a.z - b.z), dF = wq * (a.w - b.w);
      if (CX[l]) { gpx += CX[l] * dp; gEx += CX[l] * dE; gFx += CX[l] * dF; }
      if (CY[l]) { gpy += CY[l] * dp; gEy += CY[l] * dE; gFy += CY[l] * dF; }
      if (CZ[l]) { gpz += CZ[l] * dp; gEz += CZ[l] * dE; gFz += CZ[l] * dF; }
    }
    float jx, jy, jz;
    momentum<float>(xf, jx, jy, jz);
    const float gp = -P.G * psi;
    const float Fx = gp * gpx - gFx;
    const float Fy = gp * gpy - gFy;
    const float Fz = gp * gpz - gFz - P.gravity * rho;
    const float ir = recip(rho);
    const float ux = (jx + P.tau_nu * Fx) * ir, uy = (jy + P.tau_nu * Fy) * ir,
                uz = (jz + P.tau_nu * Fz) * ir;
    const float vx = (jx + 0.5f * Fx) * ir, vy = (jy + 0.5f * Fy) * ir, vz = (jz + 0.5f * Fz) * ir;
    const float T = E * ir;
    const float Ssrc = (vx * gEx + vy * gEy + vz * gEz) * P.inv_cv;
    const float gE = P.gamma * E;
    // node constants of the equilibria (deviation references folded in)
    const float Af = 3.f * P.T_lat * (rho - P.rho_ref0) - 1.5f * rho * (ux * ux + uy * uy + uz * uz);
    const float Ag = P.rho_kappa * (T - P.T_ref0) - 1.5f * gE * (vx * vx + vy * vy + vz * vz);

    float rf = 0.f, rg = 0.f;
    // plane offsets of k - 1, k, k + 1 (wrapped when z is periodic) and the
    // wall planes (uniform over the work-group)
    const uint32_t so_m = (uint32_t)phys(k - 1) * (uint32_t)plane_m;
    const uint32_t so_0 = (uint32_t)k * (uint32_t)plane_m;
    const uint32_t so_p = (uint32_t)phys(k + 1) * (uint32_t)plane_m;
    const bool wall_d = walls && k == 0, wall_u = walls && k == nz - 1;
    // store pair (a, b) as direction q of node slot xs at plane offset so;
    // (xa, xb) is what the rest pair counts as the pair's old value (the
    // decoded word of the direction, plus the wall's change to g at a wall)
    auto store = [&](int q, uint32_t so, int xs, float a, float b, float xa, float xb) {
      const rsrc_t r = mkrsrc(row_start(out, row_m, q + (int)W::kRowOff));
      if constexpr (W::kDev) {
        float da, db;
        const S wv = W::enc_diff(a, b, P.one, xa, xb, da, db);
        rf += da;
        rg += db;
        if (whole_lines(xs))
          BufIO<S>::template st<kNonTemporal>(r, xyb[xs], so, wv);
        else
          BufIO<S>::st(r, xyb[xs], so, wv);
      } else {
        if (whole_lines(xs))
          BufIO<S>::template st<kNonTemporal>(r, xyb[xs], so, make_float2(a, b));
        else
          BufIO<S>::st(r, xyb[xs], so, make_float2(a, b));
      }
    };
#pragma unroll
    for (int l = 1; l < Q; l += 2) {
      const int lb = l + 1;   // opposite of l in this velocity order
      const float w = wlat<float>(l);
      const float cu = float(CX[l]) * ux + float(CY[l]) * uy + float(CZ[l]) * uz;
      const float cv = float(CX[l]) * vx + float(CY[l]) * vy + float(CZ[l]) * vz;
      const float wr = w * rho, we = w * gE;
      const float fs = fmaf(4.5f * wr * cu, cu, w * Af), fa = 3.f * wr * cu;
      const float gs = fmaf(4.5f * we * cv, cv, w * Ag), ga = 3.f * we * cv;
      const float wS = w * Ssrc;
      const float dfa = P.omega_f * (xf[l] - (fs + fa));
      const float dfb = P.omega_f * (xf[lb] - (fs - fa));
      const float dga = fmaf(P.omega_g, xg[l] - (gs + ga), -wS);
      const float dgb = fmaf(P.omega_g, xg[lb] - (gs - ga), -wS);
      const float fna = xf[l] - dfa, fnb = xf[lb] - dfb;
      const float gna = xg[l] - dga, gnb = xg[lb] - dgb;
      // what the pairs give up: FP32 sums the collision's changes (its stores
      // are exact); the 16-bit forms sum old minus stored value per word in
      // the store (collision change and rounding at once)
      if constexpr (!W::kDev) {
        rf += dfa + dfb;
        rg += dga + dgb;
      }
      // push: direction l from node x goes to x + c_l; at a wall it comes
      // back to x in the opposite direction (anti-bounce-back for g about
      // w_l rho_kappa T_wall)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int d = h ? lb : l;
        const float fn = h ? fnb : fna, gn = h ? gnb : gna;
        const float xa = xf[d], xb = xg[d];
        if (CZ[d] == 0) {
          store(d, so_0, xy_slot(d), fn, gn, xa, xb);
        } else if (CZ[d] > 0) {
          if (wall_u) {
            const float gb = -gn + 2.f * w * P.rho_kappa * (P.T_u - P.T_ref0);
            store(OPP[d], so_0, 0, fn, gb, xa, xb + (gb - gn));
          } else {
            store(d, so_p, xy_slot(d), fn, gn, xa, xb);
          }
        } else {
          if (wall_d) {
            const float gb = -gn + 2.f * w * P.rho_kappa * (P.T_d - P.T_ref0);
            store(OPP[d], so_0, 0, fn, gb, xa, xb + (gb - gn));
          } else {
            store(d, so_m, xy_slot(d), fn, gn, xa, xb);
          }
        }
      }
    }
    // rest pair, remainder form: mass kept, energy + S
    BufIO<float2>::template st<kNonTemporal>(mkrsrc(row_start(out, row_m, 0)), xyn[0] * 8u,
                      (uint32_t)k * (uint32_t)plane_0,
                      make_float2(nw.w0.x + rf, nw.w0.y + (Ssrc + rg)));
  };

  NodeWords<C> WA, WB, WC, RR[NR];
  // prologue: moments of plane k0 - 1 and k0, words of k0 kept, k0 + 1 in flight
  {
    NodeWords<C> tmp;
    const int km = k0 - 1;
    if (exists(km)) {
      load_all(phys(km), tmp, RR);
      fill(slot(km), tmp, RR);
    }
    load_all(k0, WA, RR);
    fill(slot(k0), WA, RR);
    const int kn = k0 + 1;
    if (exists(kn)) load_all(phys(kn), WB, RR);
  }

  // one plane: prefetch k+2, moments of k+1, barrier, collide k
  auto iter = [&](int k, NodeWords<C>& Wc, NodeWords<C>& Wn, NodeWords<C>& Wp) {
    const int kn = k + 1, kp = k + 2;
    const bool pre = kp <= k1 && exists(kp);
    if (exists(kn)) fill(slot(kn), Wn, RR);
    if (pre) load_all(phys(kp), Wp, RR);
    __syncthreads();
    if (walls && (k == 0 || kn == nz)) {
      if (k == 0) ghost(slot(-1), slot(0), slot(1), P.wet_d, P.psi_wd);
      if (kn == nz) ghost(slot(kn), slot(k), slot(k - 1), P.wet_u, P.psi_wu);
      __syncthreads();
    }
    if (active) collide(k, Wc);
  };

  for (int k = k0; k < k1; k += 3) {
    iter(k, WA, WB, WC);
    if (k + 1 < k1) iter(k + 1, WB, WC, WA);
    if (k + 2 < k1) iter(k + 2, WC, WA, WB);
  }
}

}  // namespace pipe
