// Device arithmetic of one lattice node: the mean-free-path wall function,
// the effective relaxation times and the MRT collision of one species.
//
// Paper: Wang, Xu & Guo, arXiv:1603.08221, Sec. 3.1 (Eqs. (MR), (m), (S),
// (feq), (rhou), (EQFrb), (taos), (EQFrsp)) and Sec. 3.2 (Eqs. (taoq), (A12)).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "e1_table.h"

namespace lbsep {

// Precision traits: table, cut-off and math entry points per arithmetic type.
// double: IEEE-exact library exp / log / sqrt and division (the FP64 path is
// the reference precision). float: the hardware exp2 / log2 / reciprocal /
// reciprocal square root (about 1 ulp), enough for the FP32 paths' 1e-5 bound.
template <typename T> struct E1Traits;

template <> struct E1Traits<double> {
  static constexpr bool kRational = false;  // octave Chebyshev interpolants for a > 1
  static constexpr int kSeg = LBSEP_E1_F64_NSEG;
  static constexpr int kDeg = LBSEP_E1_F64_DEG;
  static constexpr int kSer = LBSEP_E1_F64_NSER;
  __device__ static double pa(int k) { return LBSEP_TBL(lbsep_psi_a_f64)[k]; }
  __device__ static double pb(int k) { return LBSEP_TBL(lbsep_psi_b_f64)[k]; }
  __device__ static double cheb(int s, int k) { return LBSEP_TBL(lbsep_e1_cheb_f64)[s][k]; }
  __device__ static double ex(double a) { return exp(a); }
  __device__ static double ln(double a) { return log(a); }
  __device__ static double rsq(double a) { return 1.0 / sqrt(a); }
  __device__ static double rcp(double a) { return 1.0 / a; }
};

template <> struct E1Traits<float> {
  static constexpr bool kRational = true;  // one rational in 1/a for a > 1
  static constexpr int kSeg = 0;
  static constexpr int kDeg = 0;
  static constexpr int kSer = LBSEP_E1_F32_NSER;
  __device__ static float pa(int k) { return LBSEP_TBL(lbsep_psi_a_f32)[k]; }
  __device__ static float pb(int k) { return LBSEP_TBL(lbsep_psi_b_f32)[k]; }
  __device__ static float cheb(int, int) { return 0.0f; }
  __device__ static float ex(float a) { return __builtin_amdgcn_exp2f(a * 1.4426950408889634f); }
  __device__ static float ln(float a) { return __builtin_amdgcn_logf(a) * 0.6931471805599453f; }
  __device__ static float rsq(float a) { return __builtin_amdgcn_rsqf(a); }
  __device__ static float rcp(float a) { return __builtin_amdgcn_rcpf(a); }
};

// c_0 + c_1 s + ... + c_10 s^10 by Horner's rule with fused multiply-adds, the
// coefficients wavefront-uniform values in scalar registers used in place (the
// compiler's own choice, the accumulating multiply-add, would first copy each
// one into vector registers: two moves per multiply-add).
__device__ __forceinline__ double horner10_uniform(double s, const double* c) {
  static_assert(LBSEP_PW_F64_DEG == 10, "one multiply-add per coefficient below");
  double p;
  asm("v_mov_b64 %0, %2\n\t"
      "v_fma_f64 %0, %0, %1, %3\n\t"
      "v_fma_f64 %0, %0, %1, %4\n\t"
      "v_fma_f64 %0, %0, %1, %5\n\t"
      "v_fma_f64 %0, %0, %1, %6\n\t"
      "v_fma_f64 %0, %0, %1, %7\n\t"
      "v_fma_f64 %0, %0, %1, %8\n\t"
      "v_fma_f64 %0, %0, %1, %9\n\t"
      "v_fma_f64 %0, %0, %1, %10\n\t"
      "v_fma_f64 %0, %0, %1, %11\n\t"
      "v_fma_f64 %0, %0, %1, %12"
      : "=&v"(p)
      : "v"(s), "s"(c[10]), "s"(c[9]), "s"(c[8]), "s"(c[7]), "s"(c[6]), "s"(c[5]), "s"(c[4]), "s"(c[3]),
        "s"(c[2]), "s"(c[1]), "s"(c[0]));
  return p;
}

// FP64 psi and h on 2^-20 <= a < 64 from the piecewise table: each octave in
// eight parts, a degree-10 polynomial per part in the local variable s (exact).
// The part index is usually the same on every lane of a wavefront (its lanes
// are neighbouring columns of one row), so the lanes are served one distinct
// index at a time (the first remaining lane's), with the coefficients as
// scalar loads shared by the wavefront.
template <bool WANT_H>
__device__ __forceinline__ void wall_psi_pw(double a, double& psi, double& h) {
  constexpr int kPer = LBSEP_PW_F64_PER_OCT, kDeg = LBSEP_PW_F64_DEG;
  static_assert(kPer == 8, "the part index takes the top three mantissa bits");
  const int hi = __double2hiint(a);
  const int e = ((hi >> 20) & 0x7ff) - 1023;
  const int m = (hi >> 17) & 7;
  const int q = min(max((e - LBSEP_PW_F64_LO_OCT) * kPer + m, 0), LBSEP_PW_F64_N - 1);
  const double s = ldexp(a, 4 - e) - double(17 + 2 * m);
  double pv = 0.0, hv = 0.0;
#pragma unroll 1
  for (;;) {
    const int u = __builtin_amdgcn_readfirstlane(q);
    const double* cp = LBSEP_TBL(lbsep_wall_pw_f64)[u][0];
    double p = horner10_uniform(s, cp);
    // keeps the evaluation in the loop on part u's coefficients (otherwise the
    // compiler substitutes q for u under the test below and loads per lane)
    asm volatile("" : "+v"(p));
    double r = 0.0;
    if (WANT_H) {
      const double* ch = LBSEP_TBL(lbsep_wall_pw_f64)[u][1];
      r = horner10_uniform(s, ch);
      asm volatile("" : "+v"(r));
    }
    if (u == q) {
      pv = p;
      hv = r;
      break;
    }
  }
  psi = pv;
  if (WANT_H) h = hv;
}

// psi = A(a) + a^2 ln a and h = B(a) + a ln a (the power series for small a).
template <typename T, bool WANT_H>
__device__ __forceinline__ void wall_psi_small(T a, T& psi, T& h) {
  using E = E1Traits<T>;
  const T la = E::ln(a);
  T A = E::pa(E::kSer - 1);
#pragma unroll
  for (int k = E::kSer - 2; k >= 1; --k) A = A * a + E::pa(k);
  psi = A * a + a * a * la;  // alpha_0 = 0
  if (WANT_H) {
    T B = E::pb(E::kSer - 1);
#pragma unroll
    for (int k = E::kSer - 2; k >= 0; --k) B = B * a + E::pb(k);
    h = B + a * la;
  }
}

// psi(a) = 1 + (a - 1) e^-a - a^2 E1(a) (wall function of Sec. 3.1) and, when
// WANT_H, h(a) = e^-a - a E1(a) = psi'(a) / 2. FP64 has two evaluations,
// chosen per channel (`table`, the same in every kernel that steps it); they
// agree to about 1e-16:
//   table, 2^-20 <= a < 64: the piecewise polynomials above. Few operations,
//                 but each evaluation waits for its coefficients: the choice
//                 for channels that fill the GPU.
//   otherwise (and below 2^-20):
//   a <= 1      : psi = A(a) + a^2 ln a, h = B(a) + a ln a, with A and B entire
//                 power series (Horner); one logarithm, no exponential.
//   1 < a       : E1 = e^-a G(a) / a with G(a) = a e^a E1(a), so
//                 psi = 1 + e^-a (a - 1 - a G) and h = e^-a (1 - G); G from the
//                 octave's Chebyshev interpolant (Clenshaw). Registers only:
//                 the choice for small channels, whose steps are latency-bound.
//   a >= 64     : psi = 1 and h = 0 to FP64 precision.
// FP32 (`table` ignored): the series for a <= 1; above, G = P(1/a) / Q(1/a),
// one (5, 5) rational on all of (1, inf), and e^-a underflows where psi rounds
// to 1.
template <typename T, bool WANT_H>
__device__ __forceinline__ void wall_psi(T a, T& psi, T& h, bool table) {
  using E = E1Traits<T>;
  if (!(a > T(0))) {
    psi = T(0);
    h = T(1);
    return;
  }
  if constexpr (!E::kRational) {
    // every argument of the table evaluation returns here (with `table` known
    // at compile time, the series form below is then not compiled in)
    if (table) {
      if (a < T(0x1p-20)) {
        wall_psi_small<T, WANT_H>(a, psi, h);
      } else if (a < T(64)) {
        wall_psi_pw<WANT_H>(a, psi, h);
      } else {
        psi = T(1);
        h = T(0);
      }
      return;
    }
  }
  if (a <= T(1)) {
    wall_psi_small<T, WANT_H>(a, psi, h);
    return;
  }
  if constexpr (E::kRational) {
    // from a = 17 on, e^-a (a - 1 - a G) is below 5e-9 in magnitude and psi
    // rounds to 1 exactly; h (below 3e-9) enters only as 1 - h, which rounds
    // to 1 as well: the shortcut gives the same bits downstream
    if (a >= T(17)) {
      psi = T(1);
      h = T(0);
      return;
    }
    const T u = E::rcp(a);
    T P = T(lbsep_e1_rat_p_f32[LBSEP_E1_F32_RAT_DEG]);
    T Q = T(lbsep_e1_rat_q_f32[LBSEP_E1_F32_RAT_DEG]);
#pragma unroll
    for (int k = LBSEP_E1_F32_RAT_DEG - 1; k >= 0; --k) {
      P = P * u + T(lbsep_e1_rat_p_f32[k]);
      Q = Q * u + T(lbsep_e1_rat_q_f32[k]);
    }
    const T g = P * E::rcp(Q);
    const T ea = E::ex(-a);
    psi = T(1) + ea * (a - T(1) - a * g);
    if (WANT_H) h = ea * (T(1) - g);
    return;
  } else {
    const int seg = ilogb(a);
    if (seg >= E::kSeg) {
      psi = T(1);
      h = T(0);
      return;
    }
    // Clenshaw on the octave's Chebyshev series, one octave at a time over a
    // wave-uniform loop: the coefficients are then scalar loads shared by the
    // wave (a wave's arguments usually span one or two octaves).
    T g = T(0);
#pragma unroll 1
    for (int sg = 0; sg < E::kSeg; ++sg) {
      if (!__any(seg == sg)) continue;
      // t = (2a - 3 * 2^sg) / 2^sg, exact for the lanes of this octave
      const T t = ldexp(a, 1 - sg) - T(3);
      const T t2 = t + t;
      T b1 = T(0), b2 = T(0);
#pragma unroll
      for (int k = E::kDeg; k >= 1; --k) {
        const T b0 = E::cheb(sg, k) + t2 * b1 - b2;
        b2 = b1;
        b1 = b0;
      }
      const T gs = E::cheb(sg, 0) + t * b1 - b2;
      if (seg == sg) g = gs;
    }
    const T ea = E::ex(-a);
    psi = T(1) + ea * (a - T(1) - a * g);
    if (WANT_H) h = ea * (T(1) - g);
  }
}

template <typename T>
__device__ __forceinline__ void wall_psi(T a, T& psi, T& h, bool table) {
  wall_psi<T, true>(a, psi, h, table);
}

template <typename T>
__device__ __forceinline__ T wall_psi_only(T a, bool table) {
  T p, h;
  wall_psi<T, false>(a, p, h, table);
  return p;
}

// Constants derived on the host from the problem statement.
struct RelaxConsts {
  double inv_m[2];  // 1 / m_sigma
  double s[2];      // s_sigma = m_min / m_sigma
  double lam_p;     // lambda * P = Kn_out * H * P_out (mean free path at pressure P is lam_p / P)
  double inv_lam_p; // 1 / lam_p
  double kpref;     // sqrt(6 m_min / pi): k = kpref / sqrt(m_x) in Eq. (taos)
  double dpref;     // (3/2) sqrt(3 m_0 m_a m_b / m_min): Eq. (EQFrsp) prefactor times m_x
  double tq_a;      // 24 varsigma^2 A2 (= 4 pi A2), Eq. (taoq)
  double tq_b;      // 30 varsigma A1, Eq. (taoq)
  double height;    // H = ny
  double tau_bgk;
  int mfp_off;
  int bgk;
  int psi_table;    // FP64 wall function from the piecewise polynomials (1) or its series/exponential form (0)
};

// Relaxation times of one node, recomputed every step from its pre-collision
// state. The common part (mixture quantities and mean free path) and the final
// formulas are shared; the seven wall-function evaluations are either done by
// one lane (relaxation_times) or split over a lane pair (relaxation_times_pair).
// tb: the FP64 wall-function evaluation (the piecewise polynomials or the
// series form, see wall_psi).
template <typename T>
struct NodeGas {
  T xa, xb, mx, il, lam, k;
};

template <typename T>
__device__ __forceinline__ NodeGas<T> node_gas(const RelaxConsts& c, T rho_a, T rho_b) {
  using E = E1Traits<T>;
  NodeGas<T> g;
  const T na = rho_a * T(c.inv_m[0]);
  const T nb = rho_b * T(c.inv_m[1]);
  const T inv_n = E::rcp(na + nb);
  g.xa = na * inv_n;
  g.xb = nb * inv_n;
  g.mx = (rho_a + rho_b) * inv_n;                                        // m_x = rho / n
  const T pres = T(1.0 / 3.0) * (T(c.s[0]) * rho_a + T(c.s[1]) * rho_b);  // P = n k_B T
  g.il = pres * T(c.inv_lam_p);                                          // 1 / lambda (R5)
  g.lam = T(c.lam_p) * E::rcp(pres);                                     // mean free path at P
  g.k = T(c.kpref) * E::rsq(g.mx);                                       // sqrt(6 m_min / (pi m_x))
  return g;
}

// tau_s (Eq. (taos)), tau_d (Eq. (EQFrsp)), tau_q (Eq. (taoq)) from the wall
// function values Psi(y; lambda), Psi(y; lambda_a), Psi(y; lambda_b) and the wall
// values tau~_s(0), tau~'_s(0).
template <typename T>
__device__ __forceinline__ void taus_from_psi(const RelaxConsts& c, const NodeGas<T>& g, T psi_m, T psi_a, T psi_b,
                                              T tt0, T dtt0, T& tau_s, T& tau_d, T& tau_q) {
  using E = E1Traits<T>;
  tau_s = T(0.5) + g.lam * psi_m * g.k;
  const T sa = E::rsq(psi_a) + E::rsq(psi_b);
  tau_d = T(0.5) + T(c.dpref) * g.lam * E::rcp(g.mx * sa * sa);
  const T r0 = E::rcp(tt0);
  tau_q = T(0.5) + (T(3) * r0 + T(c.tq_a) * tt0) * T(1.0 / 16.0) +
          dtt0 * (T(12) * r0 * r0 + T(c.tq_b) * r0) * T(1.0 / 16.0);
}

// One lane per node: all seven wall-function evaluations here.
template <typename T>
__device__ __forceinline__ void relaxation_times(const RelaxConsts& c, int j, T rho_a, T rho_b, T& tau_s,
                                                 T& tau_d, T& tau_q, bool tb) {
  if (c.bgk) {
    tau_s = tau_d = tau_q = T(c.tau_bgk);
    return;
  }
  const NodeGas<T> g = node_gas<T>(c, rho_a, rho_b);
  if (c.mfp_off) {
    taus_from_psi<T>(c, g, T(1), T(1), T(1), g.k * g.lam, T(0), tau_s, tau_d, tau_q);
    return;
  }
  const T y = T(j) + T(0.5);
  const T ay = y * g.il, ab = (T(c.height) - y) * g.il;
  const T psi_m = T(0.5) * (wall_psi_only(ay, tb) + wall_psi_only(ab, tb));
  // lambda_sigma = lambda / x_sigma  ->  y / lambda_sigma = x_sigma y / lambda (R6)
  const T psi_a = T(0.5) * (wall_psi_only(g.xa * ay, tb) + wall_psi_only(g.xa * ab, tb));
  const T psi_b = T(0.5) * (wall_psi_only(g.xb * ay, tb) + wall_psi_only(g.xb * ab, tb));
  // wall values (R8): tau~_s(0) = k lam psi(H/lam) / 2, tau~'_s(0) = k (1 - h(H/lam))
  T pw, hw;
  wall_psi(T(c.height) * g.il, pw, hw, tb);
  taus_from_psi<T>(c, g, psi_m, psi_a, psi_b, T(0.5) * g.k * g.lam * pw, g.k * (T(1) - hw), tau_s, tau_d,
                   tau_q);
}

// The value v of lane (this lane ^ m). For m = 1 and m = 2 a DPP quad
// permutation moves it in the vector ALU, for m = 32 v_permlane32_swap (its
// first result holds the lower half twice, its second the upper half twice);
// other masks go through ds_bpermute (__shfl_xor), a trip through the LDS
// crossbar. All are exact moves. The partner lane must be active.
__device__ __forceinline__ int lane_xor(int v, int m) {
  if (m == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // quad_perm [1, 0, 3, 2]
  if (m == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm [2, 3, 0, 1]
  if (m == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return (int)(__lane_id() < 32 ? r[1] : r[0]);
  }
  return __shfl_xor(v, m);
}
__device__ __forceinline__ float lane_xor(float v, int m) { return __int_as_float(lane_xor(__float_as_int(v), m)); }
__device__ __forceinline__ double lane_xor(double v, int m) {
  return __hiloint2double(lane_xor(__double2hiint(v), m), lane_xor(__double2loint(v), m));
}

// A lane pair per node (one lane per species, partner at lane ^ XOR): both
// lanes hold the node's species densities; the seven evaluations are split
// four / three between the lanes and the results swapped, so both lanes end
// with identical tau values.
template <typename T, int XOR>
__device__ __forceinline__ void relaxation_times_pair(const RelaxConsts& c, int j, int s, T rho_a, T rho_b,
                                                      T& tau_s, T& tau_d, T& tau_q, bool tb) {
  if (c.bgk) {
    tau_s = tau_d = tau_q = T(c.tau_bgk);
    return;
  }
  const NodeGas<T> g = node_gas<T>(c, rho_a, rho_b);
  if (c.mfp_off) {
    taus_from_psi<T>(c, g, T(1), T(1), T(1), g.k * g.lam, T(0), tau_s, tau_d, tau_q);
    return;
  }
  const T y = T(j) + T(0.5);
  const T ay = y * g.il, ab = (T(c.height) - y) * g.il;
  // lane a: psi(y/l), psi((H-y)/l), psi(x_a y/l), psi(x_a (H-y)/l)
  // lane b: psi(x_b y/l), psi(x_b (H-y)/l), psi and h of H/l
  const T p0 = wall_psi_only(s ? g.xb * ay : ay, tb);
  const T p1 = wall_psi_only(s ? g.xb * ab : ab, tb);
  T p2, h2;
  wall_psi<T, true>(s ? T(c.height) * g.il : g.xa * ay, p2, h2, tb);
  T p3 = T(0);
  if (s == 0) p3 = wall_psi_only(g.xa * ab, tb);
  const T X = T(0.5) * (p0 + p1);           // lane a: Psi(y; l), lane b: Psi(y; l_b)
  const T Y = s ? p2 : T(0.5) * (p2 + p3);  // lane a: Psi(y; l_a), lane b: psi(H/l)
  const T Xo = lane_xor(X, XOR);
  const T Yo = lane_xor(Y, XOR);
  const T Zo = lane_xor(h2, XOR);
  const T pw = s ? Y : Yo;
  const T hw = s ? h2 : Zo;
  taus_from_psi<T>(c, g, s ? Xo : X, s ? Yo : Y, s ? X : Xo, T(0.5) * g.k * g.lam * pw, g.k * (T(1) - hw), tau_s,
                   tau_d, tau_q);
}

// MRT collision of one species in the moment space of Eq. (m):
// m' = m - S (m - m^eq), f' = M^-1 m'. m^eq is the moment vector of Eq. (feq)
// with the mixture velocity (ux, uy), in closed form:
// (rho, rho(2s-4) + 3 rho|u|^2, rho(4-3s) - 3 rho|u|^2, rho ux, -rho ux,
//  rho uy, -rho uy, rho(ux^2 - uy^2), rho ux uy).
// M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
//
// The populations may be deviations d = f - f0 from the rest equilibrium
// f0 = w_i alpha_i rho0 of a reference density rho0: M f0 is
// (rho0, rho0(2s-4), rho0(4-3s), 0, ..., 0), so the same update holds for d
// with the conserved part rho_c = rho - rho0 in place of rho in the terms
// linear in the density (first three moments), while the velocity terms keep
// the full density rho. For plain populations rho_c = rho.
template <typename T>
__device__ __forceinline__ void collide_species(T f[9], T rho_c, T rho, T ux, T uy, T s, T w_e, T w_eps, T w_d,
                                                T w_q, T w_s) {
  const T sa = (f[1] + f[2]) + (f[3] + f[4]);
  const T sd = (f[5] + f[6]) + (f[7] + f[8]);
  T e = T(-4) * f[0] - sa + T(2) * sd;
  T eps = T(4) * f[0] - T(2) * sa + sd;
  T jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  T qx = T(-2) * (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  T jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  T qy = T(-2) * (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  T pxx = (f[1] - f[2]) + (f[3] - f[4]);
  T pxy = (f[5] - f[6]) + (f[7] - f[8]);

  const T u2 = ux * ux + uy * uy;
  const T jxe = rho * ux, jye = rho * uy;
  e -= w_e * (e - (rho_c * (T(2) * s - T(4)) + T(3) * rho * u2));
  eps -= w_eps * (eps - (rho_c * (T(4) - T(3) * s) - T(3) * rho * u2));
  jx -= w_d * (jx - jxe);
  qx -= w_q * (qx + jxe);
  jy -= w_d * (jy - jye);
  qy -= w_q * (qy + jye);
  pxx -= w_s * (pxx - rho * (ux * ux - uy * uy));
  pxy -= w_s * (pxy - rho * ux * uy);

  if constexpr (std::is_same<T, float>::value) {
    // Single precision: the float values of 1/9, 1/6, 1/12 and 1/36 all lie
    // above the exact ratios (by 7e-9 to 3e-8 relative), and the scalings of
    // M^-1 would carry that error into every collision with the same sign:
    // the species density would grow by a factor 1 + 7e-9 per step and the
    // momentum by 1 + 3e-8, a drift that builds up over the tens of
    // thousands of steps a channel takes to settle. Here the scalings use
    // the ratio as the sum of two floats (the rest below float rounding),
    // and the rest population takes what the other eight leave of the
    // species density, so that the post-collision populations carry the
    // pre-collision density up to rounding of either sign.
    constexpr float h36 = 1.0f / 36.0f, l36 = float(1.0 / 36.0 - double(1.0f / 36.0f));
    constexpr float h9 = 1.0f / 9.0f, l9 = float(1.0 / 9.0 - double(1.0f / 9.0f));
    constexpr float h6 = 1.0f / 6.0f, l6 = float(1.0 / 6.0 - double(1.0f / 6.0f));
    constexpr float h12 = 1.0f / 12.0f, l12 = float(1.0 / 12.0 - double(1.0f / 12.0f));
    const T a0 = __builtin_fmaf(rho_c, h9, rho_c * l9);
    const T a1 = __builtin_fmaf(e, h36, e * l36);
    const T a2 = __builtin_fmaf(eps, h36, eps * l36);
    const T a3 = __builtin_fmaf(jx, h6, jx * l6);
    const T a4 = __builtin_fmaf(qx, h12, qx * l12);
    const T a5 = __builtin_fmaf(jy, h6, jy * l6);
    const T a6 = __builtin_fmaf(qy, h12, qy * l12);
    const T a7 = pxx * T(0.25);
    const T a8 = pxy * T(0.25);
    const T axis = a0 - a1 - T(2) * a2;
    const T diag = a0 + T(2) * a1 + a2;
    f[1] = axis + a3 - T(2) * a4 + a7;
    f[2] = axis + a5 - T(2) * a6 - a7;
    f[3] = axis - a3 + T(2) * a4 + a7;
    f[4] = axis - a5 + T(2) * a6 - a7;
    f[5] = diag + a3 + a4 + a5 + a6 + a8;
    f[6] = diag - a3 - a4 + a5 + a6 - a8;
    f[7] = diag - a3 - a4 - a5 - a6 + a8;
    f[8] = diag + a3 + a4 - a5 - a6 - a8;
    f[0] = rho_c - (((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
  } else {
    const T a0 = rho_c * T(1.0 / 9.0);
    const T a1 = e * T(1.0 / 36.0);
    const T a2 = eps * T(1.0 / 36.0);
    const T a3 = jx * T(1.0 / 6.0);
    const T a4 = qx * T(1.0 / 12.0);
    const T a5 = jy * T(1.0 / 6.0);
    const T a6 = qy * T(1.0 / 12.0);
    const T a7 = pxx * T(0.25);
    const T a8 = pxy * T(0.25);
    const T axis = a0 - a1 - T(2) * a2;
    const T diag = a0 + T(2) * a1 + a2;
    f[0] = a0 - T(4) * a1 + T(4) * a2;
    f[1] = axis + a3 - T(2) * a4 + a7;
    f[2] = axis + a5 - T(2) * a6 - a7;
    f[3] = axis - a3 + T(2) * a4 + a7;
    f[4] = axis - a5 + T(2) * a6 - a7;
    f[5] = diag + a3 + a4 + a5 + a6 + a8;
    f[6] = diag - a3 - a4 + a5 + a6 - a8;
    f[7] = diag - a3 - a4 - a5 - a6 + a8;
    f[8] = diag + a3 + a4 - a5 - a6 - a8;
  }
}

// Diffuse-bounce-back at a wall node (Eqs. (bot), (bot2); R12): from the
// node's own leaving post-collision populations l0 (on the wall normal) and
// l1, l2 (the two diagonals), with F = l0 + l1 + l2, the returning ones are
// r feq + (1 - r) l_opposite with the wall equilibrium holding the shares
// 2/3, 1/6, 1/6 of F: v0 = r (2/3) F + (1 - r) l0, v1 = r F/6 + (1 - r) l1,
// v2 = r F/6 + (1 - r) l2, so that v0 + v1 + v2 = F. In single precision the
// float values of 2/3 and 1/6 lie above the exact ratios (3e-8 relative),
// which would let every wall node gain mass at every step; there the axis
// value takes what the diagonals leave of F instead.
template <typename T>
__device__ __forceinline__ void dbb_shares(T r, T l0, T l1, T l2, T& v0, T& v1, T& v2) {
  const T q = T(1) - r;
  const T F = (l0 + l1) + l2;
  v1 = r * (F * T(1.0 / 6.0)) + q * l1;
  v2 = r * (F * T(1.0 / 6.0)) + q * l2;
  if constexpr (std::is_same<T, float>::value)
    v0 = (F - v1) - v2;
  else
    v0 = r * (T(2.0 / 3.0) * F) + q * l0;
}

}  // namespace lbsep
