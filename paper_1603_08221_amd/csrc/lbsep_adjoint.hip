// Discrete adjoint (reverse mode) of the FP64 channel step, hand-written for
// gfx950.
//
// The forward step maps the pre-collision populations f(t) to f(t+1):
//   C : MRT collision of Sec. 3.1 (Eqs. (MR), (m), (S), (feq)) with the
//       relaxation times of Eqs. (taos), (EQFrsp), (taoq) recomputed from the
//       node's own densities (the mean-free-path wall function psi of
//       Eq. (EQFrb) included),
//   P : streaming of Eq. (MRT) with the DBB walls of Eqs. (bot), (bot2),
//   E : the extrapolation-correction inlet/outlet of Eqs. (rho1), (rho2).
// The adjoint step maps lam(t+1) = dJ/df(t+1) to lam(t) = (E P C)'^T lam(t+1)
// and accumulates the explicit partial derivatives of the step with respect to
// theta and C_in (through the inlet densities of Eq. (rho2)) and the DBB
// coefficient r. It is the derivative of the same map the forward kernels
// compute, written out by hand:
//   k_adj_post   recomputes C(f(t)) (needed by P, E and the r derivative),
//   k_adj_ends   reverses E on the inlet and outlet columns (whole-column
//                coupling through kappa) and the rho_bc dependence,
//   k_adj_main   reverses P (push of the adjoint, DBB transposed) and then C
//                node by node,
//   k_adj_params sums the per-block parameter partials in a fixed order.
// Seeds: dCL/df(T) of Eq. (CL) at the column of the smallest C_l (R16), and
// the initial state's dependence on theta and C_in (R18).
//
// Populations and adjoints use the dense FP64 layout [2][9][ny][nx] of
// lbsep_get_populations.

// this unit's own copy of the coefficient tables (see e1_table.h)
#define LBSEP_TBL(name) adj_##name

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "lbsep.h"
#include "lbsep_device.h"
#include "lbsep_view.h"

namespace lbsep {
namespace {

constexpr int kAT = 256;  // threads per block
constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr double kCs2 = 1.0 / 3.0;

struct AdjParams {
  RelaxConsts rc;
  int nx, ny;
  unsigned flags;
  double r;
  double rho_bc[2][2];
  double drho_in[2][2];  // [theta, C_in][species]: d rho_bc(inlet) / d parameter
  double inv_cl_in, cl_in;
};

__device__ __forceinline__ long long didx(const AdjParams& ap, int s, int i, int j, int x) {
  return ((long long)(s * 9 + i) * ap.ny + j) * ap.nx + x;
}

// E1(a) for a > 0 (A&S 5.1.11 below 1; e^-a G(a) / a above, with G the octave
// Chebyshev series of the wall function's series form; 0 beyond the table,
// where E1 is below 1e-29).
__device__ double e1_dev(double a) {
  if (a <= 1.0) {
    double p = 1.0, s = 0.0;
    for (int k = 1; k <= 24; ++k) {
      p *= -a / k;
      s += p / k;
    }
    return -LBSEP_EULER_GAMMA - log(a) - s;
  }
  const int seg = ilogb(a);
  if (seg >= LBSEP_E1_F64_NSEG) return 0.0;
  const double t = ldexp(a, 1 - seg) - 3.0;
  const double t2 = t + t;
  double b1 = 0.0, b2 = 0.0;
  for (int k = LBSEP_E1_F64_DEG; k >= 1; --k) {
    const double b0 = LBSEP_TBL(lbsep_e1_cheb_f64)[seg][k] + t2 * b1 - b2;
    b2 = b1;
    b1 = b0;
  }
  const double g = LBSEP_TBL(lbsep_e1_cheb_f64)[seg][0] + t * b1 - b2;
  return exp(-a) * g / a;
}

// Forward relaxation times (the same arithmetic as relaxation_times in the
// device header, so the same values) together with what their reverse needs:
// the mixture quantities and the wall-function values psi and h = psi' / 2 of
// the seven arguments, each evaluated once.
struct TauState {
  double ts, td, tq;
  NodeGas<double> g;
  double y, ay, ab, aw;
  double hay, hab, h1a, h2a, h1b, h2b, pw, hw;
  double psi_m, psi_a, psi_b;
};

__device__ TauState taus_fwd(const RelaxConsts& c, int j, double ra, double rb) {
  TauState o{};
  if (c.bgk) {
    o.ts = o.td = o.tq = c.tau_bgk;
    return o;
  }
  o.g = node_gas<double>(c, ra, rb);
  const NodeGas<double>& g = o.g;
  if (c.mfp_off) {
    o.psi_m = o.psi_a = o.psi_b = 1.0;
    taus_from_psi<double>(c, g, 1.0, 1.0, 1.0, g.k * g.lam, 0.0, o.ts, o.td, o.tq);
    return o;
  }
  const bool tb = c.psi_table != 0;
  o.y = double(j) + 0.5;
  o.ay = o.y * g.il;
  o.ab = (c.height - o.y) * g.il;
  double p1, p2;
  wall_psi<double, true>(o.ay, p1, o.hay, tb);
  wall_psi<double, true>(o.ab, p2, o.hab, tb);
  o.psi_m = 0.5 * (p1 + p2);
  wall_psi<double, true>(g.xa * o.ay, p1, o.h1a, tb);
  wall_psi<double, true>(g.xa * o.ab, p2, o.h2a, tb);
  o.psi_a = 0.5 * (p1 + p2);
  wall_psi<double, true>(g.xb * o.ay, p1, o.h1b, tb);
  wall_psi<double, true>(g.xb * o.ab, p2, o.h2b, tb);
  o.psi_b = 0.5 * (p1 + p2);
  o.aw = c.height * g.il;
  wall_psi<double, true>(o.aw, o.pw, o.hw, tb);
  taus_from_psi<double>(c, g, o.psi_m, o.psi_a, o.psi_b, 0.5 * g.k * g.lam * o.pw, g.k * (1.0 - o.hw), o.ts, o.td,
                        o.tq);
  return o;
}

// Reverse of taus_fwd: given the adjoints of (tau_s, tau_d, tau_q), add
// d/d(rho_a, rho_b) to (ga, gb).
__device__ void taus_rev(const RelaxConsts& c, const TauState& st, double ra, double rb, double bts, double btd,
                         double btq, double& ga, double& gb) {
  if (c.bgk) return;  // constant relaxation times
  const NodeGas<double>& g = st.g;
  const double inv_n = 1.0 / (ra * c.inv_m[0] + rb * c.inv_m[1]);
  const double xa = g.xa, xb = g.xb, mx = g.mx, lam = g.lam, k = g.k;
  const double pres = (1.0 / 3.0) * (c.s[0] * ra + c.s[1] * rb);
  double tt0, dtt0;
  if (c.mfp_off) {
    tt0 = k * lam;
    dtt0 = 0.0;
  } else {
    tt0 = 0.5 * k * lam * st.pw;
    dtt0 = k * (1.0 - st.hw);
  }
  const double psi_m = st.psi_m, psi_a = st.psi_a, psi_b = st.psi_b;
  const double sa = 1.0 / sqrt(psi_a) + 1.0 / sqrt(psi_b);
  const double q = c.dpref * lam / (mx * sa * sa);
  const double r0 = 1.0 / tt0;
  // tau_q = 1/2 + (3 r0 + tq_a tt0) / 16 + dtt0 (12 r0^2 + tq_b r0) / 16
  const double br0 = btq * (3.0 + dtt0 * (24.0 * r0 + c.tq_b)) / 16.0;
  double btt0 = btq * c.tq_a / 16.0 - br0 * r0 * r0;
  const double bdtt0 = btq * (12.0 * r0 * r0 + c.tq_b * r0) / 16.0;
  double bk = 0.0, blam = 0.0, bmx = 0.0, bil = 0.0, bxa = 0.0, bxb = 0.0;
  if (c.mfp_off) {
    bk += btt0 * lam;
    blam += btt0 * k;
  } else {
    bk += btt0 * 0.5 * lam * st.pw + bdtt0 * (1.0 - st.hw);
    blam += btt0 * 0.5 * k * st.pw;
    const double bpw = btt0 * 0.5 * k * lam;
    const double bhw = -bdtt0 * k;
    const double baw = bpw * 2.0 * st.hw - bhw * e1_dev(st.aw);  // psi' = 2h, h' = -E1
    bil += baw * c.height;
  }
  // tau_d = 1/2 + q, q = dpref lam / (mx sa^2)
  blam += btd * q / lam;
  bmx += -btd * q / mx;
  const double bsa = -2.0 * btd * q / sa;
  const double bpsa = bsa * (-0.5) / (psi_a * sqrt(psi_a));
  const double bpsb = bsa * (-0.5) / (psi_b * sqrt(psi_b));
  // tau_s = 1/2 + lam psi_m k
  blam += bts * psi_m * k;
  bk += bts * lam * psi_m;
  if (!c.mfp_off) {
    const double bpsm = bts * lam * k;
    double bay = bpsm * st.hay, bab = bpsm * st.hab;  // d psi_m / d ay = psi'(ay) / 2 = h(ay)
    // psi_a = (psi(xa ay) + psi(xa ab)) / 2
    const double z1a = bpsa * st.h1a, z2a = bpsa * st.h2a;
    bxa += z1a * st.ay + z2a * st.ab;
    bay += z1a * xa;
    bab += z2a * xa;
    const double z1b = bpsb * st.h1b, z2b = bpsb * st.h2b;
    bxb += z1b * st.ay + z2b * st.ab;
    bay += z1b * xb;
    bab += z2b * xb;
    bil += bay * st.y + bab * (c.height - st.y);
  }
  // k = kpref / sqrt(mx)
  bmx += bk * (-0.5) * k / mx;
  // lam = lam_p / P, il = P / lam_p
  double bp = -blam * lam / pres + bil * c.inv_lam_p;
  ga += bp * c.s[0] / 3.0;
  gb += bp * c.s[1] / 3.0;
  // mx = (ra + rb) / n, xa = na / n, xb = nb / n
  ga += bmx * inv_n;
  gb += bmx * inv_n;
  double bn = -bmx * mx * inv_n - (bxa * xa + bxb * xb) * inv_n;
  double bna = bxa * inv_n + bn, bnb = bxb * inv_n + bn;
  ga += bna * c.inv_m[0];
  gb += bnb * c.inv_m[1];
}

// Collision of both species at one node (the forward of the device header).
__device__ void collide_fwd(const RelaxConsts& rc, int j, const double fa[9], const double fb[9], double oa[9],
                            double ob[9]) {
  double ra = 0, rb = 0, jxa = 0, jya = 0, jxb = 0, jyb = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    ra += fa[i];
    rb += fb[i];
    jxa += kCx[i] * fa[i];
    jya += kCy[i] * fa[i];
    jxb += kCx[i] * fb[i];
    jyb += kCy[i] * fb[i];
  }
  const double inv = 1.0 / (ra + rb);
  const double ux = (jxa + jxb) * inv, uy = (jya + jyb) * inv;
  const TauState t = taus_fwd(rc, j, ra, rb);
  double we, weps;
  const double ws = 1.0 / t.ts;
  if (rc.bgk) {
    we = weps = ws;
  } else {
    we = 1.0 / 1.1;
    weps = 1.0 / 1.2;
  }
  const double wd = 1.0 / t.td, wq = 1.0 / t.tq;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    oa[i] = fa[i];
    ob[i] = fb[i];
  }
  collide_species<double>(oa, ra, ra, ux, uy, rc.s[0], we, weps, wd, wq, ws);
  collide_species<double>(ob, rb, rb, ux, uy, rc.s[1], we, weps, wd, wq, ws);
}

// M f (Eq. (m)), and M^T v.
__device__ __forceinline__ void mul_m(const double f[9], double m[9]) {
  m[0] = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
  m[1] = -4 * f[0] - f[1] - f[2] - f[3] - f[4] + 2 * (f[5] + f[6] + f[7] + f[8]);
  m[2] = 4 * f[0] - 2 * (f[1] + f[2] + f[3] + f[4]) + f[5] + f[6] + f[7] + f[8];
  m[3] = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  m[4] = -2 * f[1] + 2 * f[3] + f[5] - f[6] - f[7] + f[8];
  m[5] = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  m[6] = -2 * f[2] + 2 * f[4] + f[5] + f[6] - f[7] - f[8];
  m[7] = f[1] - f[2] + f[3] - f[4];
  m[8] = f[5] - f[6] + f[7] - f[8];
}

__device__ __forceinline__ void mul_mt(const double v[9], double f[9]) {
  f[0] = v[0] - 4 * v[1] + 4 * v[2];
  f[1] = v[0] - v[1] - 2 * v[2] + v[3] - 2 * v[4] + v[7];
  f[2] = v[0] - v[1] - 2 * v[2] + v[5] - 2 * v[6] - v[7];
  f[3] = v[0] - v[1] - 2 * v[2] - v[3] + 2 * v[4] + v[7];
  f[4] = v[0] - v[1] - 2 * v[2] - v[5] + 2 * v[6] - v[7];
  f[5] = v[0] + 2 * v[1] + v[2] + v[3] + v[4] + v[5] + v[6] + v[8];
  f[6] = v[0] + 2 * v[1] + v[2] - v[3] - v[4] + v[5] + v[6] - v[8];
  f[7] = v[0] + 2 * v[1] + v[2] - v[3] - v[4] - v[5] - v[6] + v[8];
  f[8] = v[0] + 2 * v[1] + v[2] + v[3] + v[4] - v[5] - v[6] - v[8];
}

// Reverse of the collision at one node: f (pre-collision, both species) and
// g = dJ/df' (both species) -> out = dJ/df.
__device__ void collide_rev(const RelaxConsts& rc, int j, const double fa[9], const double fb[9], const double ga[9],
                            const double gb[9], double oa[9], double ob[9]) {
  const double* f[2] = {fa, fb};
  const double* g[2] = {ga, gb};
  double* o[2] = {oa, ob};
  double rho[2], jx[2], jy[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    rho[s] = jx[s] = jy[s] = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      rho[s] += f[s][i];
      jx[s] += kCx[i] * f[s][i];
      jy[s] += kCy[i] * f[s][i];
    }
  }
  const double rt = rho[0] + rho[1];
  const double ux = (jx[0] + jx[1]) / rt, uy = (jy[0] + jy[1]) / rt;
  const double u2 = ux * ux + uy * uy;
  const TauState t = taus_fwd(rc, j, rho[0], rho[1]);
  double w[9];
  if (rc.bgk) {
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = 1.0 / t.ts;
  } else {
    w[0] = 1.0;
    w[1] = 1.0 / 1.1;
    w[2] = 1.0 / 1.2;
    w[3] = w[5] = 1.0 / t.td;
    w[4] = w[6] = 1.0 / t.tq;
    w[7] = w[8] = 1.0 / t.ts;
  }
  // M^-1 = M^T diag(d): M^-T g = diag(d) M g
  const double d[9] = {1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 6, 1.0 / 12, 1.0 / 6, 1.0 / 12, 1.0 / 4, 1.0 / 4};
  double bw[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double bux = 0.0, buy = 0.0, brho[2] = {0.0, 0.0};
  double bm[2][9];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double sv = rc.s[s];
    double m[9], mg[9];
    mul_m(f[s], m);
    mul_m(g[s], mg);
    const double r = rho[s];
    const double meq[9] = {r,
                           r * (2 * sv - 4) + 3 * r * u2,
                           r * (4 - 3 * sv) - 3 * r * u2,
                           r * ux,
                           -r * ux,
                           r * uy,
                           -r * uy,
                           r * (ux * ux - uy * uy),
                           r * ux * uy};
    double be[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double bmp = d[k] * mg[k];  // adjoint of m'_k
      bm[s][k] = (1.0 - w[k]) * bmp;
      be[k] = w[k] * bmp;
      bw[k] += (meq[k] - m[k]) * bmp;
    }
    brho[s] += be[0] + be[1] * (2 * sv - 4 + 3 * u2) + be[2] * (4 - 3 * sv - 3 * u2) + ux * (be[3] - be[4]) +
               uy * (be[5] - be[6]) + (ux * ux - uy * uy) * be[7] + ux * uy * be[8];
    bux += r * (6 * ux * (be[1] - be[2]) + (be[3] - be[4]) + 2 * ux * be[7] + uy * be[8]);
    buy += r * (6 * uy * (be[1] - be[2]) + (be[5] - be[6]) - 2 * uy * be[7] + ux * be[8]);
  }
  // relaxation rates -> relaxation times
  double bts, btd, btq;
  if (rc.bgk) {
    bts = btd = btq = 0.0;
  } else {
    btd = -(bw[3] + bw[5]) * w[3] * w[3];
    btq = -(bw[4] + bw[6]) * w[4] * w[4];
    bts = -(bw[7] + bw[8]) * w[7] * w[7];
  }
  taus_rev(rc, t, rho[0], rho[1], bts, btd, btq, brho[0], brho[1]);
  // u = (jx_a + jx_b) / rho
  const double bjx = bux / rt, bjy = buy / rt;
  const double brt = -(bux * ux + buy * uy) / rt;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    bm[s][0] += brho[s] + brt;
    bm[s][3] += bjx;
    bm[s][5] += bjy;
    mul_mt(bm[s], o[s]);
  }
}

// ---- kernels ------------------------------------------------------------------

__global__ __launch_bounds__(kAT) void k_adj_post(AdjParams ap, const double* __restrict__ ft,
                                                  double* __restrict__ fpost) {
  const long long n = (long long)ap.nx * ap.ny;
  const long long e = (long long)blockIdx.x * kAT + threadIdx.x;
  if (e >= n) return;
  const int j = int(e / ap.nx), x = int(e - (long long)j * ap.nx);
  double fa[9], fb[9], oa[9], ob[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    fa[i] = ft[didx(ap, 0, i, j, x)];
    fb[i] = ft[didx(ap, 1, i, j, x)];
  }
  collide_fwd(ap.rc, j, fa, fb, oa, ob);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    fpost[didx(ap, 0, i, j, x)] = oa[i];
    fpost[didx(ap, 1, i, j, x)] = ob[i];
  }
}

// Streamed and DBB-closed populations of species s at (x, j) (the inputs of
// the inlet/outlet closure), from the post-collision state.
__device__ void pulled(const AdjParams& ap, const double* __restrict__ fpost, int s, int x, int j, double out[9]) {
  const bool px = ap.flags & LBSEP_PERIODIC_X, py = ap.flags & LBSEP_PERIODIC_Y;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int xs = x - kCx[i], ys = j - kCy[i];
    if (xs < 0 || xs >= ap.nx) xs = px ? (xs + ap.nx) % ap.nx : (xs < 0 ? 0 : ap.nx - 1);  // unknown dirs: replaced
    if (ys < 0 || ys >= ap.ny) ys = py ? (ys + ap.ny) % ap.ny : j;                           // replaced by DBB
    out[i] = fpost[didx(ap, s, i, ys, xs)];
  }
  if (!py && (j == 0 || j == ap.ny - 1)) {
    const bool bot = j == 0;
    const int l0 = bot ? 4 : 2, l1 = bot ? 7 : 5, l2 = bot ? 8 : 6;
    const double a = fpost[didx(ap, s, l0, j, x)], b = fpost[didx(ap, s, l1, j, x)], c = fpost[didx(ap, s, l2, j, x)];
    const double F = (a + b) + c;
    const double v0 = ap.r * (2.0 / 3.0) * F + (1.0 - ap.r) * a;
    const double v1 = ap.r * F / 6.0 + (1.0 - ap.r) * b;
    const double v2 = ap.r * F / 6.0 + (1.0 - ap.r) * c;
    if (bot) {  // constant indices keep out in registers
      out[2] = v0;
      out[5] = v1;
      out[6] = v2;
    } else {
      out[4] = v0;
      out[7] = v1;
      out[8] = v2;
    }
  }
}

// Block sum in a fixed order (wavefront trees, then the four wavefront results
// in order); every thread gets it. sh: at least four doubles of shared memory.
__device__ double block_sum_d(double v, double* sh) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();  // sh may still be read from a previous call
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Block sums of two values per thread in a fixed order: wavefront trees
// (shuffles), then the four wavefront results in order. Every thread gets both.
__device__ void block_sum2(double& u, double& v, double (*sh)[kAT / 64]) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    u += __shfl_xor(u, off);
    v += __shfl_xor(v, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = u;
    sh[1][w] = v;
  }
  __syncthreads();
  u = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
  v = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
}

// Reverse of the inlet/outlet closure. Block (e, s): end e (0 inlet, 1 outlet),
// species s. Writes lamP[e][s][c][i][j] for c = 0 (boundary column), 1, 2
// (first and second inner layer: the adjoint passing through unchanged plus the
// closure's dependence on them) and the rho_bc partials part[e][s][0..1].
// Two passes over the column: the sums S = sum_j rho'(j) and
// kappa-bar = sum_j A(j) rho'(j) / rho_node(j) (neither needs kappa), then the
// per-row adjoints. With at most 256 rows each thread keeps its row's pulled
// populations in registers between the passes.
__global__ __launch_bounds__(kAT) void k_adj_ends(AdjParams ap, const double* __restrict__ fpost,
                                                  const double* __restrict__ lam_next, double* __restrict__ lamP,
                                                  double* __restrict__ part) {
  static_assert(kAT == 256, "block_sum2 assumes four wavefronts");
  __shared__ double sh[2][kAT / 64];
  const int e = blockIdx.x >> 1, s = blockIdx.x & 1;
  const int col = e ? ap.nx - 1 : 0, l1 = e ? ap.nx - 2 : 1, l2 = e ? ap.nx - 3 : 2;
  const int ny = ap.ny;
  double* out = lamP + (long long)(e * 2 + s) * 3 * 9 * ny;  // [c][i][j]
  auto unknown = [&](int i) { return e == 0 ? kCx[i] == 1 : kCx[i] == -1; };
  // row j's pulled populations of the end column and the two inner layers
  auto load = [&](int j, double g0[9], double g1[9], double g2[9]) {
    pulled(ap, fpost, s, col, j, g0);
    pulled(ap, fpost, s, l1, j, g1);
    pulled(ap, fpost, s, l2, j, g2);
  };
  // pass 1 of row j: its shares of S and kappa-bar
  auto shares = [&](int j, const double g0[9], const double g1[9], const double g2[9], double& accS,
                    double& accK) {
    double r1 = 0, r2 = 0, rn = 0, A = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const double gh = unknown(i) ? 2.0 * g1[i] - g2[i] : g0[i];
      r1 += g1[i];
      r2 += g2[i];
      rn += gh;
      A += lam_next[didx(ap, s, i, j, col)] * gh;
    }
    const double rp = 2.0 * r1 - r2;
    accS += rp;
    accK += A * rp / rn;
  };
  // pass 2 of row j: the adjoints of the three columns' pulled populations
  auto adjoints = [&](int j, const double g0[9], const double g1[9], const double g2[9], double kappa, double S,
                      double kbar) {
    double gh[9], lE[9];
    double r1 = 0, r2 = 0, rn = 0, A = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      gh[i] = unknown(i) ? 2.0 * g1[i] - g2[i] : g0[i];
      lE[i] = lam_next[didx(ap, s, i, j, col)];
      r1 += g1[i];
      r2 += g2[i];
      rn += gh[i];
      A += lE[i] * gh[i];
    }
    const double rp = 2.0 * r1 - r2;
    const double scale = kappa * rp / rn;
    const double brp = A * kappa / rn - kbar * kappa / S;  // d/d rho'(j), with d kappa / d rho'(j) = -kappa / S
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const double bgh = lE[i] * scale - A * scale / rn;
      double b0 = 0.0, b1 = lam_next[didx(ap, s, i, j, l1)] + 2.0 * brp,
             b2 = lam_next[didx(ap, s, i, j, l2)] - brp;
      if (unknown(i)) {
        b1 += 2.0 * bgh;
        b2 -= bgh;
      } else {
        b0 = bgh;
      }
      out[(0 * 9 + i) * ny + j] = b0;
      out[(1 * 9 + i) * ny + j] = b1;
      out[(2 * 9 + i) * ny + j] = b2;
    }
  };
  double accS = 0.0, accK = 0.0;
  if (ny <= kAT) {
    // one row per thread: the pulled values stay in registers for pass 2
    const int j = threadIdx.x;
    double g0[9], g1[9], g2[9];
    if (j < ny) {
      load(j, g0, g1, g2);
      shares(j, g0, g1, g2, accS, accK);
    }
    block_sum2(accS, accK, sh);
    const double kappa = double(ny) * ap.rho_bc[e][s] / accS;
    if (j < ny) adjoints(j, g0, g1, g2, kappa, accS, accK);
  } else {
    for (int j = threadIdx.x; j < ny; j += kAT) {
      double g0[9], g1[9], g2[9];
      load(j, g0, g1, g2);
      shares(j, g0, g1, g2, accS, accK);
    }
    block_sum2(accS, accK, sh);
    const double kappa = double(ny) * ap.rho_bc[e][s] / accS;
    for (int j = threadIdx.x; j < ny; j += kAT) {
      double g0[9], g1[9], g2[9];
      load(j, g0, g1, g2);
      adjoints(j, g0, g1, g2, kappa, accS, accK);
    }
  }
  if (threadIdx.x == 0) {
    // d J / d rho_bc = kappa-bar N / S; only the inlet densities depend on (theta, C_in)
    const double kappa_bar = accK, S = accS;
    const double brho = kappa_bar * double(ny) / S;
    part[(e * 2 + s) * 2 + 0] = e == 0 ? brho * ap.drho_in[0][s] : 0.0;
    part[(e * 2 + s) * 2 + 1] = e == 0 ? brho * ap.drho_in[1][s] : 0.0;
  }
}

// Adjoint of P at destination (x, j), direction i: lam_next, or the closure's
// reverse on the six end columns.
__device__ __forceinline__ double lam_p(const AdjParams& ap, const double* __restrict__ lam_next,
                                        const double* __restrict__ lamP, int s, int i, int j, int x) {
  if (!(ap.flags & LBSEP_PERIODIC_X)) {
    int e = -1, c = 0;
    if (x <= 2) {
      e = 0;
      c = x;
    } else if (x >= ap.nx - 3) {
      e = 1;
      c = ap.nx - 1 - x;
    }
    if (e >= 0) return lamP[((long long)((e * 2 + s) * 3 + c) * 9 + i) * ap.ny + j];
  }
  return lam_next[didx(ap, s, i, j, x)];
}

__global__ __launch_bounds__(kAT) void k_adj_main(AdjParams ap, const double* __restrict__ ft,
                                                  const double* __restrict__ fpost,
                                                  const double* __restrict__ lam_next,
                                                  const double* __restrict__ lamP, double* __restrict__ lam_out,
                                                  double* __restrict__ part_r) {
  __shared__ double sh[kAT];
  const long long n = (long long)ap.nx * ap.ny;
  const long long e = (long long)blockIdx.x * kAT + threadIdx.x;
  double dr = 0.0;
  if (e < n) {
    const int j = int(e / ap.nx), x = int(e - (long long)j * ap.nx);
    const bool px = ap.flags & LBSEP_PERIODIC_X, py = ap.flags & LBSEP_PERIODIC_Y;
    double g[2][9];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        int xd = x + kCx[i], yd = j + kCy[i];
        double v = 0.0;
        bool through_wall = false;
        if (yd < 0 || yd >= ap.ny) {
          if (py)
            yd = (yd + ap.ny) % ap.ny;
          else
            through_wall = true;
        }
        if (!through_wall) {
          bool in = true;
          if (xd < 0 || xd >= ap.nx) {
            if (px)
              xd = (xd + ap.nx) % ap.nx;
            else
              in = false;  // leaves through an end: replaced there by the closure
          }
          if (in) v = lam_p(ap, lam_next, lamP, s, i, yd, xd);
        }
        g[s][i] = v;
      }
      if (!py && (j == 0 || j == ap.ny - 1)) {
        // DBB at this node: returning k = r share_k F + (1 - r) f'_leaving(k)
        const bool bot = j == 0;
        const double share[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
        double lr[3], fl[3], F = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int rq = bot ? (q == 0 ? 2 : q == 1 ? 5 : 6) : (q == 0 ? 4 : q == 1 ? 7 : 8);
          const int lq = bot ? (q == 0 ? 4 : q == 1 ? 7 : 8) : (q == 0 ? 2 : q == 1 ? 5 : 6);
          lr[q] = lam_p(ap, lam_next, lamP, s, rq, j, x);
          fl[q] = fpost[didx(ap, s, lq, j, x)];
          F += fl[q];
        }
        double sl = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) sl += lr[q] * share[q];
        double add[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          add[q] = ap.r * sl + (1.0 - ap.r) * lr[q];
          dr += lr[q] * (share[q] * F - fl[q]);
        }
        if (bot) {  // constant indices keep g in registers
          g[s][4] += add[0];
          g[s][7] += add[1];
          g[s][8] += add[2];
        } else {
          g[s][2] += add[0];
          g[s][5] += add[1];
          g[s][6] += add[2];
        }
      }
    }
    double fa[9], fb[9], oa[9], ob[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      fa[i] = ft[didx(ap, 0, i, j, x)];
      fb[i] = ft[didx(ap, 1, i, j, x)];
    }
    collide_rev(ap.rc, j, fa, fb, g[0], g[1], oa, ob);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      lam_out[didx(ap, 0, i, j, x)] = oa[i];
      lam_out[didx(ap, 1, i, j, x)] = ob[i];
    }
  }
  const double t = block_sum_d(dr, sh);
  if (threadIdx.x == 0) part_r[blockIdx.x] = t;
}

// dparams[0..2] += (theta, C_in, r) partials, summed in a fixed order.
__global__ void k_adj_params(const double* __restrict__ part_ends, const double* __restrict__ part_r, int nr,
                             const double* __restrict__ part_cols, int ncols, double* __restrict__ dparams) {
  __shared__ double sh[kAT];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nr; k += kAT) c += part_r[k];
  for (int k = threadIdx.x; k < ncols; k += kAT) {
    a += part_cols[2 * k];
    b += part_cols[2 * k + 1];
  }
  if (part_ends && threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) {
      a += part_ends[2 * k];
      b += part_ends[2 * k + 1];
    }
  a = block_sum_d(a, sh);
  b = block_sum_d(b, sh);
  c = block_sum_d(c, sh);
  if (threadIdx.x == 0) {
    dparams[0] += a;
    dparams[1] += b;
    dparams[2] += c;
  }
}

__global__ void k_fill(double* p, long long n, double v) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    p[k] = v;
}

// Column sums N_a(x), N_b(x) of the state (Eq. (C) over the cross-section).
__global__ void k_adj_colsum(AdjParams ap, const double* __restrict__ f, double* __restrict__ cols) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ap.nx) return;
  double na = 0.0, nb = 0.0;
  for (int j = 0; j < ap.ny; ++j)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      na += f[didx(ap, 0, i, j, x)];
      nb += f[didx(ap, 1, i, j, x)];
    }
  cols[2 * x] = na * ap.rc.inv_m[0];
  cols[2 * x + 1] = nb * ap.rc.inv_m[1];
}

// Seed of CL = (C_in - C_l(x*)) / C_in at x* = argmin C_l (first on ties):
// lam(s, i, x*, j) = -(1/C_in) dC_l(x*)/d rho_s; dparams[1] += C_l(x*) / C_in^2.
__global__ void k_adj_seed(AdjParams ap, const double* __restrict__ cols, double* __restrict__ lam,
                           double* __restrict__ dparams) {
  __shared__ double bv[kAT];
  __shared__ int bi[kAT];
  double best = INFINITY;
  int arg = 0x7fffffff;
  for (int x = threadIdx.x; x < ap.nx; x += kAT) {
    const double c = cols[2 * x] / (cols[2 * x] + cols[2 * x + 1]);
    if (c < best || (c == best && x < arg)) {
      best = c;
      arg = x;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = arg;
  __syncthreads();
  for (int o = kAT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double c = bv[threadIdx.x + o];
      const int a = bi[threadIdx.x + o];
      if (c < bv[threadIdx.x] || (c == bv[threadIdx.x] && a < bi[threadIdx.x])) {
        bv[threadIdx.x] = c;
        bi[threadIdx.x] = a;
      }
    }
    __syncthreads();
  }
  int xs = bi[0];
  if (xs < 0 || xs >= ap.nx) xs = 0;  // no finite C_l: the seed is then meaningless but in range
  const double na = cols[2 * xs], nb = cols[2 * xs + 1];
  const double tot = na + nb;
  const double da = ap.rc.inv_m[0] * nb / (tot * tot);   // dC_l / d rho_a
  const double db = -ap.rc.inv_m[1] * na / (tot * tot);  // dC_l / d rho_b
  for (int k = threadIdx.x; k < 9 * ap.ny; k += kAT) {
    const int i = k / ap.ny, j = k - i * ap.ny;
    lam[didx(ap, 0, i, j, xs)] = -da * ap.inv_cl_in;
    lam[didx(ap, 1, i, j, xs)] = -db * ap.inv_cl_in;
  }
  if (threadIdx.x == 0) dparams[1] += (na / tot) * ap.inv_cl_in * ap.inv_cl_in;
}

// Initial state of R18: f0(s, i, x, j) = w_i alpha_si rho_s(x) with the
// pressure and C_l linear in x; per-column partials of lam0 . d f0 / d(theta, C_in).
__global__ void k_adj_initial(AdjParams ap, const double* __restrict__ lam0, double* __restrict__ cols) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ap.nx) return;
  const double wv[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const double frac = ap.nx > 1 ? double(x) / double(ap.nx - 1) : 0.0;
  const double pout = kCs2;
  const double pin = ap.rho_bc[0][0] * ap.rc.s[0] * kCs2 / ap.cl_in;  // theta P_out
  const double pres = pin + (pout - pin) * frac;
  const double cout = ap.rho_bc[1][0] * ap.rc.s[0] * kCs2 / pout;
  const double c = ap.cl_in + (cout - ap.cl_in) * frac;
  // d rho_s / d theta and d rho_s / d C_in
  const double dp_dth = pout * (1.0 - frac), dc_dc = 1.0 - frac;
  const double dra[2] = {c * dp_dth / (ap.rc.s[0] * kCs2), dc_dc * pres / (ap.rc.s[0] * kCs2)};
  const double drb[2] = {(1.0 - c) * dp_dth / (ap.rc.s[1] * kCs2), -dc_dc * pres / (ap.rc.s[1] * kCs2)};
  double la = 0.0, lb = 0.0;  // sum_{i, j} lam0 w_i alpha_si
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double sv = ap.rc.s[s];
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const double alpha = i == 0 ? (9.0 - 5.0 * sv) / 4.0 : sv;
      double sj = 0.0;
      for (int j = 0; j < ap.ny; ++j) sj += lam0[didx(ap, s, i, j, x)];
      acc += wv[i] * alpha * sj;
    }
    if (s == 0)
      la = acc;
    else
      lb = acc;
  }
  cols[2 * x] = la * dra[0] + lb * drb[0];
  cols[2 * x + 1] = la * dra[1] + lb * drb[1];
}

// ---- host --------------------------------------------------------------------

struct AdjLayout {
  size_t fpost, lamP, part_ends, part_r, cols, total;
  int nblocks;
};

// with_post: room for the recomputed post-collision state C(f_t) (a caller
// workspace always has it; the fixed scratch only when the call needs it)
AdjLayout adj_layout(const lbsep_params* p, bool with_post = true) {
  AdjLayout L{};
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  const long long n = (long long)p->nx * p->ny;
  L.nblocks = (int)((n + kAT - 1) / kAT);
  size_t off = 0;
  L.fpost = off;
  if (with_post) off += up(18ull * n * sizeof(double));
  L.lamP = off;
  off += up(2ull * 2 * 3 * 9 * p->ny * sizeof(double));
  L.part_ends = off;
  off += up(8 * sizeof(double));
  L.part_r = off;
  off += up((size_t)L.nblocks * sizeof(double));
  L.cols = off;
  off += up(2ull * p->nx * sizeof(double));
  L.total = off;
  return L;
}

// The channel's parameters and stream as the adjoint kernels take them.
int adj_params(const lbsep_channel* ch, AdjParams& ap, hipStream_t& st, lbsep_params* pp = nullptr) {
  ChannelView v;
  if (!channel_view(ch, &v)) return set_error(LBSEP_EINVAL, "channel is NULL");
  if (pp) *pp = v.p;
  ap.rc = v.rc;
  ap.nx = v.p.nx;
  ap.ny = v.p.ny;
  ap.flags = v.p.flags;
  ap.r = v.p.dbb_r;
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int s = 0; s < 2; ++s) ap.rho_bc[e][s] = v.rho_bc[e][s];
  const double pout = kCs2, pin = v.p.theta * pout;
  ap.drho_in[0][0] = v.p.cl_in * pout / (v.rc.s[0] * kCs2);
  ap.drho_in[0][1] = (1.0 - v.p.cl_in) * pout / (v.rc.s[1] * kCs2);
  ap.drho_in[1][0] = pin / (v.rc.s[0] * kCs2);
  ap.drho_in[1][1] = -pin / (v.rc.s[1] * kCs2);
  ap.cl_in = v.p.cl_in;
  ap.inv_cl_in = 1.0 / v.p.cl_in;
  st = v.stream;
  return LBSEP_OK;
}

int make_adj(const lbsep_channel* ch, void* ws, size_t bytes, AdjParams& ap, AdjLayout& L, hipStream_t& st) {
  lbsep_params p;
  if (int e = adj_params(ch, ap, st, &p)) return e;
  L = adj_layout(&p);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u))
    return set_error(LBSEP_EINVAL, "adjoint workspace must be a non-NULL 256-byte aligned device pointer");
  if (bytes < L.total) return set_error(LBSEP_ESIZE, "adjoint workspace too small");
  return LBSEP_OK;
}

// One reverse step (lbsep_adjoint_step) with its scratch at ws laid out by L.
int enqueue_adjoint_step(const AdjParams& ap, const AdjLayout& L, hipStream_t st, char* ws, const double* f_t,
                         const double* f_post, const double* lam_next, double* lam_out, double* dparams) {
  if (!f_t || !lam_next || !lam_out || !dparams) return set_error(LBSEP_EINVAL, "NULL buffer");
  if (lam_out == lam_next || lam_out == f_t || (f_post && lam_out == f_post))
    return set_error(LBSEP_EINVAL, "lam_out must not alias the inputs");
  const double* fpost = f_post;
  double* lamP = reinterpret_cast<double*>(ws + L.lamP);
  double* pe = reinterpret_cast<double*>(ws + L.part_ends);
  double* pr = reinterpret_cast<double*>(ws + L.part_r);
  if (!fpost) {  // recompute C(f_t) into the scratch
    double* own = reinterpret_cast<double*>(ws + L.fpost);
    hipLaunchKernelGGL(k_adj_post, dim3(L.nblocks), dim3(kAT), 0, st, ap, f_t, own);
    fpost = own;
  }
  const bool ends = !(ap.flags & LBSEP_PERIODIC_X);
  if (ends) hipLaunchKernelGGL(k_adj_ends, dim3(4), dim3(kAT), 0, st, ap, fpost, lam_next, lamP, pe);
  hipLaunchKernelGGL(k_adj_main, dim3(L.nblocks), dim3(kAT), 0, st, ap, f_t, fpost, lam_next, lamP, lam_out, pr);
  hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(kAT), 0, st, ends ? pe : nullptr, pr, L.nblocks, nullptr, 0,
                     dparams);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(LBSEP_EDEVICE, (std::string("adjoint step launch: ") + hipGetErrorString(e)).c_str());
  return LBSEP_OK;
}

// ---- fixed scratch of the allocation-free reverse step ------------------------
// One copy of this array per GPU, loaded with the code object and held until
// the process ends. Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol): the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
__device__ __align__(256) unsigned char scratch[LBSEP_FIXED_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the device of stream st.
int fixed_scratch(hipStream_t st, char** out) {
  hipDevice_t dev = -1;
  // the null stream belongs to the current device
  hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess)
    return set_error(LBSEP_EDEVICE, (std::string("device of the channel's stream: ") + hipGetErrorString(e)).c_str());
  if (dev < 0 || dev >= kMaxDevices) return set_error(LBSEP_EINVAL, "device index beyond the fixed scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int prev = -1;
    e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t e2 = (prev >= 0 && prev != dev) ? hipSetDevice(prev) : hipSuccess;
    if (e != hipSuccess || !p)
      return set_error(LBSEP_EDEVICE, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    if (e2 != hipSuccess)
      return set_error(LBSEP_EDEVICE, (std::string("hipSetDevice: ") + hipGetErrorString(e2)).c_str());
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return LBSEP_OK;
}

int hip_ok(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(LBSEP_EDEVICE, (std::string(what) + ": " + hipGetErrorString(e)).c_str());
  return LBSEP_OK;
}

}  // namespace
}  // namespace lbsep

using namespace lbsep;

extern "C" {

size_t lbsep_adjoint_workspace_bytes(const lbsep_params* p) {
  if (!p || lbsep_workspace_bytes(p) == 0) return 0;
  return adj_layout(p).total;
}

int lbsep_adjoint_step(lbsep_channel* ch, const double* f_t, const double* f_post, const double* lam_next,
                       double* lam_out, double* dparams, void* adj_ws, size_t adj_ws_bytes) {
  AdjParams ap;
  AdjLayout L;
  hipStream_t st;
  if (int e = make_adj(ch, adj_ws, adj_ws_bytes, ap, L, st)) return e;
  return enqueue_adjoint_step(ap, L, st, static_cast<char*>(adj_ws), f_t, f_post, lam_next, lam_out, dparams);
}

int lbsep_adjoint_step_noalloc(lbsep_channel* ch, const double* f_t, const double* f_post, const double* lam_next,
                               double* lam_out, double* dparams) {
  AdjParams ap;
  hipStream_t st;
  lbsep_params p;
  if (int e = adj_params(ch, ap, st, &p)) return e;
  const AdjLayout L = adj_layout(&p, f_post == nullptr);
  if (L.total > (size_t)LBSEP_FIXED_SCRATCH_BYTES)
    return set_error(LBSEP_ESIZE, ("lbsep_adjoint_step_noalloc: this channel needs " + std::to_string(L.total) +
                                   " bytes of scratch, the fixed scratch holds " +
                                   std::to_string((size_t)LBSEP_FIXED_SCRATCH_BYTES) +
                                   (f_post ? "" : " (passing f_post needs less)") +
                                   "; use lbsep_adjoint_step with a workspace")
                                      .c_str());
  char* ws = nullptr;
  if (int e = fixed_scratch(st, &ws)) return e;
  return enqueue_adjoint_step(ap, L, st, ws, f_t, f_post, lam_next, lam_out, dparams);
}

int lbsep_adjoint_seed_cl(lbsep_channel* ch, const double* f_T, double* lam_out, double* dparams, void* adj_ws,
                          size_t adj_ws_bytes) {
  AdjParams ap;
  AdjLayout L;
  hipStream_t st;
  if (int e = make_adj(ch, adj_ws, adj_ws_bytes, ap, L, st)) return e;
  if (!f_T || !lam_out || !dparams) return set_error(LBSEP_EINVAL, "NULL buffer");
  double* cols = reinterpret_cast<double*>(static_cast<char*>(adj_ws) + L.cols);
  const long long n = 18LL * ap.nx * ap.ny;
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(kAT), 0, st, lam_out, n, 0.0);
  hipLaunchKernelGGL(k_adj_colsum, dim3((ap.nx + kAT - 1) / kAT), dim3(kAT), 0, st, ap, f_T, cols);
  hipLaunchKernelGGL(k_adj_seed, dim3(1), dim3(kAT), 0, st, ap, cols, lam_out, dparams);
  return hip_ok("adjoint seed launch");
}

int lbsep_adjoint_initial(lbsep_channel* ch, const double* lam0, double* dparams, void* adj_ws, size_t adj_ws_bytes) {
  AdjParams ap;
  AdjLayout L;
  hipStream_t st;
  if (int e = make_adj(ch, adj_ws, adj_ws_bytes, ap, L, st)) return e;
  if (!lam0 || !dparams) return set_error(LBSEP_EINVAL, "NULL buffer");
  if (ap.flags & LBSEP_PERIODIC_X) return set_error(LBSEP_EINVAL, "the initial state of R18 needs inlet and outlet");
  double* cols = reinterpret_cast<double*>(static_cast<char*>(adj_ws) + L.cols);
  hipLaunchKernelGGL(k_adj_initial, dim3((ap.nx + kAT - 1) / kAT), dim3(kAT), 0, st, ap, lam0, cols);
  hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(kAT), 0, st, nullptr, nullptr, 0, cols, ap.nx, dparams);
  return hip_ok("adjoint initial launch");
}

}  // extern "C"
