// Pointwise ionic models for the monodomain step, evaluated per mesh node.
//
// The paper writes every model as du/dt + I_ion(u, w) = I_app,
// dw/dt = H(u, w) (eq. of the ionic model ODEs) and cites the four models it
// ships; the three used here are written from their original publications:
//   Aliev-Panfilov (1996)         u dimensionless, model time unit 12.9 ms
//   Bueno-Orovio minimal (2008)   EPI parameter set, u dimensionless
//   ten Tusscher-Panfilov (2006)  endo / mid / epi cells, V in mV
// One call advances the ionic state by dt at the extrapolated potential u*
// (eq. of the time-discrete ionic model) with one of two integrators, then
// returns I_ion(u*, w_{n+1}), which the monodomain step uses explicitly (eq.
// of the time-discrete monodomain equation):
//   Rush-Larsen: gating variables by the exact exponential at u*, the others
//     by one explicit step with rates at (u*, new gates, old concentrations);
//   the paper's semi-implicit BDF (`*_bdf`): (alpha w_{n+1} - w_BDF)/dt =
//     H(u_EXT, w_EXT, w_{n+1}) with the potential's BDF order; gates implicit,
//     y_{n+1} = (y_BDF + dt y_inf/tau)/(alpha + dt/tau) with y_inf, tau at
//     (u*, w_EXT); Aliev-Panfilov v implicit in its -v term with
//     eps(u*, v_EXT); TTP06 concentrations explicit from (u*, new gates,
//     extrapolated concentrations), calcium as buffered totals.
//
// Precision: R = double (FP64 path) or float (mixed path).  The TTP06 sodium
// and potassium concentrations stay in double in both, because their
// per-step increments fall below one FP32 ulp of their values.
#pragma once
#include <hip/hip_runtime.h>

namespace ep {

__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float m_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_tanh(double x) { return tanh(x); }
__device__ __forceinline__ float m_tanh(float x) { return tanhf(x); }

// Rush-Larsen update of one gate: exact solution of dy/dt = (y_inf - y)/tau
// over dt with y_inf and tau frozen at u*, y + (y_inf - y)(1 - e^{-dt/tau}).
// The fraction 1 - e^{-dt/tau} is formed by expm1: for slow gates (dt/tau
// ~ 1e-4) e^{-dt/tau} rounded to FP32 would carry a relative error of ~1e-3
// in that fraction, i.e. a biased decay rate every step.
template <typename R>
__device__ __forceinline__ R rush_larsen(R y, R y_inf, R tau, R dt) {
  return y + (y_inf - y) * (-m_expm1(-dt / tau));
}

// ---------------------------------------------------------------------------
// Aliev-Panfilov.  Parameters: k, a, eps0, mu1, mu2, T (ms per model time).
// I_ion = (k u (u-a)(u-1) + u v)/T ;  dv/dt = eps(u,v) (-v - k u (u-a-1))/T,
// eps = eps0 + mu1 v/(u + mu2).  v is not a gate: explicit step.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R ap_step(R u, R dt, const double* mp, R& v) {
  const R k = R(mp[0]), a = R(mp[1]), eps0 = R(mp[2]), mu1 = R(mp[3]), mu2 = R(mp[4]);
  const R invT = R(1.0 / mp[5]);
  const R eps = eps0 + mu1 * v / (u + mu2);
  v = v + dt * (eps * (-v - k * u * (u - a - R(1))) * invT);
  return (k * u * (u - a) * (u - R(1)) + u * v) * invT;
}

template <typename R>
__device__ __forceinline__ R ap_step_bdf(R u, R dt, R alpha, const double* mp, R v_bdf, R v_ext, R& v) {
  const R k = R(mp[0]), a = R(mp[1]), eps0 = R(mp[2]), mu1 = R(mp[3]), mu2 = R(mp[4]);
  const R invT = R(1.0 / mp[5]);
  const R eps = (eps0 + mu1 * v_ext / (u + mu2)) * invT;
  v = (v_bdf - dt * eps * (k * u * (u - a - R(1)))) / (alpha + dt * eps);
  return (k * u * (u - a) * (u - R(1)) + u * v) * invT;
}

// BDF step of a gate dy/dt = (y_inf - y)/tau, implicit in y:
// y = (y_BDF + c y_inf)/(alpha + c), c = dt/tau, written as
// y_BDF/alpha + c/(alpha + c) (y_inf - y_BDF/alpha) so that a slow gate's
// small relaxation is not formed from a quotient of two nearly equal
// rounded numbers (a biased rate in FP32).
template <typename R>
__device__ __forceinline__ R gate_bdf(R y_bdf, R y_inf, R tau, R dt, R alpha) {
  const R c = dt / tau;
  const R y0 = y_bdf / alpha;
  return y0 + c / (alpha + c) * (y_inf - y0);
}

// ---------------------------------------------------------------------------
// Bueno-Orovio minimal model.  Parameter slots (EPI defaults set by the host):
//  0 u_o  1 u_u  2 theta_v  3 theta_w  4 theta_v-  5 theta_o  6 tau_v1-
//  7 tau_v2-  8 tau_v+  9 tau_w1-  10 tau_w2-  11 k_w-  12 u_w-  13 tau_w+
//  14 tau_fi  15 tau_o1  16 tau_o2  17 tau_so1  18 tau_so2  19 k_so  20 u_so
//  21 tau_s1  22 tau_s2  23 k_s  24 u_s  25 tau_si  26 tau_winf  27 w_inf*
// Heaviside H(x) = 1 for x > 0.  v, w, s are all gates (Rush-Larsen).
// ---------------------------------------------------------------------------
// BDF = false: Rush-Larsen from (v, w, s); BDF = true: (v, w, s) are
// overwritten with the semi-implicit BDF step from their BDF combinations yb.
template <typename R, bool BDF = false>
__device__ __forceinline__ R bo_step(R u, R dt, const double* mp, R& v, R& w, R& s, R alpha = R(1),
                                     const R* yb = nullptr) {
  const bool hv = u > R(mp[2]);
  const bool hw = u > R(mp[3]);
  const bool hvm = u > R(mp[4]);
  const bool ho = u > R(mp[5]);
  // gate targets at u*
  R v_inf, tau_v;
  if (hv) { v_inf = R(0); tau_v = R(mp[8]); }
  else { v_inf = hvm ? R(0) : R(1); tau_v = hvm ? R(mp[7]) : R(mp[6]); }
  R w_inf, tau_w;
  if (hw) { w_inf = R(0); tau_w = R(mp[13]); }
  else {
    w_inf = ho ? R(mp[27]) : (R(1) - u / R(mp[26]));
    tau_w = R(mp[9]) + (R(mp[10]) - R(mp[9])) * (R(1) + m_tanh(R(mp[11]) * (u - R(mp[12])))) * R(0.5);
  }
  const R s_inf = (R(1) + m_tanh(R(mp[23]) * (u - R(mp[24])))) * R(0.5);
  const R tau_s = hw ? R(mp[22]) : R(mp[21]);
  if (BDF) {
    v = gate_bdf(yb[0], v_inf, tau_v, dt, alpha);
    w = gate_bdf(yb[1], w_inf, tau_w, dt, alpha);
    s = gate_bdf(yb[2], s_inf, tau_s, dt, alpha);
  } else {
    v = rush_larsen(v, v_inf, tau_v, dt);
    w = rush_larsen(w, w_inf, tau_w, dt);
    s = rush_larsen(s, s_inf, tau_s, dt);
  }
  // currents at (u*, w_{n+1})
  const R J_fi = hv ? -v * (u - R(mp[2])) * (R(mp[1]) - u) / R(mp[14]) : R(0);
  R J_so;
  if (hw) {
    const R tau_so = R(mp[17]) + (R(mp[18]) - R(mp[17])) * (R(1) + m_tanh(R(mp[19]) * (u - R(mp[20])))) * R(0.5);
    J_so = R(1) / tau_so;
  } else {
    J_so = (u - R(mp[0])) / (ho ? R(mp[16]) : R(mp[15]));
  }
  const R J_si = hw ? -w * s / R(mp[25]) : R(0);
  return J_fi + J_so + J_si;
}

// ---------------------------------------------------------------------------
// ten Tusscher-Panfilov 2006.  Parameter slots:
//  0 GNa 1 GK1 2 Gto 3 GKr 4 GKs 5 GCaL 6 GbNa 7 GbCa 8 GpCa 9 GpK 10 kNaCa
//  11 PNaK 12 Vrel 13 Vleak 14 Vmaxup 15 Vxfer 16 endocardial s-gate (0/1)
// State order: m h j xr1 xr2 xs s r d f f2 fcass | cai casr cass nai ki rr
// ---------------------------------------------------------------------------
namespace ttp {
constexpr double kR = 8314.472, kT = 310.0, kF = 96485.3415;
constexpr double RTF = kR * kT / kF;                 // mV
constexpr double Cm = 0.185, Vc = 0.016404, Vsr = 0.001094, Vss = 0.00005468;
constexpr double Ko = 5.4, Nao = 140.0, Cao = 2.0, pKNa = 0.03;
constexpr double KmK = 1.0, KmNa = 40.0, KmNai = 87.5, KmCa = 1.38, ksat = 0.1;
constexpr double alpha = 2.5, gamma = 0.35, KpCa = 0.0005, Kup = 0.00025;
constexpr double k1p = 0.15, k2p = 0.045, k3 = 0.060, k4 = 0.005, EC = 1.5;
constexpr double maxsr = 2.5, minsr = 1.0;
constexpr double Bufc = 0.2, Kbufc = 0.001, Bufsr = 10.0, Kbufsr = 0.3;
constexpr double Bufss = 0.4, Kbufss = 0.00025;
}  // namespace ttp

template <typename R>
struct TtpState {
  R g[12];
  R cai, casr, cass, rr;
  double nai, ki;
};

// Free concentration from the total under rapid buffering:
// positive root of c + B c/(c + K) = T, in a cancellation-free form.
template <typename R>
__device__ __forceinline__ R buffered_free(R total, R B, R K) {
  const R b = B + K - total;
  const R disc = m_sqrt(b * b + R(4) * K * total);
  return b >= R(0) ? (R(2) * K * total) / (b + disc) : R(0.5) * (disc - b);
}

// Buffered total of a free concentration c: c + B c/(c + K).
template <typename R>
__device__ __forceinline__ R buffered_total(R c, R B, R K) {
  return c + B * c / (c + K);
}

// BDF = false: Rush-Larsen, S in/out.  BDF = true: S receives w_{n+1} from the
// BDF combinations Sb (gates, nai, ki, rr; calcium as the buffered totals
// tb[3] of cai, casr, cass) and the extrapolations Se.
// (The BDF leading coefficient is named a_bdf: ttp::alpha is the Na/Ca
// exchanger's parameter.)
template <typename R, bool BDF = false>
__device__ __forceinline__ R ttp06_step(R V, R dt, const double* mp, TtpState<R>& S, R a_bdf = R(1),
                                        const TtpState<R>* Sb = nullptr, const TtpState<R>* Se = nullptr,
                                        const R* tb = nullptr) {
  using namespace ttp;
  const R one = R(1);
  // gate update: Rush-Larsen from the old gate, or implicit BDF from its combination
  auto gate = [&](int k, R inf, R tau) {
    if (BDF) S.g[k] = gate_bdf(Sb->g[k], inf, tau, dt, a_bdf);
    else S.g[k] = rush_larsen(S.g[k], inf, tau, dt);
  };
  // ---- gates: Rush-Larsen at V (fcass uses the old subspace calcium) ----
  // Exponentials of (V + a) / b with a shared b come from one exp(V / b):
  // exp((V + a) / b) = exp(a / b) exp(V / b); divisions by constants are
  // multiplications by their reciprocals.  Each rewrite changes the result
  // by a few ulps only.
  {
    const R E5 = m_exp(V * R(0.2)), iE5 = one / E5;          // exp(V/5)
    const R E10 = m_exp(V * R(0.1)), iE10 = one / E10;       // exp(V/10)
    const R E20 = m_exp(V * R(0.05)), iE20 = one / E20;      // exp(V/20)
    const R E7 = m_exp(V * R(1.0 / 7.0)), iE7 = one / E7;    // exp(V/7)
    const R iE6 = m_exp(V * R(-1.0 / 6.0));                  // exp(-V/6)
    R t = one + m_exp((R(-56.86) - V) * R(1.0 / 9.03));
    const R m_inf = one / (t * t);
    const R a_m = one / (one + R(6.14421235332821e-06) * iE5);               // (-60 - V)/5
    const R b_m = R(0.1) / (one + R(1096.6331584284585) * E5) +              // (V + 35)/5
                  R(0.1) / (one + m_exp((V - R(50.0)) * R(0.005)));
    gate(0, m_inf, a_m * b_m);

    t = one + m_exp((V + R(71.55)) * R(1.0 / 7.43));
    const R hj_inf = one / (t * t);
    R a_h, b_h, a_j, b_j;
    if (V >= R(-40.0)) {
      a_h = R(0);
      b_h = R(0.77) / (R(0.13) * (one + m_exp(-(V + R(10.66)) * R(1.0 / 11.1))));
      a_j = R(0);
      b_j = R(0.6) * m_exp(R(0.057) * V) / (one + R(0.04076220397836621) * iE10);   // -0.1 (V + 32)
    } else {
      a_h = R(0.057) * m_exp(-(V + R(80.0)) * R(1.0 / 6.8));
      b_h = R(2.7) * m_exp(R(0.079) * V) + R(3.1e5) * m_exp(R(0.3485) * V);
      a_j = (R(-2.5428e4) * m_exp(R(0.2444) * V) - R(6.948e-6) * m_exp(R(-0.04391) * V)) *
            (V + R(37.78)) / (one + m_exp(R(0.311) * (V + R(79.23))));
      b_j = R(0.02424) * m_exp(R(-0.01052) * V) / (one + m_exp(R(-0.1378) * (V + R(40.14))));
    }
    gate(1, hj_inf, one / (a_h + b_h));
    gate(2, hj_inf, one / (a_j + b_j));

    const R xr1_inf = one / (one + R(0.0243728440732796) * iE7);            // (-26 - V)/7
    const R tau_xr1 = (R(450.0) / (one + R(0.011108996538242306) * iE10)) *  // (-45 - V)/10
                      (R(6.0) / (one + m_exp((V + R(30.0)) * R(1.0 / 11.5))));
    gate(3, xr1_inf, tau_xr1);
    const R xr2_inf = one / (one + m_exp((V + R(88.0)) * R(1.0 / 24.0)));
    const R tau_xr2 = (R(3.0) / (one + R(0.049787068367863944) * iE20)) *    // (-60 - V)/20
                      (R(1.12) / (one + R(0.049787068367863944) * E20));     // (V - 60)/20
    gate(4, xr2_inf, tau_xr2);
    const R xs_inf = one / (one + m_exp((R(-5.0) - V) * R(1.0 / 14.0)));
    const R tau_xs = (R(1400.0) / m_sqrt(one + R(2.300975890892825) * iE6)) *     // (5 - V)/6
                         (one / (one + m_exp((V - R(35.0)) * R(1.0 / 15.0)))) + R(80.0);
    gate(5, xs_inf, tau_xs);
    R s_inf, tau_s;
    if (mp[16] != 0.0) {
      s_inf = one / (one + R(270.42640742615254) * E5);                      // (V + 28)/5
      tau_s = R(1000.0) * m_exp(-(V + R(67.0)) * (V + R(67.0)) * R(0.001)) + R(8.0);
    } else {
      s_inf = one / (one + R(54.598150033144236) * E5);                      // (V + 20)/5
      tau_s = R(85.0) * m_exp(-(V + R(45.0)) * (V + R(45.0)) * R(1.0 / 320.0)) +
              R(5.0) / (one + R(0.01831563888873418) * E5) + R(3.0);          // (V - 20)/5
    }
    gate(6, s_inf, tau_s);
    const R r_inf = one / (one + R(28.03162489452614) * iE6);                // (20 - V)/6
    const R tau_r = R(9.5) * m_exp(-(V + R(40.0)) * (V + R(40.0)) * R(1.0 / 1800.0)) + R(0.8);
    gate(7, r_inf, tau_r);
    const R d_inf = one / (one + m_exp((R(-8.0) - V) * R(1.0 / 7.5)));
    const R tau_d = (R(1.4) / (one + m_exp((R(-35.0) - V) * R(1.0 / 13.0))) + R(0.25)) *
                        (R(1.4) / (one + R(2.718281828459045) * E5)) +       // (V + 5)/5
                    one / (one + R(12.182493960703473) * iE20);               // (50 - V)/20
    gate(8, d_inf, tau_d);
    const R f_inf = one / (one + R(17.41170806332765) * E7);                 // (V + 20)/7
    const R e30 = R(20.085536923187668) * E10;                               // (V + 30)/10
    const R tau_f = R(1102.5) * m_exp(-(V + R(27.0)) * (V + R(27.0)) * R(1.0 / 225.0)) +
                    R(200.0) / (one + R(3.6692966676192444) * iE10) +        // (13 - V)/10
                    R(180.0) / (one + e30) + R(20.0);
    gate(9, f_inf, tau_f);
    const R f2_inf = R(0.67) / (one + R(148.4131591025766) * E7) + R(0.33);  // (V + 35)/7
    const R tau_f2 = R(600.0) * m_exp(-(V + R(25.0)) * (V + R(25.0)) * R(1.0 / 170.0)) +
                     R(31.0) / (one + R(12.182493960703473) * iE10) +         // (25 - V)/10
                     R(16.0) / (one + e30);
    gate(10, f2_inf, tau_f2);
    const R cass_g = BDF ? Se->cass : S.cass;
    const R cr = (cass_g / R(0.05)) * (cass_g / R(0.05));
    gate(11, R(0.6) / (one + cr) + R(0.4), R(80.0) / (one + cr) + R(2.0));
  }

  // ---- factors that depend on V (and the new gates) only ----
  const R rtf = R(RTF);
  const R m = S.g[0], h = S.g[1], j = S.g[2];
  const R gNa = R(mp[0]) * m * m * m * h * j;
  const R gto = R(mp[2]) * S.g[7] * S.g[6];
  const R gKr = R(mp[3]) * S.g[3] * S.g[4];       // sqrt(Ko/5.4) = 1 at Ko = 5.4
  const R gKs = R(mp[4]) * S.g[5] * S.g[5];
  const R inv_rtf = R(1.0 / RTF);
  const R Er = m_exp(V * inv_rtf), iEr = one / Er;          // exp(V F/RT)
  const R z = R(2.0) * (V - R(15.0)) * inv_rtf;
  R zf;
  if (sizeof(R) == 8) zf = (fabs((double)z) < 1e-10) ? one - R(0.5) * z : z / m_expm1(z);
  else zf = (fabsf((float)z) < 1e-4f) ? one - R(0.5) * z : z / m_expm1(z);
  const R ez = Er * Er * R(0.3252969814969026);              // exp(z) = exp(2V F/RT) exp(-30 F/RT)
  const R gCaL = R(mp[5]) * S.g[8] * S.g[9] * S.g[10] * S.g[11] * R(2.0 * kF) * zf;
  const R u1 = m_exp(R(gamma) * V * inv_rtf);
  const R u2 = u1 * iEr;                                     // exp((gamma - 1) V F/RT)
  const R naca_k = R(mp[10]) /
                   (R((KmNai * KmNai * KmNai + Nao * Nao * Nao) * (KmCa + Cao)) * (one + R(ksat) * u2));
  const R nak_k = R(mp[11] * Ko / (Ko + KmK)) /
                  (one + R(0.1245) * m_exp(R(-0.1) * V * inv_rtf) + R(0.0353) * iEr);
  const R pk_k = R(mp[9]) / (one + m_exp((R(25.0) - V) * R(1.0 / 5.98)));

  // membrane currents at concentrations (cai, cass, nai, ki)
  struct Cur { R INa, IK1, Ito, IKr, IKs, ICaL, INaCa, INaK, IpCa, IpK, IbNa, IbCa; };
  auto membrane = [&](R cai, R cass, double nai, double ki) {
    Cur c;
    const R E_Na = rtf * m_log(R(Nao / nai));
    const R E_K = rtf * m_log(R(Ko / ki));
    const R E_Ks = rtf * m_log(R((Ko + pKNa * Nao) / (ki + pKNa * nai)));
    const R E_Ca = R(0.5) * rtf * m_log(R(Cao) / cai);
    const R vk = V - E_K;
    c.INa = gNa * (V - E_Na);
    c.Ito = gto * vk;
    c.IKr = gKr * vk;
    c.IKs = gKs * (V - E_Ks);
    // exp(0.06 (vk - 200)), exp(0.1 (vk - 10)) and exp(-0.5 vk) are powers of q = exp(0.02 vk)
    const R q = m_exp(R(0.02) * vk), q2 = q * q, q4 = q2 * q2, q8 = q4 * q4;
    const R q25 = q8 * q8 * q8 * q;
    const R a_K1 = R(0.1) / (one + R(6.14421235332821e-06) * (q2 * q));
    const R b_K1 = (R(3.0) * m_exp(R(0.0002) * (vk + R(100.0))) + R(0.36787944117144233) * (q4 * q)) /
                   (one + one / q25);
    c.IK1 = R(mp[1]) * (a_K1 / (a_K1 + b_K1)) * vk;
    c.ICaL = gCaL * (R(0.25) * cass * ez - R(Cao));
    const R nai3 = R(nai * nai * nai);
    c.INaCa = naca_k * (u1 * nai3 * R(Cao) - u2 * R(Nao * Nao * Nao * alpha) * cai);
    c.INaK = nak_k * R(nai / (nai + KmNa));
    c.IpCa = R(mp[8]) * cai / (R(KpCa) + cai);
    c.IpK = pk_k * vk;
    c.IbNa = R(mp[6]) * (V - E_Na);
    c.IbCa = R(mp[7]) * (V - E_Ca);
    return c;
  };

  // ---- explicit concentration step with currents at the old concentrations ----
  {
    const TtpState<R>& C = BDF ? *Se : S;     // concentrations the explicit rates use
    const Cur c = membrane(C.cai, C.cass, C.nai, C.ki);
    const R cai = C.cai, casr = C.casr, cass = C.cass, rr = C.rr;
    const R Iup = R(mp[14]) / (one + R(Kup * Kup) / (cai * cai));
    const R Ileak = R(mp[13]) * (casr - cai);
    const R kq = R(EC) / casr;
    const R kcasr = R(maxsr) - R(maxsr - minsr) / (one + kq * kq);
    const R k1 = R(k1p) / kcasr;
    const R k2 = R(k2p) * kcasr;
    const R O = k1 * cass * cass * rr / (R(k3) + k1 * cass * cass);
    const R Irel = R(mp[12]) * O * (casr - cass);
    const R Ixfer = R(mp[15]) * (cass - cai);
    const R cmF = R(Cm / kF);
    const R d_cai = -(c.IbCa + c.IpCa - R(2) * c.INaCa) * cmF / R(2.0 * Vc) +
                    R(Vsr / Vc) * (Ileak - Iup) + Ixfer;
    const R d_casr = Iup - Ileak - Irel;
    const R d_cass = -c.ICaL * cmF / R(2.0 * Vss) + R(Vsr / Vss) * Irel - R(Vc / Vss) * Ixfer;
    const R d_nai = -(c.INa + c.IbNa + R(3) * c.INaK + R(3) * c.INaCa) * cmF / R(Vc);
    const R d_ki = -(c.IK1 + c.Ito + c.IKr + c.IKs - R(2) * c.INaK + c.IpK) * cmF / R(Vc);
    const R d_rr = -k2 * cass * rr + R(k4) * (one - rr);
    if (BDF) {
      const R ia = one / a_bdf;
      S.cai = buffered_free((tb[0] + dt * d_cai) * ia, R(Bufc), R(Kbufc));
      S.casr = buffered_free((tb[1] + dt * d_casr) * ia, R(Bufsr), R(Kbufsr));
      S.cass = buffered_free((tb[2] + dt * d_cass) * ia, R(Bufss), R(Kbufss));
      S.nai = (Sb->nai + (double)(dt * d_nai)) / (double)a_bdf;
      S.ki = (Sb->ki + (double)(dt * d_ki)) / (double)a_bdf;
      S.rr = (Sb->rr + dt * d_rr) * ia;
    } else {
      const R tot_i = buffered_total(cai, R(Bufc), R(Kbufc)) + dt * d_cai;
      const R tot_sr = buffered_total(casr, R(Bufsr), R(Kbufsr)) + dt * d_casr;
      const R tot_ss = buffered_total(cass, R(Bufss), R(Kbufss)) + dt * d_cass;
      S.cai = buffered_free(tot_i, R(Bufc), R(Kbufc));
      S.casr = buffered_free(tot_sr, R(Bufsr), R(Kbufsr));
      S.cass = buffered_free(tot_ss, R(Bufss), R(Kbufss));
      S.nai = S.nai + (double)(dt * d_nai);
      S.ki = S.ki + (double)(dt * d_ki);
      S.rr = rr + dt * d_rr;
    }
  }
  // ---- I_ion at (V, w_{n+1}) ----
  const Cur c = membrane(S.cai, S.cass, S.nai, S.ki);
  return c.INa + c.IK1 + c.Ito + c.IKr + c.IKs + c.ICaL + c.INaCa + c.INaK + c.IpCa + c.IpK +
         c.IbNa + c.IbCa;
}

}  // namespace ep
