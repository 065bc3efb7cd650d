// lbf_math.h -- register-resident mode transforms of the two lattice models,
// D3Q19 (basis of Table II) and D2Q9 (basis of Table I).
//
// The state is the scaled deviation d_i = (n_i - a_i rho0) / (a_i rho0).
// Working in units of rho0 / 36, the unscaled modes m_k = sum_i e_ki n_i
// (Sec. III) of the deviation n_i - a_i rho0 become
//     mu_k = 36 m_k / rho0 = sum_i (36 a_i) e_ki d_i,
// with integer weights 36 a_i (12, 2, 1 for D3Q19; 16, 4, 1 for D2Q9), and
// the back-transform n_i = a_i sum_k e_ki m_k / w_k (completeness of the
// orthonormal basis, Eqs. orthogonality and evectors_orthonormal) becomes
//     d_i = sum_k e_ki nu_k,   nu_k = mu_k / (36 w_k).
//
// Opposite velocities i, opp(i) share the even-parity rows of the basis and
// have opposite odd-parity rows, so both transforms run on the pair sums
// s = d_i + d_opp(i) and differences d = d_i - d_opp(i) (first member of
// each pair has the positive leading component): one block of small integer
// coefficients per parity, written out term by term below.
//
// Each model also gives the equilibrium values of its stress modes (the
// only non-conserved modes with a non-zero equilibrium part: the kinetic
// modes are orthogonal to every polynomial of degree <= 2) from mu_1..mu_d
// and 1 / R, R = 36 rho / rho0, by the stress of Eq. derived_equil_distrib
// with sigma_2 = c_s^2 = 1/3.
#pragma once

#if defined(__HIPCC__)
#define LBF_HD __host__ __device__ __forceinline__
#else
#define LBF_HD inline
#endif

namespace lbf {

// ================================================================ D3Q19
// Velocity order: 0 rest; 1..6 = +x -x +y -y +z -z; 7/8 = +-(1,1,0);
// 9/10 = +-(1,-1,0); 11/12 = +-(1,0,1); 13/14 = +-(1,0,-1);
// 15/16 = +-(0,1,1); 17/18 = +-(0,1,-1).  Modes (Table II): 0..3
// conserved, 4 bulk, 5..9 shear, 10..15 odd kinetic, 16..18 even kinetic.
struct D3Q19 {
  static constexpr int Q = 19, D = 3;
  static constexpr int NSTRESS = 6;  // stress modes k = D + 1 .. D + NSTRESS
  static constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  // 36 a_i (Sec. II: 1/3, 1/18, 1/36) and 36 w_k of Table II (w_k = sum_i a_i e_ki^2)
  static constexpr float A36[Q] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
  static constexpr float W36[Q] = {36, 12, 12, 12, 24, 48, 16, 4, 4, 4, 24, 24, 24, 8, 8, 8, 72, 48, 16};
  // mode class: 0 conserved, 1 bulk, 2 shear, 3 odd kinetic, 4 even kinetic
  static constexpr int CLS[Q] = {0, 0, 0, 0, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 4, 4, 4};

  template <class F> static LBF_HD void forward(const F d[Q], F mu[Q]);
  template <class F> static LBF_HD void back(const F nu[Q], F d[Q]);
  // equilibrium stress modes in units of rho0/36:
  // mu_4 = |j|^2 / R, mu_5 = (2 jx^2 - jy^2 - jz^2) / R, mu_6 = (jy^2 - jz^2) / R,
  // mu_7..9 = jx jy / R, jy jz / R, jz jx / R
  template <class F> static LBF_HD void stress_eq(const F mu[Q], F iR, F eq[NSTRESS]) {
    const F vx = mu[1] * iR, vy = mu[2] * iR, vz = mu[3] * iR;
    const F xx = mu[1] * vx, yy = mu[2] * vy, zz = mu[3] * vz;
    eq[0] = (xx + yy) + zz;
    eq[1] = (F(2) * xx - yy) - zz;
    eq[2] = yy - zz;
    eq[3] = mu[1] * vy;
    eq[4] = mu[2] * vz;
    eq[5] = mu[3] * vx;
  }
};

// mu_k = sum_i 36 a_i e_ki d_i for all 19 modes.
template <class F>
LBF_HD void D3Q19::forward(const F d[Q], F mu[Q]) {
  // pair sums and differences: X, Y, Z axes; A=(1,1,0) B=(1,-1,0)
  // C=(1,0,1) D=(1,0,-1) E=(0,1,1) F=(0,1,-1) diagonals
  const F sX = d[1] + d[2], dX = d[1] - d[2];
  const F sY = d[3] + d[4], dY = d[3] - d[4];
  const F sZ = d[5] + d[6], dZ = d[5] - d[6];
  const F sA = d[7] + d[8], dA = d[7] - d[8];
  const F sB = d[9] + d[10], dB = d[9] - d[10];
  const F sC = d[11] + d[12], dC = d[11] - d[12];
  const F sD = d[13] + d[14], dD = d[13] - d[14];
  const F sE = d[15] + d[16], dE = d[15] - d[16];
  const F sF = d[17] + d[18], dF = d[17] - d[18];
  const F r12 = F(12) * d[0];

  // even block: k = 0, 4, 5, 6, 7, 8, 9, 16, 17, 18
  const F Sxy = sA + sB, Sxz = sC + sD, Syz = sE + sF;
  const F Sd = (Sxy + Sxz) + Syz;      // all diagonals
  const F Tyz = sY + sZ;
  const F Sax = sX + Tyz;              // all axis pairs
  const F Dyz = sY - sZ;
  const F Pxy = Sxy + Sxz, Mxy = Sxy - Sxz;
  const F b5 = Pxy - F(2) * Syz;              // shared by k = 5 and 17
  mu[0] = r12 + F(2) * Sax + Sd;              // 1
  mu[4] = Sd - r12;                           // c^2 - 1
  mu[16] = (r12 + Sd) - F(4) * Sax;           // 3c^4 - 6c^2 + 1
  mu[5] = (b5 - F(2) * Tyz) + F(4) * sX;      // 3cx^2 - c^2
  mu[17] = (b5 + F(2) * Tyz) - F(4) * sX;     // (2c^2-3)(3cx^2-c^2)
  mu[6] = F(2) * Dyz + Mxy;                   // cy^2 - cz^2
  mu[18] = Mxy - F(2) * Dyz;                  // (2c^2-3)(cy^2-cz^2)
  mu[7] = sA - sB;                            // cx cy
  mu[8] = sE - sF;                            // cy cz
  mu[9] = sC - sD;                            // cz cx

  // odd block: k = 1, 2, 3, 10..15
  const F Ux = (dA + dB) + (dC + dD);
  const F Uy = (dA - dB) + (dE + dF);
  const F Uz = (dC - dD) + (dE - dF);
  mu[1] = F(2) * dX + Ux;                     // cx
  mu[2] = F(2) * dY + Uy;                     // cy
  mu[3] = F(2) * dZ + Uz;                     // cz
  mu[10] = Ux - F(4) * dX;                    // (3c^2-5) cx
  mu[11] = Uy - F(4) * dY;                    // (3c^2-5) cy
  mu[12] = Uz - F(4) * dZ;                    // (3c^2-5) cz
  mu[13] = (dA + dB) - (dC + dD);             // (cy^2-cz^2) cx
  mu[14] = (dE + dF) - (dA - dB);             // (cz^2-cx^2) cy
  mu[15] = (dC - dD) - (dE - dF);             // (cx^2-cy^2) cz
}

// d_i = sum_k e_ki nu_k for all 19 populations.
template <class F>
LBF_HD void D3Q19::back(const F nu[Q], F d[Q]) {
  // even parts
  const F J = nu[0] - F(2) * nu[16];
  const F M = nu[5] - nu[17];
  const F N = nu[6] - nu[18];
  const F G = (nu[0] + nu[4]) + nu[16];
  const F H = nu[5] + nu[17];
  const F K = nu[6] + nu[18];
  const F GH = G + H;
  const F GHp = GH + K, GHm = GH - K;
  const F G2 = G - F(2) * H;
  const F eX = J + F(2) * M;
  const F eYZ = J - M;
  const F eY = eYZ + N, eZ = eYZ - N;
  const F eA = GHp + nu[7], eB = GHp - nu[7];
  const F eC = GHm + nu[9], eD = GHm - nu[9];
  const F eE = G2 + nu[8], eF = G2 - nu[8];
  // odd parts (value for the first member of each pair)
  const F oX = nu[1] - F(2) * nu[10];
  const F oY = nu[2] - F(2) * nu[11];
  const F oZ = nu[3] - F(2) * nu[12];
  const F a1 = nu[1] + nu[10], a2 = nu[2] + nu[11], a3 = nu[3] + nu[12];
  const F oA = (a1 + a2) + (nu[13] - nu[14]);
  const F oB = (a1 - a2) + (nu[13] + nu[14]);
  const F oC = (a1 + a3) + (nu[15] - nu[13]);
  const F oD = (a1 - a3) - (nu[13] + nu[15]);
  const F oE = (a2 + a3) + (nu[14] - nu[15]);
  const F oF = (a2 - a3) + (nu[14] + nu[15]);

  d[0] = (nu[0] - nu[4]) + nu[16];
  d[1] = eX + oX;  d[2] = eX - oX;
  d[3] = eY + oY;  d[4] = eY - oY;
  d[5] = eZ + oZ;  d[6] = eZ - oZ;
  d[7] = eA + oA;  d[8] = eA - oA;
  d[9] = eB + oB;  d[10] = eB - oB;
  d[11] = eC + oC; d[12] = eC - oC;
  d[13] = eD + oD; d[14] = eD - oD;
  d[15] = eE + oE; d[16] = eE - oE;
  d[17] = eF + oF; d[18] = eF - oF;
}

// ================================================================ D2Q9
// Velocity order: 0 rest; 1..4 = +x -x +y -y; 5/6 = +-(1,1); 7/8 = +-(1,-1).
// Modes (Table I): 0..2 conserved, 3 bulk, 4..5 shear, 6..7 odd kinetic,
// 8 even kinetic.  Weights 4/9, 1/9, 1/36 (the three-speed solution of the
// isotropy conditions of Sec. II, with c_s^2 = 1/3).
struct D2Q9 {
  static constexpr int Q = 9, D = 2;
  static constexpr int NSTRESS = 3;
  static constexpr int CX[Q] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int CY[Q] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr int CZ[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
  static constexpr float A36[Q] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
  static constexpr float W36[Q] = {36, 12, 12, 144, 16, 4, 24, 24, 576};
  static constexpr int CLS[Q] = {0, 0, 0, 1, 2, 2, 3, 3, 4};

  // mu_k = sum_i 36 a_i e_ki d_i.  Pairs: X = (1, 2), Y = (3, 4),
  // A = (1,1) (5, 6), B = (1,-1) (7, 8).
  template <class F> static LBF_HD void forward(const F d[Q], F mu[Q]) {
    const F sX = d[1] + d[2], dX = d[1] - d[2];
    const F sY = d[3] + d[4], dY = d[3] - d[4];
    const F sA = d[5] + d[6], dA = d[5] - d[6];
    const F sB = d[7] + d[8], dB = d[7] - d[8];
    const F r16 = F(16) * d[0];
    const F Sax = sX + sY, Sd = sA + sB;
    mu[0] = (r16 + F(4) * Sax) + Sd;                          // 1
    mu[3] = F(4) * (Sax + Sd) - F(2) * r16;                   // 3c^2 - 2
    mu[4] = F(4) * (sX - sY);                                 // 2cx^2 - c^2
    mu[5] = sA - sB;                                          // cx cy
    mu[8] = (F(2) * r16 - F(16) * Sax) + F(8) * Sd;           // 9c^4 - 15c^2 + 2
    const F Px = dA + dB, Py = dA - dB;
    mu[1] = F(4) * dX + Px;                                   // cx
    mu[2] = F(4) * dY + Py;                                   // cy
    mu[6] = F(2) * Px - F(4) * dX;                            // (3c^2 - 4) cx
    mu[7] = F(2) * Py - F(4) * dY;                            // (3c^2 - 4) cy
  }

  // d_i = sum_k e_ki nu_k.
  template <class F> static LBF_HD void back(const F nu[Q], F d[Q]) {
    const F base = nu[0] + nu[3];                 // e_0 = e_3 = 1 on the axis velocities
    const F eX = (base + nu[4]) - F(4) * nu[8];
    const F eY = (base - nu[4]) - F(4) * nu[8];
    const F g = (nu[0] + F(4) * nu[3]) + F(8) * nu[8];
    const F eA = g + nu[5], eB = g - nu[5];
    const F oX = nu[1] - nu[6];
    const F oY = nu[2] - nu[7];
    const F s1 = nu[1] + F(2) * nu[6], s2 = nu[2] + F(2) * nu[7];
    const F oA = s1 + s2, oB = s1 - s2;
    d[0] = (nu[0] - F(2) * nu[3]) + F(2) * nu[8];
    d[1] = eX + oX; d[2] = eX - oX;
    d[3] = eY + oY; d[4] = eY - oY;
    d[5] = eA + oA; d[6] = eA - oA;
    d[7] = eB + oB; d[8] = eB - oB;
  }

  // mu_3 = 3 |j|^2 / R, mu_4 = (jx^2 - jy^2) / R, mu_5 = jx jy / R
  template <class F> static LBF_HD void stress_eq(const F mu[Q], F iR, F eq[NSTRESS]) {
    const F vx = mu[1] * iR, vy = mu[2] * iR;
    const F xx = mu[1] * vx, yy = mu[2] * vy;
    eq[0] = F(3) * (xx + yy);
    eq[1] = xx - yy;
    eq[2] = mu[1] * vy;
  }
};

}  // namespace lbf
