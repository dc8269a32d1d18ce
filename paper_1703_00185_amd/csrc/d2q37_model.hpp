// D2Q37 model constants, shared by host and device code of the library.
//
// Velocity set (the paper's Sec. 2 names 37 populations hopping up to 3
// sites; its figure of the set is not reproduced in the text): the shells
// (0,0) (1,0) (1,1) (2,0) (2,1) (2,2) (3,0) (3,1) with all sign and axis
// images, ordered by shell and then by (e_x, e_y) ascending.  In this order
// the opposite of population l is the mirror position inside its shell.
//
// Weights and velocity scale r: the unique positive solution of the
// isotropy conditions sum_l w_l (r e_lx)^(2a) (r e_ly)^(2b) =
// (2a-1)!! (2b-1)!! for a + b <= 4, written to 40 significant digits; the
// compiler rounds them to binary64.
#pragma once

#include <cstdint>

#define D2Q37_HD __host__ __device__

namespace d2q37 {

constexpr int NPOP = 37;
constexpr int NSHELL = 8;
constexpr int HALO = 3;       // halo columns on each side (max |e_x|)
constexpr int WALL_ROWS = 3;  // bc rows at each wall

constexpr int EX[NPOP] = {
    0,                                  // (0,0)
    -1, 0, 0, 1,                        // (1,0)
    -1, -1, 1, 1,                       // (1,1)
    -2, 0, 0, 2,                        // (2,0)
    -2, -2, -1, -1, 1, 1, 2, 2,         // (2,1)
    -2, -2, 2, 2,                       // (2,2)
    -3, 0, 0, 3,                        // (3,0)
    -3, -3, -1, -1, 1, 1, 3, 3};        // (3,1)
constexpr int EY[NPOP] = {
    0,
    0, -1, 1, 0,
    -1, 1, -1, 1,
    0, -2, 2, 0,
    -1, 1, -2, 2, -2, 2, -1, 1,
    -2, 2, -2, 2,
    0, -3, 3, 0,
    -1, 1, -3, 3, -3, 3, -1, 1};
constexpr int SHELL_START[NSHELL + 1] = {0, 1, 5, 9, 13, 21, 25, 29, 37};
constexpr int SHELL_N2[NSHELL] = {0, 1, 2, 4, 5, 8, 9, 10};  // |e|^2 per shell

constexpr double R = 1.196979770393074358972388463853275434844;
constexpr double R2 = R * R;
constexpr double W_SHELL[NSHELL] = {
    0.2331506691323525022865067040668499509961,
    0.1073060915422190024124642871831399358510,
    0.05766785988879488203006921539333941471077,
    0.01420821615845075026469894234413445497343,
    0.005353049000513775232731501662188493535094,
    0.001011937592673575475410908506639114714702,
    0.0002453010277577173454659166432678444638839,
    0.0002834142529941982174005252941948802334792};

D2Q37_HD constexpr int shell_of(int l) {
  int s = 0;
  while (SHELL_START[s + 1] <= l) ++s;
  return s;
}
D2Q37_HD constexpr int opp_of(int l) {
  const int s = shell_of(l);
  return SHELL_START[s] + SHELL_START[s + 1] - 1 - l;
}
D2Q37_HD constexpr double weight_of(int l) { return W_SHELL[shell_of(l)]; }
D2Q37_HD constexpr double inv_weight_of(int l) { return 1.0 / W_SHELL[shell_of(l)]; }

// Wall factor K_l(T) (zero-velocity equilibrium per unit density at
// temperature T).  Evaluated with no contraction in this exact order:
//   w_l * (1 + th*(C-2)/2 + th*th*(C*C - 8C + 8)/8),  th = T-1, C = (r*r)|e_l|^2.
inline double wall_factor(int l, double t_wall) {
  const double r2 = R * R;
  const double th = t_wall - 1.0;
  const double n2 = static_cast<double>(EX[l] * EX[l] + EY[l] * EY[l]);
  const double C = r2 * n2;
  return weight_of(l) * (1.0 + th * (C - 2.0) / 2.0 + th * th * (C * C - 8.0 * C + 8.0) / 8.0);
}

}  // namespace d2q37
