// ROS4 coefficients in the transformed form of paper Sec. 2.3 (u_i = sum_j
// gamma_ij k_j; a = alpha Gamma^-1, C = diag(1/gamma) - Gamma^-1,
// m = b Gamma^-1, e = (b - bhat) Gamma^-1).
//
// The paper names ROS4 with Hairer-Wanner coefficients (Table T:solvers) but
// prints no table.  This library uses an L-stable 4-stage set of order 4 with
// an embedded order-3 solution, obtained by solving the Rosenbrock order
// conditions: gamma = 1/x2 with x2 the second root of the Laguerre polynomial
// L4 (so R(inf) = 0), alpha_4j = alpha_3j (three f evaluations per step),
// free parameters alpha_21 = 2 gamma, alpha_3 = 0.45, b_4 = 0.4 and an
// embedded solution with bhat_4 = 0.
#pragma once

namespace chem {
constexpr double ROS4_GAMMA = 0.57281606248213485541;
constexpr double ROS4_A21 = 2.0;
constexpr double ROS4_A31 = 1.491001215556513813960407;
constexpr double ROS4_A32 = 0.2283940090236591778889569;
constexpr double ROS4_C21 = -7.137649921358897064355991;
constexpr double ROS4_C31 = -6.196702482993044766389505;
constexpr double ROS4_C32 = -0.8558736500387530085234008;
constexpr double ROS4_C41 = 5.964333552759764215600564;
constexpr double ROS4_C42 = 0.4379266338878570570784905;
constexpr double ROS4_C43 = 2.525577246716920611308754;
constexpr double ROS4_M1 = 1.63885860954486232683164;
constexpr double ROS4_M2 = 0.474955117534000084335749;
constexpr double ROS4_M3 = -0.07416508734030706110427568;
constexpr double ROS4_M4 = 0.6983044404633386302747267;
constexpr double ROS4_E1 = 0.09734671529814985040858406;
constexpr double ROS4_E2 = 0.2866125685892372986834792;
constexpr double ROS4_E3 = 0.6849355088701844022099764;
constexpr double ROS4_E4 = 0.6983044404633386302747267;
}  // namespace chem
