// Coefficients of the linearly implicit Rosenbrock solvers of the paper's
// solver table (Table T:solvers), in the transformed form of Sec. 2.3: with
// u_i = sum_j gamma_ij k_j each stage solves
//   (I/(h gamma) - J) u_i = f(y + sum_{j<i} a_ij u_j) + sum_{j<i} (c_ij / h) u_j
// and y_new = y + sum_j m_j u_j, with the error estimate sum_j e_j u_j, where
// a = alpha Gamma^-1, C = diag(1/gamma) - Gamma^-1, m = b Gamma^-1 and
// e = (b - bhat) Gamma^-1 (bhat the embedded weights).
//
// The values are the published ones of the references the table gives: ROS3
// and RODAS3 from Sandu et al. (1997); ROS4 - Hairer and Wanner's L-stable
// set - and RODAS4 from Hairer and Wanner, Solving ODEs II.  ROS34PW2 (Rang
// and Angermann 2005) is a W-method, the paper's future work: its order
// conditions hold for any matrix in the place of J, so the Jacobian may be
// kept over several steps; it is published in the standard form and
// transformed here at compile time.  `elo` is the order of the estimate's
// leading term, the exponent of the step-size rule.
// `newf[i]` is 0 when stage i's argument equals stage i-1's (row i of a equal
// to row i-1), so that stage reuses the previous f.
#pragma once

namespace chem {

constexpr int MAX_STAGES = 6;

struct RosTable {
  int s;
  double gamma, elo;
  double a[MAX_STAGES][MAX_STAGES];
  double c[MAX_STAGES][MAX_STAGES];
  double m[MAX_STAGES];
  double e[MAX_STAGES];
  int newf[MAX_STAGES];
};

enum MethodId : int {
  METHOD_ROS4 = 0,
  METHOD_ROS3 = 1,
  METHOD_RODAS3 = 2,
  METHOD_RODAS4 = 3,
  METHOD_ROS34PW2 = 4,
  N_METHODS = 5
};

// A method in the standard form: alpha and gamma below the diagonal, gamma on
// it, weights b and embedded weights bhat.
struct RosStandard {
  int s;
  double gamma, elo;
  double alpha[MAX_STAGES][MAX_STAGES];
  double gam[MAX_STAGES][MAX_STAGES];
  double b[MAX_STAGES], bhat[MAX_STAGES];
};

// The transformed coefficients: Gamma^-1 column by column (forward
// substitution), then a = alpha Gamma^-1, c = -Gamma^-1 below the diagonal,
// m = b Gamma^-1, e = (b - bhat) Gamma^-1.
constexpr RosTable transform(const RosStandard& f) {
  RosTable t{};
  t.s = f.s;
  t.gamma = f.gamma;
  t.elo = f.elo;
  double gi[MAX_STAGES][MAX_STAGES] = {};
  for (int col = 0; col < f.s; ++col)
    for (int i = 0; i < f.s; ++i) {
      double r = (i == col) ? 1.0 : 0.0;
      for (int j = 0; j < i; ++j) r -= f.gam[i][j] * gi[j][col];
      gi[i][col] = r / f.gamma;
    }
  for (int i = 0; i < f.s; ++i)
    for (int j = 0; j < i; ++j) {
      double a = 0.0;
      for (int l = 0; l < f.s; ++l) a += f.alpha[i][l] * gi[l][j];
      t.a[i][j] = a;
      t.c[i][j] = -gi[i][j];
    }
  for (int j = 0; j < f.s; ++j) {
    double m = 0.0, e = 0.0;
    for (int l = 0; l < f.s; ++l) {
      m += f.b[l] * gi[l][j];
      e += (f.b[l] - f.bhat[l]) * gi[l][j];
    }
    t.m[j] = m;
    t.e[j] = e;
  }
  for (int i = 0; i < f.s; ++i) {
    bool same = i > 0;
    for (int j = 0; j < i && same; ++j) same = t.a[i][j] == (j < i - 1 ? t.a[i - 1][j] : 0.0);
    t.newf[i] = same ? 0 : 1;
  }
  return t;
}

// ROS34PW2, Rang and Angermann (2005): order 3, embedded 2, stiffly accurate.
constexpr RosStandard ROS34PW2_STD = {
    4, 0.435866521508459, 3.0,
    {{0}, {0.87173304301691801}, {0.84457060015369423, -0.11299064236484185}, {0.0, 0.0, 1.0}},
    {{0},
     {-0.87173304301691801},
     {-0.90338057013044082, 0.054180672388095326},
     {0.24212380706095346, -1.2232505839045147, 0.54526025533510214}},
    {0.24212380706095346, -1.2232505839045147, 1.5452602553351020, 0.435866521508459},
    {0.37810903145819369, -0.096042292212423178, 0.5, 0.2179332607542295}};

constexpr RosTable TABLES[N_METHODS] = {
    // ROS4, Hairer-Wanner L-stable set (gamma is the L-stable root 1/x2 of the
    // Laguerre polynomial L4, published to five digits)
    {4, 0.57282, 4.0,
     {{0}, {2.0}, {1.867943637803922, 0.2344449711399156},
      {1.867943637803922, 0.2344449711399156, 0.0}},
     {{0}, {-7.137615036412310}, {2.580708087951457, 0.6515950076447975},
      {-2.137148994382534, -0.3214669691237626, -0.6949742501781779}},
     {2.255570073418735, 0.2870493262186792, 0.4353179431840180, 1.093502252409163},
     {-0.2815431932141155, -0.07276199124938920, -0.1082196201495311, -1.093502252409163},
     {1, 1, 1, 0}},
    // ROS3, Sandu et al.
    {3, 0.43586652150845899941601945119356, 3.0,
     {{0}, {1.0}, {1.0, 0.0}},
     {{0}, {-1.0156171083877702091975600115545},
      {4.0759956452537699824805835358067, 9.2076794298330791242156818474003}},
     {1.0, 6.1697947043828245592553615689730, -0.42772256543218573326238373806514},
     {0.5, -2.9079558716805469821718236208017, 0.22354069897811569627360909276199},
     {1, 1, 0}},
    // RODAS3, Sandu et al. (stiffly accurate)
    {4, 0.5, 3.0,
     {{0}, {0.0}, {2.0, 0.0}, {2.0, 0.0, 1.0}},
     {{0}, {4.0}, {1.0, -1.0}, {1.0, -1.0, -8.0 / 3.0}},
     {2.0, 0.0, 1.0, 1.0},
     {0.0, 0.0, 0.0, 1.0},
     {1, 0, 1, 1}},
    // RODAS4, Hairer-Wanner (stiffly accurate, six stages)
    {6, 0.25, 4.0,
     {{0},
      {1.544},
      {0.9466785280815826, 0.2557011698983284},
      {3.314825187068521, 2.896124015972201, 0.9986419139977817},
      {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950},
      {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0}},
     {{0},
      {-5.6688},
      {-2.430093356833875, -0.2063599157091915},
      {-0.1073529058151375, -9.594562251023355, -20.47028614809616},
      {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160},
      {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
       -6.058818238834054}},
     {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 1.0},
     {0.0, 0.0, 0.0, 0.0, 0.0, 1.0},
     {1, 1, 1, 1, 1, 1}},
    transform(ROS34PW2_STD),
};

// ROS4 coefficients by name, for the discrete adjoint (which is written for
// ROS4's stage structure: four stages, the fourth reusing the third's f).
constexpr const RosTable& R4 = TABLES[METHOD_ROS4];
constexpr double ROS4_GAMMA = R4.gamma;
constexpr double ROS4_A21 = R4.a[1][0], ROS4_A31 = R4.a[2][0], ROS4_A32 = R4.a[2][1];
constexpr double ROS4_C21 = R4.c[1][0], ROS4_C31 = R4.c[2][0], ROS4_C32 = R4.c[2][1];
constexpr double ROS4_C41 = R4.c[3][0], ROS4_C42 = R4.c[3][1], ROS4_C43 = R4.c[3][2];
constexpr double ROS4_M1 = R4.m[0], ROS4_M2 = R4.m[1], ROS4_M3 = R4.m[2], ROS4_M4 = R4.m[3];
static_assert(R4.a[3][0] == R4.a[2][0] && R4.a[3][1] == R4.a[2][1] && R4.a[3][2] == 0.0,
              "the adjoint assumes ROS4's fourth stage reuses the third's argument");

}  // namespace chem
