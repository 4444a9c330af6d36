// Mechanism tables: host-side parse result and the device view the kernels read.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace chem {

constexpr double RU = 8314.462618;  // J/(kmol K)
constexpr double PATM = 101325.0;   // Pa
constexpr int MAX_SPECIES = 255;
constexpr int MAX_REACTIONS = 4095;
constexpr int MAX_SIDE = 3;         // species per reaction side

enum RxnType : int32_t { RX_ELEM = 0, RX_THIRD = 1, RX_LIND = 2, RX_TROE = 3 };

// Device view of a mechanism.  All arrays are device pointers into one blob
// (each array 256-byte aligned and followed by at least 256 zero bytes, so a
// read just past an array's end stays in the blob).
// A reaction's fields sit in a few per-reaction records (info, species,
// coefficients, Arrhenius).  The one-cell-per-thread kernel reads them at a
// wavefront-uniform reaction index (scalar loads); the one-wavefront-per-cell
// kernels put one reaction on each lane, so neighbouring lanes read
// neighbouring records.
struct MechView {
  int32_t K, Nr, N;          // species, reactions, state size K + 1
  const double* W;           // [K]
  const double* nasa;        // [K][15]: T_mid, a_lo[7], a_hi[7]
  const int32_t* rinfo;      // [Nr][8]: type, nr, np, eff_begin, eff_end, fo_index, 0, 0
  const int32_t* rspec;      // [Nr][6]: reactant idx x3, product idx x3 (unused = 0)
  const int32_t* rnu;        // [Nr][6]: coefficients (unused = 0)
  const double* arr;         // [Nr][4]: lnA, b, theta, sum(nu)
  const int32_t* eff_idx;    // [n_eff]
  const double* eff_am1;     // [n_eff]: alpha - 1
  const double* fo;          // [n_fo][8]: lnA0 - lnA, b0, theta0, a, T3, T1, T2, 0
  const int32_t* rorig;      // [Nr]: file index of internal reaction j (ln A override, gradients)
};

struct HostMech {
  int32_t K = 0, Nr = 0, E = 0;
  std::vector<std::string> names;
  std::vector<double> W, nasa;
  std::vector<int32_t> comp;
  std::vector<int32_t> rinfo, rspec, rnu, eff_idx;
  std::vector<double> arr, eff_am1, fo;
  std::vector<int32_t> rorig;   // file index of internal reaction j
};

// Groups reactions by type (elementary, third body, Lindemann, Troe) keeping
// file order inside a group, so that the lanes of a wavefront walking the
// reaction list mostly take the same branch.  rorig records the permutation.
void group_reactions_by_type(HostMech& m);

// Returns 0, or a CHEM_E* code.
int parse_mechanism(const char* path, HostMech& m);

}  // namespace chem
