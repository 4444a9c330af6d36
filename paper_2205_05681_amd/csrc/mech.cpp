// Text mechanism parser (host).  The format is line oriented:
//   CHEMMECH 1
//   ELEMENTS <E> <symbols>
//   SPECIES <K>
//   <name> <W> <E counts> <T_mid> <a_lo x7> <a_hi x7>
//   REACTIONS <Nr>
//   <E|T|L|F> <nr> (<i> <nu>)x nr <np> (<i> <nu>)x np <lnA> <b> <theta>
//             <neff> (<i> <alpha>)x neff [<lnA0> <b0> <theta0>] [<a> <T3> <T1> <T2>]
// SI units (kmol, m3, s, K); theta = Ea / R.
#include "mech.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <tuple>

#include "../../include/chem.h"

namespace chem {

namespace {
bool expect(std::istream& in, const char* word) {
  std::string t;
  return (in >> t) && t == word;
}
}  // namespace

int parse_mechanism(const char* path, HostMech& m) {
  std::ifstream in(path);
  if (!in) return CHEM_EPARSE;
  int version = 0;
  if (!expect(in, "CHEMMECH") || !(in >> version) || version != 1) return CHEM_EPARSE;
  if (!expect(in, "ELEMENTS") || !(in >> m.E) || m.E < 0 || m.E > 64) return CHEM_EPARSE;
  for (int e = 0; e < m.E; ++e) {
    std::string s;
    if (!(in >> s)) return CHEM_EPARSE;
  }
  if (!expect(in, "SPECIES") || !(in >> m.K) || m.K < 2) return CHEM_EPARSE;
  if (m.K > MAX_SPECIES) return CHEM_EUNSUPPORTED;
  m.names.resize(m.K);
  m.W.resize(m.K);
  m.comp.resize((size_t)m.K * m.E);
  m.nasa.resize((size_t)m.K * 15);
  for (int k = 0; k < m.K; ++k) {
    if (!(in >> m.names[k] >> m.W[k])) return CHEM_EPARSE;
    for (int e = 0; e < m.E; ++e)
      if (!(in >> m.comp[(size_t)k * m.E + e])) return CHEM_EPARSE;
    for (int i = 0; i < 15; ++i)
      if (!(in >> m.nasa[(size_t)k * 15 + i])) return CHEM_EPARSE;
    if (!(m.W[k] > 0)) return CHEM_EPARSE;
  }
  if (!expect(in, "REACTIONS") || !(in >> m.Nr) || m.Nr < 0) return CHEM_EPARSE;
  if (m.Nr > MAX_REACTIONS) return CHEM_EUNSUPPORTED;
  m.rinfo.assign((size_t)m.Nr * 8, 0);
  m.rspec.assign((size_t)m.Nr * 6, 0);
  m.rnu.assign((size_t)m.Nr * 6, 0);
  m.arr.assign((size_t)m.Nr * 4, 0.0);
  for (int j = 0; j < m.Nr; ++j) {
    std::string kind;
    if (!(in >> kind) || kind.size() != 1) return CHEM_EPARSE;
    int type;
    switch (kind[0]) {
      case 'E': type = RX_ELEM; break;
      case 'T': type = RX_THIRD; break;
      case 'L': type = RX_LIND; break;
      case 'F': type = RX_TROE; break;
      default: return CHEM_EPARSE;
    }
    int32_t* info = &m.rinfo[(size_t)j * 8];
    info[0] = type;
    double dnu = 0;
    for (int side = 0; side < 2; ++side) {
      int cnt;
      if (!(in >> cnt) || cnt < 0) return CHEM_EPARSE;
      if (cnt > MAX_SIDE) return CHEM_EUNSUPPORTED;
      info[1 + side] = cnt;
      for (int i = 0; i < cnt; ++i) {
        int idx, nu;
        if (!(in >> idx >> nu)) return CHEM_EPARSE;
        if (idx < 0 || idx >= m.K || nu < 1 || nu > 3) return CHEM_EPARSE;
        m.rspec[(size_t)j * 6 + side * 3 + i] = idx;
        m.rnu[(size_t)j * 6 + side * 3 + i] = nu;
        dnu += side ? nu : -nu;
      }
    }
    double* a = &m.arr[(size_t)j * 4];
    if (!(in >> a[0] >> a[1] >> a[2])) return CHEM_EPARSE;
    a[3] = dnu;
    int neff;
    if (!(in >> neff) || neff < 0 || neff > m.K) return CHEM_EPARSE;
    info[3] = (int32_t)m.eff_idx.size();
    for (int i = 0; i < neff; ++i) {
      int idx;
      double alpha;
      if (!(in >> idx >> alpha) || idx < 0 || idx >= m.K) return CHEM_EPARSE;
      m.eff_idx.push_back(idx);
      m.eff_am1.push_back(alpha - 1.0);
    }
    info[4] = (int32_t)m.eff_idx.size();
    info[5] = -1;
    if (type == RX_LIND || type == RX_TROE) {
      double lnA0, b0, th0;
      if (!(in >> lnA0 >> b0 >> th0)) return CHEM_EPARSE;
      double f[8] = {lnA0 - a[0], b0, th0, 0, 1, 1, 0, 0};
      if (type == RX_TROE) {
        if (!(in >> f[3] >> f[4] >> f[5] >> f[6])) return CHEM_EPARSE;
        if (!(f[4] > 0) || !(f[5] > 0) || f[6] < 0) return CHEM_EPARSE;
      }
      info[5] = (int32_t)(m.fo.size() / 8);
      m.fo.insert(m.fo.end(), f, f + 8);
    }
  }
  if (in.fail()) return CHEM_EPARSE;
  m.rorig.resize(m.Nr);
  for (int j = 0; j < m.Nr; ++j) m.rorig[j] = j;
  return CHEM_OK;
}

void group_reactions_by_type(HostMech& m) {
  // by type, then by the number of participants (reactants + products,
  // then reactants), file order within: the lanes of a wavefront then mostly
  // use the same species slots
  std::vector<int32_t> order(m.Nr);
  for (int j = 0; j < m.Nr; ++j) order[j] = j;
  auto key = [&](int j) {
    const int32_t* in = &m.rinfo[(size_t)j * 8];
    return std::make_tuple(in[0], in[1] + in[2], in[1]);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
  HostMech r = m;
  for (int jn = 0; jn < m.Nr; ++jn) {
    const int j = order[jn];
    for (int i = 0; i < 8; ++i) r.rinfo[(size_t)jn * 8 + i] = m.rinfo[(size_t)j * 8 + i];
    for (int i = 0; i < 6; ++i) r.rspec[(size_t)jn * 6 + i] = m.rspec[(size_t)j * 6 + i];
    for (int i = 0; i < 6; ++i) r.rnu[(size_t)jn * 6 + i] = m.rnu[(size_t)j * 6 + i];
    for (int i = 0; i < 4; ++i) r.arr[(size_t)jn * 4 + i] = m.arr[(size_t)j * 4 + i];
  }
  r.rorig = order;
  m = r;
}

}  // namespace chem
