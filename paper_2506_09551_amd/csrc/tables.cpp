// Per-spin basis and hopping tables (host side).
//
// For one spin species with N electrons on L sites the configurations are the
// L-bit integers with N set bits, in ascending order.  Every bond (i, j) of
// the model (Sec. III, Eq. Hubbard) moves one electron between i and j; the
// matrix element of -t (c+_i c_j + c+_j c_i) between configurations c and c'
// is -t times the Jordan-Wigner parity (-1)^{#occupied sites strictly between
// i and j}.  With all spin-up operators ordered before all spin-down
// operators, a hop of either species picks up no sign from the other species,
// which is what makes the Kronecker form H_up (x) I + I (x) H_dn exact.
#include <algorithm>
#include <string>
#include <vector>

#include "msb_internal.h"

namespace msb {

bool build_spin_table(int L, int N, const std::vector<int>& bi, const std::vector<int>& bj,
                      const std::vector<int>& bt_fwd, const std::vector<int>& bt_bwd, SpinTable& out,
                      std::string& err) {
  if (L < 1 || L > 20 || N < 0 || N > L) {
    err = "spin table: need 1 <= L <= 20 and 0 <= N <= L";
    return false;
  }
  out = SpinTable();
  out.L = L;
  out.N = N;
  const uint32_t full = 1u << L;
  std::vector<int32_t> rank(full, -1);
  for (uint32_t c = 0; c < full; ++c) {
    if (__builtin_popcount(c) == N) {
      rank[c] = (int32_t)out.conf.size();
      out.conf.push_back(c);
    }
  }
  out.n = (int)out.conf.size();
  if (out.n > 65535) {
    err = "spin table: more than 65535 configurations per spin";
    return false;
  }
  out.off.assign(out.n + 1, 0);
  out.hop.clear();
  for (int r = 0; r < out.n; ++r) {
    const uint32_t c = out.conf[r];
    std::vector<uint32_t> row;
    for (size_t b = 0; b < bi.size(); ++b) {
      const int i = bi[b], j = bj[b];
      const bool oi = (c >> i) & 1u, oj = (c >> j) & 1u;
      if (oi == oj) continue;                       // nothing to hop
      const uint32_t c2 = c ^ (1u << i) ^ (1u << j);
      const int lo = std::min(i, j), hi = std::max(i, j);
      const uint32_t between = (hi - lo > 1) ? (((1u << hi) - 1u) & ~((1u << (lo + 1)) - 1u)) : 0u;
      const uint32_t neg = __builtin_popcount(c & between) & 1u;
      const int32_t r2 = rank[c2];
      // row c, column c2: the electron ends on j (hop i -> j) when j is
      // occupied in c, on i (hop j -> i) otherwise
      const int type = oj ? bt_fwd[b] : bt_bwd[b];
      row.push_back(((uint32_t)r2 << 16) | ((uint32_t)type << 1) | neg);
    }
    // Deterministic order: by target rank, then type.
    std::sort(row.begin(), row.end());
    out.max_hops = std::max(out.max_hops, (int)row.size());
    out.hop.insert(out.hop.end(), row.begin(), row.end());
    out.off[r + 1] = (uint32_t)out.hop.size();
  }
  // Level order: a hop between sites i and i+1 changes the sum of the
  // occupied site indices by one, so on chains most hops join neighbouring
  // levels; walking the rows level by level keeps a row's neighbours close
  // in time (the apply kernel can use it for cache reuse).
  std::vector<std::pair<int, uint32_t>> lev(out.n);
  for (int r = 0; r < out.n; ++r) {
    int s = 0;
    for (int i = 0; i < L; ++i) s += ((out.conf[r] >> i) & 1u) ? i : 0;
    lev[r] = {s, (uint32_t)r};
  }
  std::sort(lev.begin(), lev.end());
  out.order.resize(out.n);
  for (int r = 0; r < out.n; ++r) out.order[r] = lev[r].second;
  return true;
}

}  // namespace msb
