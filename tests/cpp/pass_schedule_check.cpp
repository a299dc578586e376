// Invariants of the pass scheduler (schedule_passes) on random pair lists,
// one and two atoms per lane: every pair in exactly one slot of a pass of
// the group width; within a pass each atom is the first endpoint of at most
// cap/2 slots and the second of at most cap/2; each atom's pull list names
// exactly those slots (first half added, second half subtracted) and the
// zero entry elsewhere; the cap is one the kernel reads.  Prints the number
// of violations and the pass count against ceil(P / width); exits nonzero on
// any violation.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include "dock_internal.h"
using namespace dock;
int main() {
  std::mt19937 rng(1);
  int bad = 0;
  long tot_pass = 0, tot_min = 0;
  for (int trial = 0; trial < 3000; ++trial) {
    const int apl = 1 + trial % 2;
    const int n = apl == 1 ? 2 + rng() % 63 : 2 + rng() % 127;
    const int width = apl == 1 ? (n <= 16 ? 16 : (n <= 32 ? 32 : 64)) : (n <= 32 ? 16 : (n <= 64 ? 32 : 64));
    std::vector<int> pi, pj;
    const double dens = (rng() % 100) / 100.0;
    const bool hub = rng() % 5 == 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j)
        if ((rng() % 1000) < dens * 1000 || (hub && i == 0)) { pi.push_back(i); pj.push_back(j); }
    const PassPlan pl = schedule_passes(n, pi, pj, width, apl);
    if (pi.empty()) { if (pl.n_pass != 0) bad++; continue; }
    if (int(pl.slot_i.size()) != pl.n_pass * width || pl.n_pull != apl * width ||
        int(pl.pulls.size()) != pl.n_pass * pl.n_pull) { bad++; continue; }
    const int half = pl.cap / 2;
    std::multiset<std::pair<int,int>> want, got;
    for (size_t p = 0; p < pi.size(); ++p) want.insert({pi[p], pj[p]});
    for (int ps = 0; ps < pl.n_pass; ++ps) {
      std::vector<std::vector<int>> plus(n), minus(n);
      for (int s = 0; s < width; ++s) {
        const int a = pl.slot_i[ps * width + s], b = pl.slot_j[ps * width + s];
        if (a < 0) { if (b >= 0) bad++; continue; }
        got.insert({std::min(a, b), std::max(a, b)});
        plus[a].push_back(s); minus[b].push_back(s);
      }
      for (int a = 0; a < n; ++a) {
        if (int(plus[a].size()) > half || int(minus[a].size()) > half || pl.cap > kMaxPull || (apl == 2 && pl.cap > 4) || (pl.cap != 2 && pl.cap != 4 && pl.cap != 8)) bad++;
        uint64_t w = pl.pulls[ps * pl.n_pull + a];
        std::vector<int> dp, dm;
        for (int c = 0; c < 8; ++c) {
          int e = (w >> (8 * c)) & 0xff;
          if (e == width) continue;
          if (e > width || c >= pl.cap) { bad++; continue; }
          (c < half ? dp : dm).push_back(e);
        }
        if (dp != plus[a] || dm != minus[a]) bad++;
        // zero entries only after the used ones within each half
        for (int c = 0; c < pl.cap; ++c) {
          int e = (w >> (8 * c)) & 0xff;
          int k = c < half ? c : c - half;
          int cnt = c < half ? int(plus[a].size()) : int(minus[a].size());
          if ((k < cnt) != (e != width)) bad++;
        }
      }
      for (int a = n; a < pl.n_pull; ++a) if (pl.pulls[ps * pl.n_pull + a] != uint64_t(width) * 0x0101010101010101ull) bad++;
    }
    if (want != got) bad++;
    tot_pass += pl.n_pass;
    tot_min += (pi.size() + width - 1) / width;
  }
  printf("bad %d passes %ld minimal %ld\n", bad, tot_pass, tot_min);
  return bad != 0;
}
