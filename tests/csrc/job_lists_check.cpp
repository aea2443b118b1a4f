// Host-side check of the step kernel's job lists (dmpt_lists.h): for each
// shape given on the command line, every output tile of a step launch runs
// exactly once (as a regular job, inside a 256 x 256 wide job, or as the two
// K-split halves of one scratch slot), no tile outside the upper triangle
// is listed, and the lists fit the workspace the runtime reserves for them.
// Usage: job_lists_check n_pad:nobs:with_p[:cus] ...  Prints one line per
// shape and exits non-zero on the first violation.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "dmpt_lists.h"

using namespace dmpt;

namespace {

struct Tile {
  int kind, obs, i, j;
  bool operator<(const Tile& o) const { return std::tie(kind, obs, i, j) < std::tie(o.kind, o.obs, o.i, o.j); }
  bool operator==(const Tile& o) const { return std::tie(kind, obs, i, j) == std::tie(o.kind, o.obs, o.i, o.j); }
};

int fails = 0;

void check(bool ok, const char* what, int n_pad, int nobs, int with_p) {
  if (ok) return;
  std::printf("FAIL n_pad=%d nobs=%d with_p=%d: %s\n", n_pad, nobs, with_p, what);
  ++fails;
}

// Tiles a list covers, each with its multiplicity; false on a malformed job.
bool cover(const std::vector<uint32_t>& jobs, const std::vector<uint32_t>* slots,
           const std::vector<uint32_t>* cjobs, std::multiset<Tile>& out, std::string& why) {
  std::vector<int> halves(cjobs ? cjobs->size() * 2 : 0, 0);
  for (size_t q = 0; q < jobs.size(); ++q) {
    const uint32_t job = jobs[q];
    const int kind = (int)(job & 1u), obs = (int)((job >> 1) & 63u);
    const int ti = (int)((job >> 8) & 4095u), tj = (int)((job >> 20) & 2047u);
    if (job & kJobSplit) {
      if (!slots || !cjobs || q >= slots->size()) { why = "split job without a slot"; return false; }
      const uint32_t slot = (*slots)[q];
      if (slot >= cjobs->size()) { why = "split slot out of range"; return false; }
      if ((job & ~(kJobSplit | kJobHalf1)) != (*cjobs)[slot]) { why = "split job differs from its slot's tile"; return false; }
      ++halves[slot * 2 + ((job & kJobHalf1) ? 1 : 0)];
      if (!(job & kJobHalf1)) out.insert({kind, obs, ti, tj});   // the tile counts once, with its first half
    } else if (kind == kJobZ && (job & kJobWide)) {
      if (tj < ti) { why = "wide tile below the diagonal"; return false; }
      out.insert({kind, obs, ti, 2 * tj});
      out.insert({kind, obs, ti, 2 * tj + 1});
    } else {
      if (job & kJobWide) { why = "wide bit on a P-job"; return false; }
      out.insert({kind, obs, ti, tj});
    }
  }
  for (size_t h = 0; h < halves.size(); ++h)
    if (halves[h] != 1) { why = "a split slot does not have exactly one job per half"; return false; }
  return true;
}

std::multiset<Tile> expected(int n_pad, int nobs, bool with_p) {
  std::multiset<Tile> e;
  const int tr = n_pad / kStepTM, tc = n_pad / kStepTN;
  for (int k = 0; k < nobs; ++k)
    for (int i = 0; i < tr; ++i)
      for (int j = 2 * i; j < tc; ++j) e.insert({kJobZ, k, i, j});
  if (with_p)
    for (int i = 0; i < tr; ++i)
      for (int j = 2 * i; j < tc; ++j) e.insert({kJobP, 0, i, j});
  return e;
}

}  // namespace

int main(int argc, char** argv) {
  for (int a = 1; a < argc; ++a) {
    int n_pad = 0, nobs = 0, with_p = 0, cus = 256;
    if (std::sscanf(argv[a], "%d:%d:%d:%d", &n_pad, &nobs, &with_p, &cus) < 3 || n_pad % kStepTM) {
      std::printf("bad shape %s\n", argv[a]);
      return 2;
    }
    const int ut = step_tile_count(n_pad);
    const std::multiset<Tile> want = expected(n_pad, nobs, with_p != 0);
    std::string why;
    // the regular list of a step launch (no wide or split jobs)
    {
      const std::vector<uint32_t> jobs = build_jobs(n_pad, nobs, with_p != 0);
      std::multiset<Tile> got;
      check(cover(jobs, nullptr, nullptr, got, why), why.c_str(), n_pad, nobs, with_p);
      check(got == want, "regular list: tiles not covered exactly once", n_pad, nobs, with_p);
      check((int)jobs.size() <= ut * (1 + nobs), "regular list longer than its workspace", n_pad, nobs, with_p);
    }
    // the list with wide sweep tiles and a K-split tail
    const auto t0 = std::chrono::steady_clock::now();
    const JobList& L = cached_wide_list(n_pad, nobs, with_p != 0, cus);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::multiset<Tile> got;
    check(L.slots.size() == L.jobs.size(), "slot table and list differ in length", n_pad, nobs, with_p);
    check(cover(L.jobs, &L.slots, &L.cjobs, got, why), why.c_str(), n_pad, nobs, with_p);
    check(got == want, "wide list: tiles not covered exactly once", n_pad, nobs, with_p);
    check((int)L.cjobs.size() <= kMaxSplit, "more split tiles than the scratch holds", n_pad, nobs, with_p);
    const int cap = with_p ? ut * (1 + nobs) + kMaxSplit : ut * std::max(nobs, 1) + kMaxSplit;
    check((int)L.jobs.size() <= cap, "wide list longer than its workspace", n_pad, nobs, with_p);
    int wide = 0;
    for (uint32_t j : L.jobs) wide += !(j & kJobSplit) && (j & 1u) && (j & kJobWide);
    std::printf("n_pad=%d nobs=%d with_p=%d cus=%d: %zu jobs, %d wide, %zu split tiles, built in %.1f ms\n", n_pad,
                nobs, with_p, cus, L.jobs.size(), wide, L.cjobs.size(), ms);
    if (fails) return 1;
  }
  return 0;
}
