// Host-side job lists of the step kernel: which output tiles a persistent
// step launch runs, in which order, on which XCD queue, and which of them
// run as K-split halves.  Pure host code (no HIP calls), shared by the
// runtime and its host-side tests.
#pragma once

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <queue>
#include <tuple>
#include <utility>
#include <vector>

#include "dmpt_internal.h"

namespace dmpt {

constexpr int kMaxSplit = 256;   // K-split tail tiles per job list at most

// Job list over the step tiles (I, J), J >= 2I.  Z-jobs (the heavier
// products) come first, then P-jobs.  Within a kind the tiles are cut into
// groups of kGroupI x kGroupJ neighbouring tiles (a group shares kGroupI
// 256-row A panels and kGroupJ 128-row B panels; groups on the diagonal are
// the upper-triangle part of their square, 20 tiles), and whole groups are
// dealt to the eight XCDs: position p of the list belongs to the queue of XCD
// p % 8, from which the step kernel's workgroups on that XCD take their tiles
// in order.  One XCD holds 32 resident workgroups, so a full group keeps them
// streaming the same panels through its L2.  Full groups go first in every
// queue and are dealt to the queue with the fewest tiles; the partial diagonal
// groups close the queues.
constexpr int kXcds = 8, kGroupI = 4, kGroupJ = 8;

inline std::vector<std::vector<std::pair<int, int>>> tile_groups(int n_pad) {
  const int tr = n_pad / kStepTM, tc = n_pad / kStepTN;
  std::vector<std::vector<std::pair<int, int>>> full, part;
  for (int gi = 0; gi < tr; gi += kGroupI)
    for (int gj = 0; gj < tc; gj += kGroupJ) {
      std::vector<std::pair<int, int>> g;
      for (int i = gi; i < std::min(tr, gi + kGroupI); ++i)
        for (int j = std::max(gj, 2 * i); j < std::min(tc, gj + kGroupJ); ++j) g.emplace_back(i, j);
      if (g.empty()) continue;
      (g.size() == (size_t)(kGroupI * kGroupJ) ? full : part).push_back(std::move(g));
    }
  full.insert(full.end(), part.begin(), part.end());
  return full;
}

inline void append_xcd_ordered(std::vector<uint32_t>& out, const std::vector<std::vector<uint32_t>>& groups) {
  std::vector<std::vector<uint32_t>> q(kXcds);
  size_t total = 0;
  for (const auto& g : groups) {
    int x = 0;
    for (int y = 1; y < kXcds; ++y)
      if (q[y].size() < q[x].size()) x = y;
    q[x].insert(q[x].end(), g.begin(), g.end());
    total += g.size();
  }
  std::vector<size_t> head(kXcds, 0);
  for (size_t left = total; left > 0; --left) {
    int x = (int)(out.size() % kXcds);
    if (head[x] == q[x].size()) {   // this XCD's queue ran dry: take from the longest one
      size_t best = 0;
      for (int y = 0; y < kXcds; ++y)
        if (q[y].size() - head[y] > best) { best = q[y].size() - head[y]; x = y; }
    }
    out.push_back(q[x][head[x]++]);
  }
}

inline std::vector<uint32_t> build_jobs(int n_pad, int nobs_z, bool with_p) {
  const auto groups = tile_groups(n_pad);
  std::vector<uint32_t> out;
  std::vector<std::vector<uint32_t>> kg(groups.size());
  auto add_kind = [&](int kind, int obs) {
    for (size_t g = 0; g < groups.size(); ++g) {
      kg[g].clear();
      for (const auto& t : groups[g]) kg[g].push_back(job_pack(kind, obs, t.first, t.second));
    }
    append_xcd_ordered(out, kg);
  };
  for (int k = 0; k < nobs_z; ++k) add_kind(kJobZ, k);
  if (with_p) add_kind(kJobP, 0);
  return out;
}

// Sweep-product jobs (Z-jobs) with 256 x 256 output tiles (kJobWide): tile
// (I, J), J >= I, on the 256 grid covers the regular tiles (I, 2J) and
// (I, 2J + 1), and a 4 x 4 group of them the regular 4 x 8 group, so the
// groups above are reused: a group is either wide as a whole or regular.
// A wide tile streams two 256-row panels per stage where a regular one
// streams 256 + 128 rows for half the products: a third fewer bytes and LDS
// reads per unit of work.  Measured on MI355X at N = 8192 (Z-only launches
// of 1056 regular, 528 wide tiles; two-term and plain BF16 alike), a wide
// tile takes 1.6 - 1.7 times a regular one, and a P-job of the three-term
// split about as long as a regular Z-job.
constexpr double kWideCost = 1.65;
// K-split tail: the last regular tiles of a list run as two half-K jobs (cost
// in regular-tile units, with the partial-sum store) and a combine launch
// adds the halves and runs their epilogue (a fixed cost per launch).
constexpr double kHalfCost = 0.53, kCombineCost = 0.08;

inline std::vector<uint32_t> wide_group(const std::vector<std::pair<int, int>>& g, int obs) {
  std::vector<uint32_t> w;
  for (const auto& t : g) {
    if (t.second & 1) continue;   // (I, 2J + 1) belongs to the wide tile of (I, 2J)
    w.push_back(job_pack(kJobZ, obs, t.first, t.second / 2) | kJobWide);
  }
  // a diagonal group's (I, 2I + 1) has its partner (I, 2I) in the list: no tile is lost
  return w;
}

// List scheduling of a persistent launch: jobs are dealt in order to `cus`
// workgroups, each taking the next job when it is free; times in
// regular-tile units.
struct ListSim {
  std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
  double end = 0.0;   // the makespan so far
  explicit ListSim(int cus) {
    for (int c = 0; c < cus; ++c) free_at.push(0.0);
  }
  void add(double cost) {
    const double t = free_at.top() + cost;
    free_at.pop();
    free_at.push(t);
    end = std::max(end, t);
  }
};

// Best K-split tail for a list of job costs: the last k regular tiles (k a
// multiple of 8, at most kMaxSplit, only from the trailing run of regular
// tiles) become 2k half-K jobs, plus the combine launch; returns the modelled
// makespan and k (0: no split; on a tie the smaller k).  Every candidate
// shares the jobs before the tail, so the schedule of that prefix is
// simulated once and extended by 8 jobs per candidate.
inline std::pair<double, int> best_split(const std::vector<double>& base, int cus) {
  int trailing = 0;
  for (size_t q = base.size(); q > 0 && base[q - 1] == 1.0; --q) ++trailing;
  const int kmax = std::min(kMaxSplit, trailing) / 8 * 8;
  ListSim sim(cus);
  size_t pos = 0;
  for (; pos < base.size() - (size_t)kmax; ++pos) sim.add(base[pos]);
  std::vector<double> t(kmax / 8 + 1);   // t[k / 8]: modelled makespan with k split tiles
  for (int k = kmax; k >= 0; k -= 8) {   // the simulated prefix is base[0, size - k)
    if (k > 0) {
      ListSim tail = sim;
      for (int h = 0; h < 2 * k; ++h) tail.add(kHalfCost);
      t[k / 8] = tail.end + kCombineCost;
    } else {
      t[0] = sim.end;
    }
    for (int r = 0; r < 8 && pos < base.size(); ++r) sim.add(base[pos++]);
  }
  std::pair<double, int> best(t[0], 0);
  for (int k = 8; k <= kmax; k += 8)
    if (t[k / 8] < best.first - 1e-9) best = {t[k / 8], k};
  return best;
}

// A step-launch list on 256 x 256 sweep tiles: the Z-jobs of nobs
// observables (leading groups wide, the rest regular), then, with with_p, the
// P-jobs (regular), then the K-split tail (see kJobSplit): the last k regular
// tiles as pairs of half-K jobs with their scratch slots (slots: the slot of
// every list position; cjobs: the tile of each slot).  The number of wide
// groups and k together minimise the launch's modelled makespan on `cus`
// workgroups.
struct JobList {
  std::vector<uint32_t> jobs, slots, cjobs;
};

inline JobList build_wide_list(int n_pad, int nobs, bool with_p, int cus) {
  const auto groups = tile_groups(n_pad);
  const std::vector<uint32_t> pj = with_p ? build_jobs(n_pad, 0, true) : std::vector<uint32_t>();
  std::vector<std::pair<int, size_t>> order;   // (obs, group)
  for (int k = 0; k < nobs; ++k)
    for (size_t g = 0; g < groups.size(); ++g) order.emplace_back(k, g);
  size_t best_w = 0;
  int best_k = 0;
  {
    double best = 0.0;
    std::vector<size_t> cand;   // many observables: a coarse search
    const size_t stride = std::max<size_t>(1, order.size() / 64);
    for (size_t nw = 0; nw < order.size(); nw += stride) cand.push_back(nw);
    cand.push_back(order.size());
    for (size_t nw : cand) {
      std::vector<double> c;
      for (size_t q = 0; q < nw; ++q)
        c.insert(c.end(), (groups[order[q].second].size() + 1) / 2, kWideCost);
      for (size_t q = nw; q < order.size(); ++q) c.insert(c.end(), groups[order[q].second].size(), 1.0);
      c.insert(c.end(), pj.size(), 1.0);
      const auto t = best_split(c, cus);
      if (nw == 0 || t.first < best - 1e-9) { best = t.first; best_w = nw; best_k = t.second; }
    }
  }
  JobList L;
  std::vector<std::vector<uint32_t>> wg, rg;
  for (size_t q = 0; q < order.size(); ++q) {
    const auto& g = groups[order[q].second];
    if (q < best_w) {
      wg.push_back(wide_group(g, order[q].first));
    } else {
      std::vector<uint32_t> r;
      for (const auto& t : g) r.push_back(job_pack(kJobZ, order[q].first, t.first, t.second));
      rg.push_back(std::move(r));
    }
  }
  append_xcd_ordered(L.jobs, wg);
  append_xcd_ordered(L.jobs, rg);
  L.jobs.insert(L.jobs.end(), pj.begin(), pj.end());
  // the tail: the last best_k regular tiles, re-appended as half pairs
  std::vector<uint32_t> tail(L.jobs.end() - best_k, L.jobs.end());
  L.jobs.resize(L.jobs.size() - best_k);
  L.slots.assign(L.jobs.size() + 2 * (size_t)best_k, 0u);
  for (int i = 0; i < best_k; ++i) {
    L.cjobs.push_back(tail[i]);
    L.slots[L.jobs.size()] = (uint32_t)i;
    L.jobs.push_back(tail[i] | kJobSplit);
    L.slots[L.jobs.size()] = (uint32_t)i;
    L.jobs.push_back(tail[i] | kJobSplit | kJobHalf1);
  }
  return L;
}

// The lists depend only on the shape; the search runs once per shape and
// process (the modelled makespans take milliseconds of host time).
inline const JobList& cached_wide_list(int n_pad, int nobs, bool with_p, int cus) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, bool, int>, JobList> cache;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(n_pad, nobs, with_p, cus);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, build_wide_list(n_pad, nobs, with_p, cus)).first;
  return it->second;
}

}  // namespace dmpt
