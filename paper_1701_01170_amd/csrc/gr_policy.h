// Per-iteration strategy selection (host side).
//
// The heuristic follows Sec. 5.1: merge-based load balancing (LB) when the
// graph's average degree is at least lb_min_avg_degree (paper: 5), dynamic
// grouping (TWC) otherwise; inside LB, input-frontier balance below
// lb_light_threshold frontier vertices (paper: 4096).  The push/pull
// direction switches push -> pull when m_f > m_u * do_a and pull -> push when
// m_f < m_u * do_b (Sec. 5.1, push vs. pull).  m_f and m_u are exact here (the
// frontier statistics kernel sums frontier degrees; the unvisited degree sum
// is kept by subtraction) instead of the paper's average-degree estimates.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "gr.h"

namespace gr {

struct LevelFeatures {
  int32_t level = 0;
  int64_t V = 0, E = 0;
  int64_t n_f = 0, m_f = 0, n_u = 0, m_u = 0, max_deg_f = 0;
  int32_t prev_pull = 0;  // the previous step pulled (the unvisited frontier exists)
  int32_t ms_k = 0;       // batched traversal: its number of sources (0: single source)
};

// The eight selector inputs, each log2(1 + x) / 32:
//   n_f, m_f, n_u, m_u, max frontier degree, V, E, and the size of the
//   unvisited-frontier generation a pull step would need now (V after a push
//   step, 0 after a pull step) -- for a batched traversal instead its number
//   of sources.
inline void selector_features(const LevelFeatures& lf, float out[8]) {
  auto f = [](double x) { return (float)(std::log2(1.0 + (x > 0 ? x : 0.0)) / 32.0); };
  out[0] = f((double)lf.n_f);
  out[1] = f((double)lf.m_f);
  out[2] = f((double)lf.n_u);
  out[3] = f((double)lf.m_u);
  out[4] = f((double)lf.max_deg_f);
  out[5] = f((double)lf.V);
  out[6] = f((double)lf.E);
  out[7] = lf.ms_k > 0 ? f((double)lf.ms_k) : f(lf.prev_pull ? 0.0 : (double)lf.V);
}

struct Selector {
  gr_opts o{};
  bool pull_ok = false;
  bool sssp = false;
  bool learned = false;
  bool mode_pull = false;
  int last_heuristic = -1;  // the heuristic's action at the last decide() (learned policy)
  uint64_t rng = 0;
  double avg_degree = 0.0;

  void init(const gr_opts& opts, int64_t V, int64_t E, bool pull_allowed, bool is_sssp,
            bool have_learned) {
    o = opts;
    pull_ok = pull_allowed && !is_sssp;
    sssp = is_sssp;
    learned = have_learned && opts.policy == GR_POLICY_LEARNED;
    mode_pull = false;
    rng = opts.policy_seed ^ 0x9e3779b97f4a7c15ull;
    avg_degree = V > 0 ? (double)E / (double)V : 0.0;
  }

  static uint64_t next(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }

  int heuristic(const LevelFeatures& lf) const {
    bool pull = mode_pull;
    if (pull_ok) {
      if (!mode_pull) {
        if ((double)lf.m_f > (double)lf.m_u * (double)o.do_a) pull = true;
      } else {
        if ((double)lf.m_f < (double)lf.m_u * (double)o.do_b) pull = false;
      }
    }
    // The paper has a single pull advance; its early exit makes per-vertex
    // dynamic grouping the natural mapping, so the heuristic pulls with TWC.
    if (pull) return GR_PULL_TWC;
    return push_action();
  }

  int push_action() const {
    return avg_degree >= (double)o.lb_min_avg_degree ? GR_PUSH_LB : GR_PUSH_TWC;
  }

  // device_choice: the network's argmin over the allowed actions, pred: its
  // predicted log2 step times (both from the device; -1 / null when none).
  // The learned policy is guarded: it keeps the heuristic's action unless the
  // network predicts its own choice faster by more than o.learned_margin.
  // keep_push: the level fits a block of device-predicated push levels, which
  // makes pushing it far cheaper than a level with its own host round trip
  // (the tail levels of a direction-optimised BFS stay in pull mode, since
  // m_f < m_u * do_b rarely holds once few vertices are left, and each would
  // cost a round trip for a few microseconds of work): such a level is
  // pushed; the network may turn the heuristic's pull into a push, but not a
  // push into a pull.  last_heuristic keeps the threshold rule's own answer,
  // so that a block started against it keeps pushing.
  int decide(const LevelFeatures& lf, int device_choice = -1, const float* pred = nullptr,
             bool keep_push = false) {
    int a;
    const int raw = (o.policy == GR_POLICY_FIXED || o.policy == GR_POLICY_RANDOM) ? -1 : heuristic(lf);
    const int h = keep_push && raw >= GR_PULL_TWC ? push_action() : raw;
    if (o.policy == GR_POLICY_FIXED) a = o.fixed_action;
    else if (o.policy == GR_POLICY_RANDOM) a = (int)(next(rng) % 4);
    else if (o.policy == GR_POLICY_LEARNED && learned && device_choice >= 0 && pred) {
      a = (device_choice != h && pred[device_choice] + o.learned_margin < pred[h]) ? device_choice : h;
      if (keep_push && h < GR_PULL_TWC && a >= GR_PULL_TWC) a = h;
      last_heuristic = raw;
    } else {
      a = h;
      last_heuristic = raw;
    }
    if (!pull_ok && a >= GR_PULL_TWC) a -= 2;  // same balancing, push direction
    mode_pull = a >= GR_PULL_TWC;
    return a;
  }
};

}  // namespace gr
