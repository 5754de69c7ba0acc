// Host model of the one-launch LU sweep protocol (paper_2410_05865_amd/csrc/
// lu_flow.hpp): threads stand in for wavefronts and run flow_run with GCC
// atomics.  Built with -fsanitize=thread: every task reads the data of the
// nodes it depends on with plain loads, so a missing happens-before edge in
// the protocol is a reported race.  Checks:
//   * forward sweeps (a task waits on its node's children; tasks add into the
//     accumulators of their parent and grandparent with relaxed atomics and
//     read their own node's accumulator with a plain load) and backward
//     sweeps (a task waits on its node's parent and reads the plain outputs of
//     the parent's and grandparent's tasks) give the sequential results;
//   * trees: random forests, a chain, a star, one node; 1, 2, 7 and 33 threads,
//     threads starting late; 1, 2, 4 or 5 tickets taken at a time; repeated
//     sweeps with the counters reset between them (the replays of a captured
//     graph);
//   * a node that never completes (its count one short): every wait on it
//     gives up within the bound, the error word is set and the run ends.
// Exit status 0 and a line "all ok" on success.  Built with PLANT_RELAXED_SIGNAL
// (completion counts without release) or PLANT_NO_WAITS (no dependencies) it
// must fail: a reported race or wrong results.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../paper_2410_05865_amd/csrc/lu_flow.hpp"

namespace {

// Fence plus relaxed RMW on the device is, by the memory model, a release RMW;
// the sanitizer does not model standalone fences, so the host states the
// equivalent release RMW and acquire load directly.
struct HostSync {
  static int next_ticket(int* t, int n) { return __atomic_fetch_add(t, n, __ATOMIC_RELAXED); }
  static int load_acquire(const int* p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
  static int load_relaxed(const int* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
  static void set_err(int* p) { __atomic_store_n(p, 1, __ATOMIC_RELAXED); }
  static long long now() {
    return std::chrono::duration_cast<std::chrono::microseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
  }
  static void pause() { std::this_thread::yield(); }
  static void acquire_fence() {}
  static void release_fence() {}
#ifdef PLANT_RELAXED_SIGNAL
  static void signal(int* p) { __atomic_fetch_add(p, 1, __ATOMIC_RELAXED); }  // planted mistake
#else
  static void signal(int* p) { __atomic_fetch_add(p, 1, __ATOMIC_RELEASE); }
#endif
};

struct Tree {
  std::vector<int> parent;  // -1 for roots; parent > child
  std::vector<int> ntask;   // tasks per node
  std::vector<int> height;
};

Tree finish(std::vector<int> parent, std::mt19937& rng, int max_tasks) {
  Tree T;
  const int n = (int)parent.size();
  T.parent = parent;
  T.ntask.resize(n);
  T.height.assign(n, 0);
  std::uniform_int_distribution<int> nt(1, max_tasks);
  for (int v = 0; v < n; ++v) T.ntask[v] = nt(rng);
  for (int v = 0; v < n; ++v)
    if (parent[v] >= 0) T.height[parent[v]] = std::max(T.height[parent[v]], T.height[v] + 1);
  return T;
}

Tree random_forest(int n, std::mt19937& rng) {
  std::vector<int> parent(n, -1);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int v = 0; v < n - 1; ++v)
    if (u(rng) < 0.97) parent[v] = v + 1 + (int)(u(rng) * std::min(n - v - 1, 12));
  return finish(parent, rng, 4);
}
Tree chain(int n, std::mt19937& rng) {
  std::vector<int> parent(n, -1);
  for (int v = 0; v < n - 1; ++v) parent[v] = v + 1;
  return finish(parent, rng, 3);
}
Tree star(int n, std::mt19937& rng) {
  std::vector<int> parent(n, n - 1);
  parent[n - 1] = -1;
  return finish(parent, rng, 2);
}

struct Sweep {
  std::vector<int> node, wait_ptr, wait, need, done, first;  // first: first ticket of each node
  int ticket = 0, err = 0, batch = 1;
  cc::FlowGraph graph() {
    cc::FlowGraph G;
    G.ntask = (int)node.size();
    G.node = node.data();
    G.wait_ptr = wait_ptr.data();
    G.wait = wait.data();
    G.need = need.data();
    G.done = done.data();
    G.ticket = &ticket;
    G.err = &err;
    G.batch = batch;
    return G;
  }
};

// forward: tickets by height ascending, waits on children; backward: tickets
// by height descending, waits on the parent
Sweep make_sweep(const Tree& T, bool fwd) {
  const int n = (int)T.parent.size();
  Sweep S;
  std::vector<int> order(n);
  for (int v = 0; v < n; ++v) order[v] = v;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return fwd ? T.height[a] < T.height[b] : T.height[a] > T.height[b];
  });
  S.first.assign(n, 0);
  for (int v : order) {
    S.first[v] = (int)S.node.size();
    for (int k = 0; k < T.ntask[v]; ++k) S.node.push_back(v);
  }
  S.wait_ptr.assign(n + 1, 0);
  std::vector<std::vector<int>> w(n);
  for (int v = 0; v < n; ++v) {
#ifndef PLANT_NO_WAITS
    if (fwd && T.parent[v] >= 0) w[T.parent[v]].push_back(v);
    if (!fwd && T.parent[v] >= 0) w[v].push_back(T.parent[v]);
#endif
  }
  for (int v = 0; v < n; ++v) {
    S.wait_ptr[v + 1] = S.wait_ptr[v] + (int)w[v].size();
    for (int u : w[v]) S.wait.push_back(u);
  }
  S.need = T.ntask;
  S.done.assign(n, 0);
  return S;
}

long long contrib(int t) { return 1000003LL * (t + 1) % 977 + 1; }

int failures = 0;
void check(bool ok, const char* what, int a, int b) {
  if (!ok) {
    std::printf("FAIL %s (%d, %d)\n", what, a, b);
    ++failures;
  }
}

// one forward and one backward sweep with `threads` threads, `batch` tickets
// taken at a time; `replays` times
void run_case(const char* name, const Tree& T, int threads, int replays, std::mt19937& rng, int batch = 1) {
  const int n = (int)T.parent.size();
  Sweep F = make_sweep(T, true), B = make_sweep(T, false);
  F.batch = B.batch = batch;
  const int nt = (int)F.node.size();
  std::vector<long long> acc(n), fout(nt), bout(nt);
  std::vector<long long> acc_ref(n, 0), fout_ref(nt), bout_ref(nt);
  // sequential references
  {
    std::vector<long long> a(n, 0);
    for (int t = 0; t < nt; ++t) {  // ticket order is a valid sequential order
      const int v = F.node[t];
      fout_ref[t] = a[v] + t;
      const int p = T.parent[v];
      if (p >= 0) {
        a[p] += contrib(t);
        if (T.parent[p] >= 0) a[T.parent[p]] += 2 * contrib(t);
      }
    }
    for (int t = 0; t < nt; ++t) {
      const int v = B.node[t];
      long long s = t;
      for (int anc = T.parent[v], lev = 0; anc >= 0 && lev < 2; anc = T.parent[anc], ++lev)
        for (int k = 0; k < T.ntask[anc]; ++k) s += bout_ref[B.first[anc] + k] % 1000;
      bout_ref[t] = s;
    }
  }
  std::uniform_int_distribution<int> delay(0, 200);
  for (int rep = 0; rep < replays; ++rep) {
    // the counters are reset before every sweep (a fill kernel on the device)
    std::fill(F.done.begin(), F.done.end(), 0);
    std::fill(B.done.begin(), B.done.end(), 0);
    F.ticket = B.ticket = 0;
    F.err = B.err = 0;
    std::fill(acc.begin(), acc.end(), 0);
    for (int sweep = 0; sweep < 2; ++sweep) {
      const bool fwd = sweep == 0;
      Sweep& S = fwd ? F : B;
      cc::FlowGraph G = S.graph();
      std::vector<std::thread> th;
      std::vector<int> d(threads);
      for (int i = 0; i < threads; ++i) d[i] = delay(rng);
      for (int i = 0; i < threads; ++i)
        th.emplace_back([&, i] {
          std::this_thread::sleep_for(std::chrono::microseconds(d[i]));
          cc::flow_run<HostSync>(G, 2000000 /* us */, [&](int t) {
            const int v = S.node[t];
            if (fwd) {
              fout[t] = acc[v] + t;  // plain read of the accumulator
              const int p = T.parent[v];
              if (p >= 0) {
                __atomic_fetch_add(&acc[p], contrib(t), __ATOMIC_RELAXED);
                if (T.parent[p] >= 0) __atomic_fetch_add(&acc[T.parent[p]], 2 * contrib(t), __ATOMIC_RELAXED);
              }
            } else {
              long long s = t;
              for (int anc = T.parent[v], lev = 0; anc >= 0 && lev < 2; anc = T.parent[anc], ++lev)
                for (int k = 0; k < T.ntask[anc]; ++k) s += bout[B.first[anc] + k] % 1000;  // plain reads
              bout[t] = s;
            }
          });
        });
      for (auto& x : th) x.join();
      check(S.err == 0, fwd ? "forward wait gave up" : "backward wait gave up", rep, threads);
      check(S.ticket >= S.graph().ntask, "tickets not exhausted", S.ticket, S.graph().ntask);
      for (int v = 0; v < n; ++v) check(S.done[v] == T.ntask[v], "node count", v, S.done[v]);
    }
    for (int t = 0; t < nt; ++t) {
      check(fout[t] == fout_ref[t], "forward result", t, rep);
      check(bout[t] == bout_ref[t], "backward result", t, rep);
    }
  }
  std::printf("ok %s: %d nodes, %d tasks, %d threads, %d tickets at a time, %d replays\n", name, n, nt, threads,
              batch, replays);
}

// a node one task short of its count: every wait on it must give up
void run_give_up(std::mt19937& rng) {
  Tree T = chain(6, rng);
  Sweep F = make_sweep(T, true);
  F.batch = 2;
  F.need[2] += 1;  // node 2 never completes
  cc::FlowGraph G = F.graph();
  const long long t0 = HostSync::now();
  std::vector<std::thread> th;
  for (int i = 0; i < 4; ++i)
    th.emplace_back([&] { cc::flow_run<HostSync>(G, 50000 /* us */, [&](int) {}); });
  for (auto& x : th) x.join();
  const long long us = HostSync::now() - t0;
  check(F.err == 1, "error word not set", F.err, 0);
  check(us < 5000000, "give-up took too long", (int)(us / 1000), 0);
  check(F.ticket >= G.ntask, "tickets not exhausted after give-up", F.ticket, G.ntask);
  std::printf("ok give-up: error word set, run ended after %lld ms\n", us / 1000);
}

}  // namespace

int main() {
  std::mt19937 rng(12345);
  Tree one = finish({-1}, rng, 3);
  run_case("single node", one, 3, 3, rng);
  for (int threads : {1, 2, 7, 33}) {
    Tree f = random_forest(300, rng);
    run_case("random forest", f, threads, 3, rng);
  }
  for (int batch : {2, 5}) {
    Tree f = random_forest(300, rng);
    run_case("random forest", f, 7, 3, rng, batch);
  }
  Tree c = chain(120, rng);
  run_case("chain", c, 7, 3, rng);
  run_case("chain", c, 7, 3, rng, 4);
  Tree s = star(400, rng);
  run_case("star", s, 7, 3, rng);
  run_give_up(rng);
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("all ok\n");
  return 0;
}
