// Dataflow order of one supernodal LU sweep in a single launch (the
// LU-correction and bottom solve of Sec. 5.3): a unit of execution (a
// wavefront on the device, a thread in the host model of the protocol) takes
// tasks by ticket, waits until the nodes its task depends on are complete,
// runs the task and signals its own node.
//
// Tickets follow the tree order of the sweep (forward: heights ascending,
// backward: descending), and a task depends only on nodes whose tasks all come
// earlier in that order (forward: the node's children; backward: its parent).
// A unit takes `batch` consecutive tickets at a time and runs them in order.
// A unit holding ticket t therefore waits only on tickets below t, which units
// already running hold, and those never wait on a ticket above their own (a
// unit's own earlier tickets are smaller): the smallest unfinished ticket
// always makes progress, so the sweep cannot deadlock as long as a unit that
// took a ticket keeps running (nothing preempts a running wavefront), however
// many units the grid has.
//
// Memory ordering: a task's writes (plain stores and atomic additions into
// later equations) are made visible by a release fence before its node's
// completion count is incremented; a waiter reads the counts with acquire
// loads and issues an acquire fence before its task reads anything.  Every
// wait is bounded in time: past `limit` clock ticks the waiter sets the error
// word and goes on, and every later wait sees the error word and stops
// waiting, so the launch always ends; the caller reports the error.  The
// counters (done, ticket) must be zero before each sweep.
//
// This header has no device or host dependencies: the sync policy S supplies
// the atomics, fences, clock and pause of the unit (see the device policy in
// kernels.hip; the host model under tests/ uses GCC atomics on threads).
#pragma once

#ifdef __HIPCC__
#define CC_FLOW_HD __host__ __device__
#else
#define CC_FLOW_HD
#endif

namespace cc {

struct FlowGraph {
  int ntask;              // tasks in ticket order
  const int* node;        // node of each task
  const int* wait_ptr;    // per node: range [wait_ptr[v], wait_ptr[v + 1]) of `wait`
  const int* wait;        // nodes that must be complete before a task of v runs
  const int* need;        // per node: number of its tasks (its count when complete)
  int* done;              // per node: tasks completed (zero before the sweep)
  int* ticket;            // next ticket (zero before the sweep)
  int* err;               // nonzero once a wait gave up
  int batch;              // tickets taken at a time (at least 1)
};

// Runs tasks until the tickets are exhausted; work(t) runs task t.
// S::next_ticket(int*, int n) relaxed fetch-add of n, the value uniform over the unit
// S::load_acquire(const int*) acquire load of a counter
// S::load_relaxed(const int*) relaxed load of the error word
// S::set_err(int*)            relaxed store of 1
// S::now()                    clock ticks (signed 64-bit)
// S::pause()                  short back-off
// S::acquire_fence(), S::release_fence()
// S::signal(int*)             relaxed fetch-add of 1 (one per unit)
template <class S, class Work>
CC_FLOW_HD inline void flow_run(const FlowGraph& G, long long limit, Work&& work) {
  for (;;) {
    const int tb = S::next_ticket(G.ticket, G.batch);
    if (tb >= G.ntask) return;
    const int te = tb + G.batch < G.ntask ? tb + G.batch : G.ntask;
    for (int t = tb; t < te; ++t) {
      const int v = G.node[t];
      for (int k = G.wait_ptr[v]; k < G.wait_ptr[v + 1]; ++k) {
        const int u = G.wait[k];
        const int need = G.need[u];
        const long long t0 = S::now();
        while (S::load_acquire(G.done + u) < need) {
          if (S::load_relaxed(G.err) != 0) break;
          if (S::now() - t0 > limit) {
            S::set_err(G.err);
            break;
          }
          S::pause();
        }
      }
      S::acquire_fence();
      work(t);
      S::release_fence();
      S::signal(G.done + v);
    }
  }
}

}  // namespace cc
