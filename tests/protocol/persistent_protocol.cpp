// Host-thread model of the persistent batch kernel's scheduling protocol
// (test infrastructure).  Workgroups are threads, grouped by XCD; each group
// has a queue head, each domain a counter of finished tiles; a work item q of
// a group is tile q mod nt of pair q / nt; an item of pair s > 0 waits until
// its domain has finished all its tiles of pair s - 1 (counter >= ntiles * s),
// with a bounded wait that aborts the batch through an error flag; a finished
// tile is counted, then the next item is taken.  The model adds random delays
// at every step (adversarial interleavings) and checks, each time an item
// starts, that its domain is exactly between pairs s - 1 and s: every tile of
// the domain has finished pair s - 1 and none has finished pair s + 1... or
// started it.  It exits with status 0 if every run ends with every tile at the
// last pair (or, for the abort runs, ends with the error flag set), and with
// status 1 on a violated invariant or a run that did not end in time.
//
//   persistent_protocol <seed> <runs>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

struct Tile {
  int domain;
  int index;  // within the domain
};

struct Batch {
  int ngroups, npairs;
  std::vector<int> ntiles;                 // per domain
  std::vector<std::vector<Tile>> group;    // tiles of each group, domain by domain
  std::vector<std::atomic<unsigned>> head;
  std::vector<std::atomic<unsigned>> done;
  std::vector<std::vector<std::atomic<int>>> state;  // pairs finished, per tile
  std::vector<std::atomic<int>> started;            // per domain: items in flight
  std::atomic<int> err{0};
  std::atomic<int> violations{0};
  long long spin_limit;
  Batch(int ngroups_, int npairs_, const std::vector<int>& nt, const std::vector<int>& owner, long long spin)
      : ngroups(ngroups_), npairs(npairs_), ntiles(nt), group(ngroups_), head(ngroups_), done(nt.size()),
        state(nt.size()), started(nt.size()), spin_limit(spin) {
    for (auto& h : head) h = 0;
    for (size_t d = 0; d < nt.size(); ++d) {
      done[d] = 0;
      started[d] = 0;
      state[d] = std::vector<std::atomic<int>>(nt[d]);
      for (auto& x : state[d]) x = 0;
      for (int t = 0; t < nt[d]; ++t) group[owner[d]].push_back({(int)d, t});
    }
  }
};

static void jitter(std::mt19937& rng, int max_us) {
  const int r = (int)(rng() % 8);
  if (r == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % (max_us + 1)));
  else if (r < 3) std::this_thread::yield();
}

// One workgroup: the same steps as the kernel's tile loop.  `stall` > 0 makes
// this worker sleep that long inside its first item (a forced slow producer).
static void worker(Batch& b, int g, unsigned seed, int max_us, int stall_ms) {
  std::mt19937 rng(seed);
  const unsigned nt = (unsigned)b.group[g].size();
  const unsigned total = nt * (unsigned)b.npairs;
  if (nt == 0) return;
  unsigned q = b.head[g].fetch_add(1);
  for (unsigned it = 0; it < total && q < total; ++it) {
    jitter(rng, max_us);
    const unsigned s = q / nt;
    const Tile tl = b.group[g][q % nt];
    const int d = tl.domain;
    if (s > 0) {
      const unsigned target = (unsigned)b.ntiles[d] * s;
      bool ok = true;
      for (long long k = 0;; ++k) {
        if (b.done[d].load() >= target) break;
        if (b.err.load() != 0) { ok = false; break; }
        if (k >= b.spin_limit) { b.err.fetch_or(1); ok = false; break; }
        jitter(rng, max_us);
      }
      if (!ok) break;
    }
    // the domain must be exactly between pairs s - 1 and s
    b.started[d].fetch_add(1);
    for (int t = 0; t < b.ntiles[d]; ++t) {
      const int st = b.state[d][t].load();
      if (st < (int)s || st > (int)s + 1) b.violations.fetch_add(1);
    }
    if (b.state[d][tl.index].load() != (int)s) b.violations.fetch_add(1);
    jitter(rng, max_us);
    if (stall_ms > 0 && it == 0) std::this_thread::sleep_for(std::chrono::milliseconds(stall_ms));
    b.state[d][tl.index].store((int)s + 1);
    b.started[d].fetch_sub(1);
    jitter(rng, max_us);
    b.done[d].fetch_add(1);
    q = b.head[g].fetch_add(1);
  }
}

// Returns 0 when the run ended as expected.
static int run(unsigned seed, bool abort_run) {
  std::mt19937 rng(seed);
  const int ngroups = 1 + (int)(rng() % 4);
  const int ndom = ngroups + (int)(rng() % 12);
  const int npairs = 1 + (int)(rng() % 40);
  std::vector<int> nt(ndom), owner(ndom);
  for (int d = 0; d < ndom; ++d) {
    nt[d] = 1 + (int)(rng() % 9);
    owner[d] = d % ngroups;  // every group holds at least one domain
  }
  const long long spin = abort_run ? 2000 : (1ll << 40);
  Batch b(ngroups, npairs, nt, owner, spin);
  std::vector<std::thread> th;
  int workers = 0;
  for (int g = 0; g < ngroups; ++g) {
    const int w = 1 + (int)(rng() % 6);
    for (int k = 0; k < w; ++k, ++workers)
      th.emplace_back(worker, std::ref(b), g, seed * 977u + (unsigned)workers, 20,
                      (abort_run && workers == 0) ? 150 : 0);
  }
  const auto t0 = std::chrono::steady_clock::now();
  for (auto& t : th) t.join();
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (secs > 60.0) { std::printf("seed %u: took %.1f s\n", seed, secs); return 1; }
  if (b.violations.load() != 0) { std::printf("seed %u: %d barrier violations\n", seed, b.violations.load()); return 1; }
  if (abort_run) {
    // a group whose only worker stalled may finish late, but never wrongly; the
    // others either finished or left through the error flag
    if (npairs > 1 && b.err.load() == 0) {
      bool all = true;
      for (int d = 0; d < ndom; ++d) all = all && b.done[d].load() == (unsigned)(nt[d] * npairs);
      if (!all) { std::printf("seed %u: incomplete without an error\n", seed); return 1; }
    }
    return 0;
  }
  if (b.err.load() != 0) { std::printf("seed %u: error flag without a stall\n", seed); return 1; }
  for (int d = 0; d < ndom; ++d) {
    if (b.done[d].load() != (unsigned)(nt[d] * npairs)) { std::printf("seed %u: domain %d incomplete\n", seed, d); return 1; }
    for (int t = 0; t < nt[d]; ++t)
      if (b.state[d][t].load() != npairs) { std::printf("seed %u: tile %d/%d at %d\n", seed, d, t, b.state[d][t].load()); return 1; }
  }
  return 0;
}

int main(int argc, char** argv) {
  const unsigned seed0 = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
  const int runs = argc > 2 ? std::atoi(argv[2]) : 40;
  int bad = 0, aborted = 0;
  for (int r = 0; r < runs; ++r) {
    bad += run(seed0 + (unsigned)r, false);
    bad += run(seed0 + 100000u + (unsigned)r, true);
    ++aborted;
  }
  std::printf("%d runs of the protocol, %d with a stalled producer: %d failures\n", runs, aborted, bad);
  return bad == 0 ? 0 : 1;
}
