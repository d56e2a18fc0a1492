// Test driver for the serving loop's admission policy (sched_policy.hpp):
// reads scenarios from stdin, prints the decision for each.
//
// A scenario line:  slots largest_free capacity max_batch nreq  then nreq
// request tokens  S<bytes>  (single request with that workspace) or
// B<opts>:<bytes>  (batched request with an options class and its own
// workspace; a batch of k needs the sum of its members plus 16 bytes).
// Output per scenario: "<kind> <count>" with kind wait/single/batch/reject.
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "sched_policy.hpp"

using namespace tsylv::policy;

struct R {
  bool batched;
  int opts;
  std::size_t bytes;
};

int main() {
  std::size_t slots, largest, capacity, max_batch, n;
  while (std::cin >> slots >> largest >> capacity >> max_batch >> n) {
    std::vector<R> q(n);
    for (auto& r : q) {
      std::string tok;
      std::cin >> tok;
      if (tok[0] == 'S') {
        r = {false, -1, std::stoull(tok.substr(1))};
      } else {
        const auto c = tok.find(':');
        r = {true, std::stoi(tok.substr(1, c - 1)), std::stoull(tok.substr(c + 1))};
      }
    }
    QueueView v;
    v.size = q.size();
    v.batched = [&](std::size_t i) { return q[i].batched; };
    v.batchable = [&](std::size_t i, std::size_t j) { return q[i].opts == q[j].opts; };
    v.need_single = [&](std::size_t i) { return q[i].bytes; };
    v.need_batch = [&](std::size_t k) {
      std::size_t b = 16;
      for (std::size_t i = 0; i < k; ++i) b += q[i].bytes;
      return b;
    };
    const Decision d = next_admission(v, slots, largest, capacity, max_batch);
    const char* kind = d.kind == Kind::Wait     ? "wait"
                       : d.kind == Kind::Single ? "single"
                       : d.kind == Kind::Batch  ? "batch"
                                                : "reject";
    std::printf("%s %zu\n", kind, d.count);
  }
  return 0;
}
