// Admission policy of the serving loop (project addition), kept free of any
// GPU dependency so the host logic can be checked on a machine without one.
//
// The queue is served in FIFO order with head-of-line blocking: the request
// at the head is admitted when a slot is free and its workspace fits in the
// largest free block of the arena; otherwise nothing behind it is admitted
// either (no reordering, so no starvation of large requests).  A head that
// could never fit, even in an empty arena, is rejected (out of memory).
// Requests of the batched method at the head, consecutive and with options
// that allow one batch, are admitted together: the longest prefix of them
// (up to max_batch) whose joint workspace fits.
#pragma once

#include <cstddef>
#include <functional>

namespace tsylv {
namespace policy {

struct QueueView {
  std::size_t size = 0;
  std::function<bool(std::size_t)> batched;                 // request i takes the batched path
  std::function<bool(std::size_t, std::size_t)> batchable;  // i can share a batch with j
  std::function<std::size_t(std::size_t)> need_single;      // workspace of request i alone
  std::function<std::size_t(std::size_t)> need_batch;       // workspace of the first k together
};

enum class Kind { Wait, Single, Batch, Reject };

struct Decision {
  Kind kind;
  std::size_t count;  // requests taken from the head of the queue
};

inline Decision next_admission(const QueueView& q, std::size_t free_slots,
                               std::size_t largest_free, std::size_t capacity,
                               std::size_t max_batch) {
  if (q.size == 0 || free_slots == 0) return {Kind::Wait, 0};
  if (q.batched(0)) {
    std::size_t k = 1;
    while (k < q.size && k < max_batch && q.batched(k) && q.batchable(k, 0)) ++k;
    std::size_t take = k;
    while (take > 0 && q.need_batch(take) > largest_free) --take;
    if (take > 0) return {Kind::Batch, take};
    if (q.need_batch(1) > capacity) return {Kind::Reject, 1};
    return {Kind::Wait, 0};
  }
  const std::size_t need = q.need_single(0);
  if (need > capacity) return {Kind::Reject, 1};
  if (need > largest_free) return {Kind::Wait, 0};
  return {Kind::Single, 1};
}

}  // namespace policy
}  // namespace tsylv
