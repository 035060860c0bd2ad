// Byte-budgeted least-recently-used cache of device tables with pins.
//
// Host-only C++ (no HIP): the library keeps its kernel spectra and zoom
// chirp vectors here, keyed by geometry.  Values are opaque handles whose
// device memory the caller releases through a callback.
//
//  * Every lookup or insert stamps the slot with the caller's epoch (one
//    epoch per library call), so a call never evicts a table it already
//    fetched.
//  * Pinned slots (a plan holds a pin on every table its kernels or captured
//    graphs address) are never evicted and survive clear_unpinned().
//  * evict_to() drops unpinned slots of earlier epochs, oldest first, until
//    the total falls to a target size.  It reports the victims before
//    releasing any, so the caller can wait for in-flight work once per
//    eviction round instead of once per table.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <map>
#include <utility>
#include <vector>

namespace lp {

template <class Key, class Val>
class TableCache {
 public:
  struct Slot {
    Val v{};
    size_t bytes = 0;
    uint64_t last = 0;  // epoch of the last lookup or insert
    int pins = 0;
  };

  // Slot of `k` stamped with `epoch`, or nullptr.
  Slot* find(const Key& k, uint64_t epoch) {
    auto it = map_.find(k);
    if (it == map_.end()) return nullptr;
    it->second.last = std::max(it->second.last, epoch);
    return &it->second;
  }
  const Slot* peek(const Key& k) const {
    auto it = map_.find(k);
    return it == map_.end() ? nullptr : &it->second;
  }
  // New slot (the key must be absent), stamped with `epoch`.
  Slot* insert(const Key& k, const Val& v, size_t bytes, uint64_t epoch) {
    auto r = map_.emplace(k, Slot{});
    Slot& s = r.first->second;
    if (!r.second) return nullptr;
    s.v = v;
    s.bytes = bytes;
    s.last = epoch;
    bytes_ += bytes;
    return &s;
  }
  // Tables added to an existing slot later (e.g. another kernel kind).
  bool add_bytes(const Key& k, size_t bytes) {
    auto it = map_.find(k);
    if (it == map_.end()) return false;
    it->second.bytes += bytes;
    bytes_ += bytes;
    return true;
  }
  bool pin(const Key& k) {
    auto it = map_.find(k);
    if (it == map_.end()) return false;
    ++it->second.pins;
    return true;
  }
  // false if the key is absent or was not pinned.
  bool unpin(const Key& k) {
    auto it = map_.find(k);
    if (it == map_.end() || it->second.pins <= 0) return false;
    --it->second.pins;
    return true;
  }

  // Evict unpinned slots last used before `epoch`, least recently used
  // first, until bytes() <= target.  before(n) is called once with the
  // number of victims (n > 0) before the first release(value).  Returns the
  // number of slots released.
  template <class Before, class Release>
  size_t evict_to(size_t target, uint64_t epoch, Before before, Release release) {
    if (bytes_ <= target) return 0;
    std::vector<std::pair<uint64_t, const Key*>> cand;
    for (auto& kv : map_)
      if (kv.second.pins == 0 && kv.second.last < epoch) cand.emplace_back(kv.second.last, &kv.first);
    std::sort(cand.begin(), cand.end(),
              [](const std::pair<uint64_t, const Key*>& a, const std::pair<uint64_t, const Key*>& b) {
                return a.first < b.first;
              });
    size_t drop = 0, left = bytes_;
    while (drop < cand.size() && left > target) left -= map_.find(*cand[drop++].second)->second.bytes;
    if (drop == 0) return 0;
    before(drop);
    for (size_t i = 0; i < drop; ++i) {
      auto it = map_.find(*cand[i].second);
      release(it->second.v);
      bytes_ -= it->second.bytes;
      map_.erase(it);
    }
    evictions_ += drop;
    return drop;
  }

  // Release every unpinned slot.  Returns the number released.
  template <class Release>
  size_t clear_unpinned(Release release) {
    size_t n = 0;
    for (auto it = map_.begin(); it != map_.end();) {
      if (it->second.pins > 0) {
        ++it;
        continue;
      }
      release(it->second.v);
      bytes_ -= it->second.bytes;
      it = map_.erase(it);
      ++n;
    }
    return n;
  }

  size_t bytes() const { return bytes_; }
  size_t size() const { return map_.size(); }
  size_t pinned() const {
    size_t n = 0;
    for (auto& kv : map_) n += kv.second.pins > 0 ? 1 : 0;
    return n;
  }
  uint64_t evictions() const { return evictions_; }
  template <class F>
  void for_each(F f) {
    for (auto& kv : map_) f(kv.first, kv.second);
  }

 private:
  std::map<Key, Slot> map_;
  size_t bytes_ = 0;
  uint64_t evictions_ = 0;
};

}  // namespace lp
