// Host-only checks of the library's table cache and argument validation,
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitized.py.  Exits non-zero on the first failure.
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <string>
#include <tuple>
#include <vector>

#include "cache.hpp"
#include "tune_cache.hpp"
#include "validate.hpp"

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

// A device table stand-in: heap memory that must be released exactly once.
struct Tab {
  int* mem = nullptr;
  int id = -1;
};

using Key = std::tuple<int, double>;

static void test_lru_pins() {
  lp::TableCache<Key, Tab> c;
  std::vector<int> released;
  auto rel = [&](Tab& t) {
    released.push_back(t.id);
    delete[] t.mem;
    t.mem = nullptr;
  };
  int rounds = 0;
  auto before = [&](size_t n) {
    CHECK(n > 0);
    ++rounds;
  };
  uint64_t epoch = 0;
  for (int i = 0; i < 5; ++i) {
    ++epoch;
    Tab t;
    t.mem = new int[16];
    t.id = i;
    CHECK(c.insert(Key{i, 0.5 * i}, t, 100, epoch) != nullptr);
  }
  CHECK(c.size() == 5 && c.bytes() == 500);
  // duplicate insert is refused and leaves the slot alone
  CHECK(c.insert(Key{0, 0.0}, Tab{}, 7, epoch) == nullptr && c.bytes() == 500);
  // touch entry 0 (now most recent), pin entry 1
  ++epoch;
  CHECK(c.find(Key{0, 0.0}, epoch) != nullptr);
  CHECK(c.pin(Key{1, 0.5}));
  CHECK(!c.pin(Key{9, 9.0}));
  CHECK(c.pinned() == 1);
  // evict to 250 bytes within a later call: LRU unpinned are 2, 3, 4 (epochs 3, 4, 5), then 0
  ++epoch;
  size_t n = c.evict_to(250, epoch, before, rel);
  CHECK(n == 3);
  CHECK(rounds == 1);
  CHECK(released.size() == 3 && released[0] == 2 && released[1] == 3 && released[2] == 4);
  CHECK(c.bytes() == 200 && c.size() == 2);
  // an entry used in the current call is never a victim
  CHECK(c.find(Key{0, 0.0}, epoch) != nullptr);
  n = c.evict_to(0, epoch, before, rel);
  CHECK(n == 0 && rounds == 1);
  // below the target nothing happens and before() is not called
  CHECK(c.evict_to(1000, epoch + 1, before, rel) == 0 && rounds == 1);
  // clear keeps pinned tables
  CHECK(c.clear_unpinned(rel) == 1);
  CHECK(c.size() == 1 && c.peek(Key{1, 0.5}) != nullptr && c.bytes() == 100);
  // pins nest; unpin of an unpinned or absent key is refused
  CHECK(c.pin(Key{1, 0.5}));
  CHECK(c.unpin(Key{1, 0.5}) && c.unpin(Key{1, 0.5}));
  CHECK(!c.unpin(Key{1, 0.5}));
  CHECK(!c.unpin(Key{7, 1.0}));
  CHECK(c.add_bytes(Key{1, 0.5}, 50) && c.bytes() == 150);
  CHECK(!c.add_bytes(Key{8, 0.0}, 50));
  CHECK(c.clear_unpinned(rel) == 1 && c.size() == 0 && c.bytes() == 0);
  CHECK(released.size() == 5);
  CHECK(c.evictions() == 3);
}

// A distance-optimisation loop: every step asks for tables of new distances;
// the budget holds the cached bytes bounded whatever the number of steps.
static void test_budget_loop() {
  lp::TableCache<Key, Tab> c;
  const size_t limit = 10 * 64;
  size_t live = 0, peak = 0;
  uint64_t epoch = 0;
  auto rel = [&](Tab& t) {
    delete[] t.mem;
    --live;
  };
  for (int step = 0; step < 200; ++step) {
    for (int link = 0; link < 4; ++link) {
      ++epoch;
      Tab t;
      t.mem = new int[8];
      ++live;
      c.insert(Key{link, 1e-3 * step + link}, t, 64, epoch);
      if (c.bytes() > limit) c.evict_to(limit / 4 * 3, epoch, [](size_t) {}, rel);
      peak = c.bytes() > peak ? c.bytes() : peak;
    }
  }
  CHECK(peak <= limit);
  CHECK(live == c.size());
  c.clear_unpinned(rel);
  CHECK(live == 0);
}

static bool is_len(int v) {
  // powers of two up to 8192 and 3 * 2^k from 96 to 6144
  for (int p = 1; p <= 8192; p *= 2)
    if (v == p) return true;
  for (int p = 96; p <= 6144; p *= 2)
    if (v == p) return true;
  return false;
}

static void test_validation() {
  for (int n = -3; n <= 8200; ++n) {
    int want = -1;
    if (n >= 1)
      for (int v = n; v <= 8192; ++v)
        if (is_len(v)) {
          want = v;
          break;
        }
    if (lp::fft_len(n) != want) {
      std::fprintf(stderr, "fft_len(%d) = %d, want %d\n", n, lp::fft_len(n), want);
      ++failures;
      break;
    }
  }
  prop_grid g{16, 8, 1e-6, 1e-6, 0.0, 0.0};
  CHECK(lp::check_grid(&g) == PROP_OK);
  CHECK(lp::check_grid(nullptr) == PROP_ENULL);
  prop_grid b = g;
  b.nx = 0;
  CHECK(lp::check_grid(&b) == PROP_ESHAPE);
  b = g;
  b.dy = -1.0;
  CHECK(lp::check_grid(&b) == PROP_EPARAM);
  b = g;
  b.cx = std::numeric_limits<double>::infinity();
  CHECK(lp::check_grid(&b) == PROP_EPARAM);
  b = g;
  b.dx = std::numeric_limits<double>::quiet_NaN();
  CHECK(lp::check_grid(&b) == PROP_EPARAM);
  CHECK(lp::check_common(PROP_C64, 1, 500e-9) == PROP_OK);
  CHECK(lp::check_common((prop_dtype)7, 1, 500e-9) == PROP_EPARAM);
  CHECK(lp::check_common(PROP_C128, -1, 500e-9) == PROP_ESHAPE);
  CHECK(lp::check_common(PROP_C128, 1, 0.0) == PROP_EPARAM);
  prop_lens L{0.9, 2e-3};
  CHECK(lp::check_lens(&L) == PROP_OK && lp::check_lens(nullptr) == PROP_OK);
  L.na = 1.0;
  CHECK(lp::check_lens(&L) == PROP_EPARAM);
  prop_grid big{4097, 4, 1e-6, 1e-6, 0, 0};
  CHECK(lp::check_rs_shape(&g) == PROP_OK && lp::check_rs_shape(&big) == PROP_ESHAPE);
  prop_grid w{8192, 8, 1e-6, 1e-6, 0, 0};
  CHECK(lp::check_czt_shapes(&g, &g) == PROP_OK && lp::check_czt_shapes(&w, &g) == PROP_ESHAPE);
  // aliasing of byte ranges
  std::vector<char> buf(256);
  const char* p = buf.data();
  CHECK(lp::check_alias({{p, 64}}, {{p + 64, 64}}) == PROP_OK);
  CHECK(lp::check_alias({{p, 65}}, {{p + 64, 64}}) == PROP_EALIAS);
  CHECK(lp::check_alias({{p, 64}}, {{p + 64, 64}, {p + 100, 8}}) == PROP_EALIAS);
  CHECK(lp::check_alias({{p, 64}}, {{p + 64, 64}, {p + 128, 8}}) == PROP_OK);
  CHECK(lp::overlap(p, 1, p, 1) && !lp::overlap(p, 0, p, 8));
  // sampling warning: 1 mm grid of 128 at 650 nm is under-sampled at 5 mm,
  // fine at 30 mm; a pitch below lambda/2 never warns
  prop_grid s{128, 128, 1e-3 / 128, 1e-3 / 128, 0, 0};
  CHECK(lp::sampling(&s, 650e-9, 5e-3) == PROP_WUNDERSAMPLED);
  CHECK(lp::sampling(&s, 650e-9, 30e-3) == PROP_OK);
  prop_grid fine{128, 128, 0.3e-6, 0.3e-6, 0, 0};
  CHECK(lp::sampling(&fine, 650e-9, 1e-6) == PROP_OK);
}

// Tuning-cache records: round trip, and every corruption is rejected
// (never a crash, never a half-filled record).
static void test_tune_records() {
  lp::TuneRecord r;
  r.arch = "gfx950";
  r.elem = 4;
  r.kind = 2;
  r.n = 3072;
  r.lines = 2048;
  r.n_in = 2048;
  r.n_out = 1024;
  r.batch = 8;
  r.variant = 3;
  const std::string line = lp::format_tune_record(r);
  lp::TuneRecord q;
  CHECK(lp::parse_tune_record(line, &q));
  CHECK(q.arch == r.arch && q.elem == 4 && q.kind == 2 && q.n == 3072 && q.lines == 2048 && q.n_in == 2048 &&
        q.n_out == 1024 && q.batch == 8 && q.variant == 3);
  const char* bad[] = {
      "", "libprop-tune", "libprop-tune 2 gfx950 4 2 3072 2048 2048 1024 8 3",
      "libprop-tune 1 gfx950 4 2 3072 2048 2048 1024 8 3 extra", "libprop-tune 1 gfx950 4 2 3072 2048 2048 1024 8",
      "libprop-tune 1 gfx950 5 2 3072 2048 2048 1024 8 3", "libprop-tune 1 gfx950 4 9 3072 2048 2048 1024 8 3",
      "libprop-tune 1 gfx950 4 2 9000 2048 2048 1024 8 3", "libprop-tune 1 gfx950 4 2 3072 0 2048 1024 8 3",
      "libprop-tune 1 gfx950 4 2 3072 2048 4000 1024 8 3", "libprop-tune 1 gfx950 4 2 3072 2048 2048 1024 -1 3",
      "libprop-tune 1 gfx950 4 2 3072 2048 2048 1024 8 6", "libprop-tune 1 gfx950 4 2 3072 2048 2048 1024 8 -1",
      "libprop-tune 1 gfx9$0 4 2 3072 2048 2048 1024 8 3", "libprop-tune 1 gfx950 4 2 3072 2048 2048 1024 8 x",
      "libprop-tune 1 gfx950 4 2 99999999999999999999 2048 2048 1024 8 3", "other-tag 1 gfx950 4 2 3072 2048 2048 1024 8 3",
  };
  for (const char* b : bad) {
    lp::TuneRecord z;
    z.variant = -7;
    if (lp::parse_tune_record(b, &z)) {
      std::fprintf(stderr, "accepted a corrupt tuning record: '%s'\n", b);
      ++failures;
    }
    CHECK(z.variant == -7);
  }
  // random bytes and truncations of a good line never crash the parser
  unsigned x = 12345u;
  for (int t = 0; t < 20000; ++t) {
    std::string g;
    const int len = (int)(x % 96);
    for (int k = 0; k < len; ++k) {
      x = x * 1103515245u + 12345u;
      g.push_back((char)(x >> 16));
    }
    x = x * 1103515245u + 12345u;
    lp::TuneRecord z;
    (void)lp::parse_tune_record(g, &z);
    (void)lp::parse_tune_record(line.substr(0, x % (line.size() + 1)), &z);
  }
}

int main() {
  test_tune_records();
  test_lru_pins();
  test_budget_loop();
  test_validation();
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("host cache/validation checks passed\n");
  return 0;
}
