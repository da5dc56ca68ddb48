// Host-only checks of the request server's admission policy (gwc::Admission)
// on a fake executor: worker threads that "run" a request by sleeping, with no
// device.  Built and run by tests/test_host_admission.py under the address,
// undefined-behaviour and thread sanitizers.  Exit status 0 when every check
// holds; otherwise the failed check is printed.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "gwc_admission.h"

namespace {

struct Item {
  int id = 0;
  size_t footprint = 0;
  int sleep_us = 0;
  std::atomic<bool> hold{false};  // the fake executor waits while set
};

#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      std::exit(1);                                                        \
    }                                                                      \
  } while (0)

void sleep_us(int us) { std::this_thread::sleep_for(std::chrono::microseconds(us)); }

// FIFO order with one worker: requests start exactly in submission order.
void fifo_single_worker() {
  gwc::Admission<Item> adm(100);
  std::vector<Item> items(30);
  for (int i = 0; i < 30; ++i) {
    items[i].id = i;
    items[i].footprint = 1 + (size_t)((i * 37) % 100);
    CHECK(adm.submit(&items[i], items[i].footprint));
  }
  std::vector<int> order;
  std::thread w([&] {
    for (;;) {
      size_t fp = 0;
      Item *it = adm.acquire(fp);
      if (!it) return;
      CHECK(fp == it->footprint);
      order.push_back(it->id);
      adm.release(fp);
    }
  });
  adm.stop();
  w.join();
  CHECK((int)order.size() == 30);
  for (int i = 0; i < 30; ++i) CHECK(order[i] == i);
  CHECK(adm.stats().completed == 30 && adm.stats().in_use == 0);
}

// Several workers: the footprints in flight never exceed the budget, every
// request completes, and small requests do run concurrently.
void budget_invariant_many_workers() {
  const size_t budget = 100;
  gwc::Admission<Item> adm(budget);
  const int n = 400, workers = 6;
  std::vector<Item> items(n);
  std::atomic<size_t> in_flight{0};
  std::atomic<size_t> max_in_flight{0};
  std::atomic<int> done{0};
  std::vector<std::thread> ws;
  for (int k = 0; k < workers; ++k)
    ws.emplace_back([&] {
      for (;;) {
        size_t fp = 0;
        Item *it = adm.acquire(fp);
        if (!it) return;
        const size_t now = in_flight.fetch_add(fp) + fp;
        size_t m = max_in_flight.load();
        while (now > m && !max_in_flight.compare_exchange_weak(m, now)) {
        }
        sleep_us(it->sleep_us);
        in_flight.fetch_sub(fp);
        done.fetch_add(1);
        adm.release(fp);
      }
    });
  unsigned x = 12345u;
  for (int i = 0; i < n; ++i) {
    x = x * 1664525u + 1013904223u;
    items[i].id = i;
    items[i].footprint = 1 + (x >> 8) % budget;   // 1 .. budget
    items[i].sleep_us = 50 + (int)((x >> 4) % 400);
    CHECK(adm.submit(&items[i], items[i].footprint));
    if (i % 7 == 0) sleep_us(30);
  }
  adm.stop();
  for (auto &t : ws) t.join();
  const auto st = adm.stats();
  CHECK(done.load() == n && st.completed == n);
  CHECK(max_in_flight.load() <= budget);
  CHECK(st.peak_in_use <= budget && st.in_use == 0 && st.queued == 0 && st.active == 0);
  CHECK(st.peak_active > 1 && st.peak_active <= workers);
}

// A request larger than the whole budget is refused and never queued.
void oversize_refused() {
  gwc::Admission<Item> adm(100);
  Item big;
  CHECK(!adm.submit(&big, 101));
  CHECK(adm.stats().queued == 0);
  Item fits;
  CHECK(adm.submit(&fits, 100));
  CHECK(adm.stats().queued == 1);
}

// Head of line: with 60 in use, a queued 50 does not fit and a 10 behind it
// must wait (no overtaking); releasing the 60 lets both run.
void head_of_line() {
  gwc::Admission<Item> adm(100);
  Item a, b, c;
  a.id = 0; a.footprint = 60; a.hold = true;
  b.id = 1; b.footprint = 50;
  c.id = 2; c.footprint = 10;
  std::atomic<int> started{0};
  std::vector<int> order(3, -1);  // by admission ticket (taken under the policy's lock)
  std::vector<std::thread> ws;
  for (int k = 0; k < 3; ++k)
    ws.emplace_back([&] {
      for (;;) {
        size_t fp = 0;
        long long ticket = -1;
        Item *it = adm.acquire(fp, &ticket);
        if (!it) return;
        CHECK(ticket >= 0 && ticket < 3);
        order[ticket] = it->id;
        started.fetch_add(1);
        while (it->hold.load()) sleep_us(100);
        adm.release(fp);
      }
    });
  CHECK(adm.submit(&a, a.footprint));
  while (started.load() < 1) sleep_us(100);
  CHECK(adm.submit(&b, b.footprint));
  CHECK(adm.submit(&c, c.footprint));
  sleep_us(20000);
  // the 10 would fit next to the 60 but stays behind the 50
  CHECK(started.load() == 1);
  auto st = adm.stats();
  CHECK(st.active == 1 && st.queued == 2 && st.in_use == 60);
  a.hold = false;
  adm.stop();
  for (auto &t : ws) t.join();
  CHECK(started.load() == 3);
  CHECK(order[0] == 0 && order[1] == 1 && order[2] == 2);
  st = adm.stats();
  CHECK(st.peak_in_use == 60 && st.completed == 3 && st.in_use == 0);
}

// stop() with nothing queued releases idle workers at once.
void stop_releases_idle_workers() {
  gwc::Admission<Item> adm(10);
  std::vector<std::thread> ws;
  std::atomic<int> exited{0};
  for (int k = 0; k < 4; ++k)
    ws.emplace_back([&] {
      size_t fp = 0;
      CHECK(adm.acquire(fp) == nullptr);
      exited.fetch_add(1);
    });
  sleep_us(5000);
  CHECK(exited.load() == 0);
  adm.stop();
  for (auto &t : ws) t.join();
  CHECK(exited.load() == 4);
}

}  // namespace

// Kept bytes: a finished request that keeps part of its footprint (device
// memory it built for a resident system) shrinks the budget for the rest; a
// queued request that can then never fit is handed out as refused instead of
// blocking the ones behind it, and a new one is refused at submission.
void kept_bytes() {
  gwc::Admission<Item> adm(100);
  Item a, b, c, d;
  CHECK(adm.submit(&a, 60));
  size_t fp = 0;
  bool refused = true;
  Item *it = adm.acquire(fp, nullptr, &refused);
  CHECK(it == &a && !refused && fp == 60);
  CHECK(adm.submit(&b, 60));  // fits beside nothing kept so far
  CHECK(adm.submit(&c, 40));
  adm.release(60, 50);  // a keeps 50 of its 60
  CHECK(adm.stats().kept == 50 && adm.stats().in_use == 50 && adm.stats().active == 0);
  it = adm.acquire(fp, nullptr, &refused);  // b: 60 > 100 - 50, refused
  CHECK(it == &b && refused && fp == 60);
  it = adm.acquire(fp, nullptr, &refused);  // c: 50 + 40 <= 100
  CHECK(it == &c && !refused && fp == 40);
  CHECK(!adm.submit(&d, 70));  // 70 > 100 - 50: refused at submission
  adm.release(40);
  const auto st = adm.stats();
  CHECK(st.in_use == 50 && st.kept == 50 && st.refused == 1 && st.completed == 3);
  adm.stop();
  CHECK(adm.acquire(fp) == nullptr);
}

int main() {
  fifo_single_worker();
  budget_invariant_many_workers();
  oversize_refused();
  head_of_line();
  stop_releases_idle_workers();
  kept_bytes();
  std::printf("admission: all checks passed\n");
  return 0;
}
