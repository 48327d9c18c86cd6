// CPU harness for the serving scheduler (serve_core.hpp) with a stand-in
// backend: a "sweep" halves every pixel of every admitted request, so a
// request with tolerance tol finishes after a known number of sweeps.  Used by
// tests/test_serve_scheduler.py to exercise admission, back-pressure, errors
// and concurrency without a GPU.  Prints "ok <case>" per passing case.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>

#include "serve_core.hpp"

using namespace smre_serve;

struct Fake : Backend {
  int nslots;
  size_t bytes;
  int step_sleep_us = 0;
  int fail_at = -1;
  std::atomic<int> steps{0}, max_active{0};
  struct S {
    bool on = false;
    std::vector<float> x;
    int sweeps = 0, max_sweeps = 0;
    double tol = 0, last = 0;
    bool conv = false;
  };
  std::vector<S> s;
  Fake(int n, size_t b) : nslots(n), bytes(b), s(n) {}
  int slots() const override { return nslots; }
  size_t budget() const override { return bytes; }
  size_t footprint(const Request& r) const override { return (size_t)r.H * r.W * 4 * 2; }
  int admit(Request& r, int k) override {
    s[k] = S();
    s[k].on = true;
    s[k].x = r.in;
    s[k].max_sweeps = r.max_sweeps;
    s[k].tol = r.tol;
    int a = 0;
    for (auto& q : s) a += q.on;
    if (a > max_active) max_active = a;
    return SMRE_OK;
  }
  int step(std::vector<int>& fin) override {
    if (step_sleep_us) std::this_thread::sleep_for(std::chrono::microseconds(step_sleep_us));
    if (fail_at >= 0 && steps >= fail_at) return SMRE_EDEVICE;
    ++steps;
    for (int k = 0; k < nslots; ++k) {
      S& q = s[k];
      if (!q.on) continue;
      double d = 0;
      for (float& v : q.x) {
        const float nv = v * 0.5f;
        d = std::max(d, (double)std::fabs(nv - v));
        v = nv;
      }
      q.last = d;
      ++q.sweeps;
      if (q.tol > 0 && d < q.tol) q.conv = true;
      if (q.conv || q.sweeps >= q.max_sweeps) fin.push_back(k);
    }
    return SMRE_OK;
  }
  int retire(Request& r, int k) override {
    S& q = s[k];
    r.out = q.x;
    r.rep.sweeps = q.sweeps;
    r.rep.converged = q.conv;
    r.rep.last_delta = q.last;
    q.on = false;
    return SMRE_OK;
  }
};

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);       \
      ++fails;                                                     \
    }                                                              \
  } while (0)

static smre_params params(double tol, int maxs, const int32_t* sides, const double* r2, int n) {
  smre_params p{};
  p.n_sides = n;
  p.sides = sides;
  p.radius2 = r2;
  p.tol = tol;
  p.max_sweeps = maxs;
  return p;
}

static int wait(Server& s, uint64_t t, std::vector<float>& out, smre_report* rep) {
  for (int i = 0; i < 200000; ++i) {
    const int rc = s.poll(t, out.data(), out.size(), rep, nullptr);
    if (rc != SMRE_PENDING) return rc;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  return -999;
}

// sweeps the fake needs: first k with 2^-k * max|x| < tol
static int expected_sweeps(float mx, double tol) {
  int k = 0;
  float v = mx;
  for (;;) {
    ++k;
    const float nv = v * 0.5f;
    if (std::fabs(nv - v) < tol) return k;
    v = nv;
  }
}

int main(int argc, char** argv) {
  const std::string only = argc > 1 ? argv[1] : "";
  const int32_t sides[1] = {1};
  const double r2[1] = {1.0};

  if (only.empty() || only == "basic") {
    auto* f = new Fake(4, 1 << 20);
    Server s(std::unique_ptr<Backend>(f), 64);
    std::vector<uint64_t> t(10);
    for (int i = 0; i < 10; ++i) {
      std::vector<float> x((i + 2) * 3, float(i + 1));
      const smre_params p = params(1e-3, 1000, sides, r2, 1);
      CHECK(s.submit(x.data(), i + 2, 3, &p, &t[i]) == SMRE_OK);
    }
    for (int i = 0; i < 10; ++i) {
      std::vector<float> out((i + 2) * 3);
      smre_report rep{};
      CHECK(wait(s, t[i], out, &rep) == SMRE_OK);
      const int k = expected_sweeps(float(i + 1), 1e-3);
      CHECK(rep.sweeps == k && rep.converged == 1);
      CHECK(out[0] == std::ldexp(float(i + 1), -k));
    }
    CHECK(f->max_active <= 4);
    CHECK(s.stats().completed == 10);
    // the scheduler's own count of co-resident requests agrees with the
    // backend's, and requests joined a running mix
    CHECK(s.stats().peak_active == f->max_active && f->max_active >= 2);
    CHECK(s.stats().joined_running >= 1);
    std::printf("ok basic\n");
  }
  if (only.empty() || only == "admission") {
    auto* f = new Fake(8, 100 * 4 * 2);  // budget: one 10x10 request at a time
    Server s(std::unique_ptr<Backend>(f), 64);
    std::vector<uint64_t> t(5);
    for (int i = 0; i < 5; ++i) {
      std::vector<float> x(100, 1.0f);
      const smre_params p = params(1e-2, 1000, sides, r2, 1);
      CHECK(s.submit(x.data(), 10, 10, &p, &t[i]) == SMRE_OK);
    }
    for (auto tk : t) {
      std::vector<float> out(100);
      CHECK(wait(s, tk, out, nullptr) == SMRE_OK);
    }
    CHECK(f->max_active == 1);
    CHECK(s.stats().peak_active == 1 && s.stats().joined_running == 0);
    std::vector<float> big(400, 1.0f);
    uint64_t tk;
    const smre_params p = params(1e-2, 10, sides, r2, 1);
    CHECK(s.submit(big.data(), 20, 20, &p, &tk) == SMRE_ETOOBIG);
    std::printf("ok admission\n");
  }
  if (only.empty() || only == "busy") {
    auto* f = new Fake(1, 1 << 20);
    f->step_sleep_us = 2000;
    Server s(std::unique_ptr<Backend>(f), 1);
    std::vector<float> x(4, 1.0f);
    const smre_params p = params(1e-6, 50, sides, r2, 1);
    uint64_t a, b, c;
    CHECK(s.submit(x.data(), 2, 2, &p, &a) == SMRE_OK);
    for (int i = 0; i < 1000 && s.stats().active < 1; ++i)
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    CHECK(s.submit(x.data(), 2, 2, &p, &b) == SMRE_OK);
    CHECK(s.submit(x.data(), 2, 2, &p, &c) == SMRE_EBUSY);
    std::vector<float> out(4);
    CHECK(wait(s, a, out, nullptr) == SMRE_OK);
    CHECK(wait(s, b, out, nullptr) == SMRE_OK);
    std::printf("ok busy\n");
  }
  if (only.empty() || only == "errors") {
    auto* f = new Fake(2, 1 << 20);
    Server s(std::unique_ptr<Backend>(f), 8);
    std::vector<float> x(4, 1.0f), out(4);
    uint64_t t;
    smre_params p = params(1e-30, 3, sides, r2, 1);
    CHECK(s.submit(x.data(), 2, 2, &p, &t) == SMRE_OK);
    smre_report rep{};
    CHECK(wait(s, t, out, &rep) == SMRE_NOT_CONVERGED);
    CHECK(rep.sweeps == 3 && rep.converged == 0);
    x[1] = NAN;
    CHECK(s.submit(x.data(), 2, 2, &p, &t) == SMRE_ENONFINITE);
    x[1] = 1.0f;
    CHECK(s.poll(12345, out.data(), out.size(), nullptr, nullptr) == SMRE_EUNKNOWN_TICKET);
    const int32_t bad_side[1] = {3};
    p = params(1e-3, 3, bad_side, r2, 1);
    CHECK(s.submit(x.data(), 2, 2, &p, &t) == SMRE_EINVAL);
    std::printf("ok errors\n");
  }
  if (only.empty() || only == "device_failure") {
    auto* f = new Fake(2, 1 << 20);
    f->fail_at = 5;
    f->step_sleep_us = 500;
    Server s(std::unique_ptr<Backend>(f), 8);
    std::vector<float> x(4, 1.0f), out(4);
    const smre_params p = params(1e-30, 1000, sides, r2, 1);
    uint64_t t[4];
    for (auto& tk : t) CHECK(s.submit(x.data(), 2, 2, &p, &tk) == SMRE_OK);
    for (auto tk : t) CHECK(wait(s, tk, out, nullptr) == SMRE_EDEVICE);
    uint64_t tk;
    CHECK(s.submit(x.data(), 2, 2, &p, &tk) == SMRE_EDEVICE);
    std::printf("ok device_failure\n");
  }
  if (only.empty() || only == "threads") {
    auto* f = new Fake(6, 1 << 22);
    Server s(std::unique_ptr<Backend>(f), 4096);
    std::atomic<int> good{0};
    std::vector<std::thread> th;
    for (int w = 0; w < 8; ++w)
      th.emplace_back([&, w] {
        for (int i = 0; i < 40; ++i) {
          const int H = 1 + (w + i) % 7, W = 1 + (w * 3 + i) % 5;
          std::vector<float> x(H * W, float(1 + (w + i) % 9)), out(H * W);
          const smre_params p = params(1e-2, 500, sides, r2, 1);
          uint64_t t;
          if (s.submit(x.data(), H, W, &p, &t) != SMRE_OK) continue;
          smre_report rep{};
          if (wait(s, t, out, &rep) == SMRE_OK &&
              rep.sweeps == expected_sweeps(float(1 + (w + i) % 9), 1e-2))
            ++good;
        }
      });
    for (auto& t : th) t.join();
    CHECK(good == 320);
    CHECK(f->max_active <= 6);
    std::printf("ok threads\n");
  }
  if (only.empty() || only == "shutdown") {
    auto* f = new Fake(1, 1 << 20);
    f->step_sleep_us = 1000;
    {
      Server s(std::unique_ptr<Backend>(f), 16);
      std::vector<float> x(4, 1.0f);
      const smre_params p = params(1e-30, 100000, sides, r2, 1);
      uint64_t t;
      for (int i = 0; i < 5; ++i) CHECK(s.submit(x.data(), 2, 2, &p, &t) == SMRE_OK);
    }  // destroy with work in flight: must not hang
    std::printf("ok shutdown\n");
  }
  return fails ? 1 : 0;
}
