// Exercises the serving loop (server.hip) against the stub runtime from
// several threads, for host-only builds under AddressSanitizer +
// UndefinedBehaviorSanitizer and under ThreadSanitizer.  Prints one line per
// scenario and "ok" at the end; any failed check prints the reason and
// exits with status 1.  Test infrastructure only.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <complex>
#include <random>
#include <thread>
#include <vector>

#include "nufft2.h"
#include "stub_control.h"

namespace {

#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            exit(1);                                                     \
        }                                                                \
    } while (0)

struct Req {
    int prec, F;
    int64_t K, n;
    std::vector<std::complex<float>> c32;
    std::vector<std::complex<double>> c64;
    std::vector<double> phi, theta;
    std::vector<std::complex<float>> o32;
    std::vector<std::complex<double>> o64;

    Req(int prec_, int F_, int64_t K_, int64_t n_, std::mt19937_64 &rng) : prec(prec_), F(F_), K(K_), n(n_)
    {
        std::uniform_real_distribution<double> u(-1.0, 1.0);
        const size_t nc = (size_t)F * K * K;
        if (prec == NUFFT2_FP32) {
            c32.resize(nc);
            for (auto &x : c32) x = {(float)u(rng), (float)u(rng)};
            o32.assign((size_t)F * n, {0.f, 0.f});
        } else {
            c64.resize(nc);
            for (auto &x : c64) x = {u(rng), u(rng)};
            o64.assign((size_t)F * n, {0.0, 0.0});
        }
        phi.resize(n);
        theta.resize(n);
        for (int64_t j = 0; j < n; ++j) {
            phi[j] = 3.0 + 3.0 * u(rng);
            theta[j] = 1.5 + 1.5 * u(rng);
        }
    }

    nufft2_request request() const
    {
        nufft2_request r{};
        r.prec = prec;
        r.n_fields = F;
        r.n_modes_theta = r.n_modes_phi = K;
        r.eps = prec == NUFFT2_FP32 ? 1e-6 : 1e-12;
        r.n_pts = n;
        r.coeffs_host = prec == NUFFT2_FP32 ? (const void *)c32.data() : (const void *)c64.data();
        r.phi_host = phi.data();
        r.theta_host = theta.data();
        r.out_host = prec == NUFFT2_FP32 ? (void *)o32.data() : (void *)o64.data();
        r.t_arrival = NAN;  // set by the caller
        return r;
    }

    // the stub exec's value: c[f][0][0] + (f + 1) phi + i theta
    bool output_ok() const
    {
        for (int f = 0; f < F; ++f)
            for (int64_t j = 0; j < n; ++j) {
                const size_t o = (size_t)f * n + j;
                if (prec == NUFFT2_FP32) {
                    const auto c = c32[(size_t)f * K * K];
                    const std::complex<float> want{c.real() + (float)((f + 1) * phi[j]), c.imag() + (float)theta[j]};
                    if (o32[o] != want) return false;
                } else {
                    const auto c = c64[(size_t)f * K * K];
                    const std::complex<double> want{c.real() + (f + 1) * phi[j], c.imag() + theta[j]};
                    if (o64[o] != want) return false;
                }
            }
        return true;
    }
};

uint64_t submit(nufft2_server s, const Req &q)
{
    nufft2_request r = q.request();
    r.t_arrival = nufft2_server_clock(s);
    uint64_t t = 0;
    CHECK(nufft2_server_submit(s, &r, &t) == NUFFT2_OK);
    return t;
}

nufft2_status wait(nufft2_server s, uint64_t t)
{
    nufft2_status rs = NUFFT2_OK;
    double lat = 0;
    CHECK(nufft2_server_wait(s, t, &rs, &lat) == NUFFT2_OK);
    return rs;
}

// Four submitting threads with mixed requests and a thread reading the stats
// meanwhile, under a budget that forces queueing and plan eviction.
void mixed(uint64_t budget)
{
    stub_reset_peak();
    const size_t base = stub_device_bytes();
    nufft2_server_opts o{budget, 4, 0};
    nufft2_server s = nullptr;
    CHECK(nufft2_server_create(&o, &s) == NUFFT2_OK);
    std::atomic<bool> done{false};
    std::thread reader([&] {
        nufft2_server_stats_t st;
        while (!done.load()) {
            CHECK(nufft2_server_stats(s, &st) == NUFFT2_OK);
            CHECK(st.completed + st.failed <= st.submitted);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    const int threads = 4, per = 60;
    std::vector<std::thread> ts;
    for (int k = 0; k < threads; ++k)
        ts.emplace_back([&, k] {
            std::mt19937_64 rng(100 + k);
            std::vector<Req> reqs;
            reqs.reserve(per);
            const int64_t Ks[] = {15, 31, 63, 127};
            for (int i = 0; i < per; ++i)
                reqs.emplace_back(i % 5 == 0 ? NUFFT2_FP64 : NUFFT2_FP32, 1 + (int)(rng() % 3), Ks[rng() % 4],
                                  100 + (int64_t)(rng() % 4000), rng);
            std::vector<uint64_t> tickets;
            for (auto &q : reqs) tickets.push_back(submit(s, q));
            for (size_t i = 0; i < reqs.size(); ++i) {
                CHECK(wait(s, tickets[i]) == NUFFT2_OK);
                CHECK(reqs[i].output_ok());
            }
        });
    for (auto &t : ts) t.join();
    done.store(true);
    reader.join();
    nufft2_server_stats_t st;
    CHECK(nufft2_server_stats(s, &st) == NUFFT2_OK);
    CHECK(st.completed == threads * per && st.failed == 0);
    CHECK(st.hbm_high_water <= budget);
    CHECK(stub_device_peak() - base <= budget);
    printf("mixed: %lld requests, %lld plans created, %lld evicted, high water %.1f MiB, stub peak %.1f MiB\n",
           (long long)st.completed, (long long)st.plans_created, (long long)st.plans_evicted,
           st.hbm_high_water / 1048576.0, (stub_device_peak() - base) / 1048576.0);
    CHECK(nufft2_server_destroy(s) == NUFFT2_OK);
    CHECK(stub_device_bytes() == base);
}

// One plan key reused with growing point counts under a budget that the
// plan's growth plus a second slot buffer would exceed: every request must
// complete (none may wait forever) within the budget.
void growing_points()
{
    stub_reset_peak();
    const size_t base = stub_device_bytes();
    const uint64_t budget = 48ull << 20;
    nufft2_server_opts o{budget, 2, 0};
    nufft2_server s = nullptr;
    CHECK(nufft2_server_create(&o, &s) == NUFFT2_OK);
    std::mt19937_64 rng(7);
    for (int64_t n : {1000, 50000, 200000, 400000, 800000}) {
        Req q(NUFFT2_FP32, 1, 63, n, rng);
        const auto t0 = std::chrono::steady_clock::now();
        CHECK(wait(s, submit(s, q)) == NUFFT2_OK);
        CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(20));
        CHECK(q.output_ok());
    }
    nufft2_server_stats_t st;
    CHECK(nufft2_server_stats(s, &st) == NUFFT2_OK);
    CHECK(st.completed == 5 && st.hbm_high_water <= budget);
    CHECK(stub_device_peak() - base <= budget);
    printf("growing points: high water %.1f MiB of %.0f\n", st.hbm_high_water / 1048576.0, budget / 1048576.0);
    CHECK(nufft2_server_destroy(s) == NUFFT2_OK);
    CHECK(stub_device_bytes() == base);
}

// Allocation failures: a request whose plan cannot be allocated fails with
// ERR_ALLOC, the next one succeeds; a request above the budget is refused at
// submit.
void failures()
{
    const size_t base = stub_device_bytes();
    nufft2_server_opts o{256ull << 20, 2, 0};
    nufft2_server s = nullptr;
    CHECK(nufft2_server_create(&o, &s) == NUFFT2_OK);
    std::mt19937_64 rng(9);
    Req big(NUFFT2_FP64, 3, 255, 2000, rng), small(NUFFT2_FP32, 1, 31, 500, rng);
    stub_fail_allocations_of_at_least(8 << 20);  // the big plan's grids
    CHECK(wait(s, submit(s, big)) == NUFFT2_ERR_ALLOC);
    CHECK(wait(s, submit(s, small)) == NUFFT2_OK && small.output_ok());
    stub_fail_allocations_of_at_least(-1);
    CHECK(wait(s, submit(s, big)) == NUFFT2_OK && big.output_ok());
    Req huge(NUFFT2_FP64, 3, 2047, 1000, rng);
    nufft2_request r = huge.request();
    r.t_arrival = 0;
    uint64_t t = 0;
    CHECK(nufft2_server_submit(s, &r, &t) == NUFFT2_ERR_ARG);  // above the budget
    nufft2_server_stats_t st;
    CHECK(nufft2_server_stats(s, &st) == NUFFT2_OK);
    CHECK(st.failed == 1 && st.completed == 2);
    printf("failures: ERR_ALLOC reported, server kept working, oversized request refused\n");
    CHECK(nufft2_server_destroy(s) == NUFFT2_OK);
    CHECK(stub_device_bytes() == base);
}

// Destroy with requests still queued and in flight: it drains them first.
void destroy_while_busy()
{
    const size_t base = stub_device_bytes();
    nufft2_server_opts o{64ull << 20, 3, 0};
    nufft2_server s = nullptr;
    CHECK(nufft2_server_create(&o, &s) == NUFFT2_OK);
    std::mt19937_64 rng(11);
    std::vector<Req> reqs;
    reqs.reserve(40);
    for (int i = 0; i < 40; ++i) reqs.emplace_back(NUFFT2_FP32, 2, 31 + 32 * (i % 3), 2000, rng);
    for (auto &q : reqs) (void)submit(s, q);
    CHECK(nufft2_server_destroy(s) == NUFFT2_OK);
    for (auto &q : reqs) CHECK(q.output_ok());
    CHECK(stub_device_bytes() == base);
    printf("destroy while busy: 40 requests drained\n");
}

}  // namespace

int main()
{
    mixed(16ull << 20);
    growing_points();
    failures();
    destroy_while_busy();
    printf("ok\n");
    return 0;
}
