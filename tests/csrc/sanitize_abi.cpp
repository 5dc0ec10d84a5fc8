// sanitize_abi.cpp -- driver of the library built with host-side ASan/UBSan (test infrastructure):
// calls every C-ABI entry point with invalid arguments, which the host-side validation must turn
// into an error before any GPU work (no GPU is needed), plus the workspace-size queries, the
// per-call option checks and the error strings.  Any sanitizer report makes the process fail.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "hawkes.h"
#include "hawkes_mlp.h"

static int fails = 0;
#define EXPECT(cond)                                                  \
    do {                                                              \
        if (!(cond)) {                                                \
            std::printf("FAIL line %d: %s\n", __LINE__, #cond);       \
            ++fails;                                                  \
        }                                                             \
    } while (0)

int main()
{
    hawkes_theta th = {0.5, 10.0, 7.0, 0.3, 2.0, 0.2};
    const auto fake = reinterpret_cast<double *>(uintptr_t(0x200000));  // never dereferenced
    hawkes_events ev = {1000, fake, fake, fake, fake, 0.0};
    for (int prec = 0; prec < 3; ++prec)
        for (int64_t n : {int64_t(1), int64_t(2), int64_t(513), int64_t(100000), int64_t(1) << 30}) {
            const size_t a = hawkes_workspace_min_bytes(n, prec), b = hawkes_workspace_bytes(n, prec);
            EXPECT(a > 0 && a <= b && a % 256 == 0 && b % 256 == 0);
        }
    EXPECT(hawkes_workspace_bytes(0, 1) == 0 && hawkes_workspace_bytes((int64_t(1) << 30) + 1, 1) == 0);
    EXPECT(hawkes_workspace_min_bytes(5, 9) == 0);
    const size_t ws = hawkes_workspace_bytes(1000, 1);
    double out;
    EXPECT(hawkes_loglik(nullptr, &th, 1, 0, 10, fake, ws, &out, nullptr, nullptr) == HAWKES_EINVAL);
    hawkes_events bad = ev;
    bad.n = 0;
    EXPECT(hawkes_loglik(&bad, &th, 1, 0, 0, fake, ws, &out, nullptr, nullptr) == HAWKES_EINVAL);
    bad = ev;
    bad.area = -1.0;
    EXPECT(hawkes_loglik(&bad, &th, 1, 0, 10, fake, ws, &out, nullptr, nullptr) == HAWKES_EINVAL);
    EXPECT(std::strstr(hawkes_last_error(), "area") != nullptr);
    for (int k = 0; k < 6; ++k) {
        hawkes_theta b = th;
        (&b.mu)[k] = -1.0;
        EXPECT(hawkes_loglik_grad(&ev, &b, 1, 0, 10, fake, ws, &out, fake, nullptr, nullptr) == HAWKES_EINVAL);
    }
    EXPECT(hawkes_loglik(&ev, &th, 7, 0, 10, fake, ws, &out, nullptr, nullptr) == HAWKES_EINVAL);
    EXPECT(hawkes_loglik(&ev, &th, 1, 5, 4, fake, ws, &out, nullptr, nullptr) == HAWKES_ERANGE);
    EXPECT(hawkes_loglik(&ev, &th, 1, 0, 1001, fake, ws, &out, nullptr, nullptr) == HAWKES_ERANGE);
    EXPECT(hawkes_loglik(&ev, &th, 1, 0, 10, fake, 256, &out, nullptr, nullptr) == HAWKES_EWORKSPACE);
    EXPECT(hawkes_loglik(&ev, &th, 1, 0, 10, reinterpret_cast<char *>(fake) + 8, ws, &out, nullptr, nullptr) ==
           HAWKES_EWORKSPACE);
    EXPECT(hawkes_loglik_grad(&ev, &th, 1, 0, 10, fake, ws, &out, nullptr, nullptr, nullptr) == HAWKES_EINVAL);
    EXPECT(hawkes_event_terms(&ev, &th, 1, 0, 10, fake, 256, fake, fake, nullptr, nullptr) == HAWKES_EWORKSPACE);
    hawkes_options o;
    std::memset(&o, 0, sizeof(o));
    o.row_workgroups = -3;
    EXPECT(hawkes_loglik(&ev, &th, 1, 0, 10, fake, ws, &out, &o, nullptr) == HAWKES_EINVAL);
    o.row_workgroups = 0;
    o.symmetric_groups = 5000;
    EXPECT(hawkes_loglik(&ev, &th, 1, 0, 10, fake, ws, &out, &o, nullptr) == HAWKES_EINVAL);
    o.symmetric_groups = 0;
    o.reserved = 1;
    EXPECT(hawkes_loglik(&ev, &th, 1, 0, 10, fake, ws, &out, &o, nullptr) == HAWKES_EINVAL);
    o.reserved = 0;
    o.timing_start = fake;
    EXPECT(hawkes_loglik(&ev, &th, 1, 0, 10, fake, ws, &out, &o, nullptr) == HAWKES_EINVAL);
    hawkes_theta two[2] = {th, th};
    two[1].omega = 0.0;
    EXPECT(hawkes_loglik_batch(&ev, two, 2, 1, 0, 10, fake, ws, &out, nullptr, nullptr) == HAWKES_EINVAL);
    EXPECT(hawkes_loglik_batch(&ev, two, 0, 1, 0, 10, fake, ws, &out, nullptr, nullptr) == HAWKES_EINVAL);
    EXPECT(hawkes_resample_locations(10, nullptr, fake, 3, 1, 2, fake, fake, nullptr) == HAWKES_EINVAL);
    EXPECT(hawkes_resample_locations(10, reinterpret_cast<int32_t *>(fake), fake, 0, 1, 2, fake, fake, nullptr) ==
           HAWKES_EINVAL);
    EXPECT(hawkes_workspace_status(nullptr, nullptr, nullptr) == HAWKES_EINVAL);
    EXPECT(hawkes_mlp_state_bytes() > 0 && hawkes_mlp_workspace_bytes(256) > 0);
    EXPECT(hawkes_mlp_workspace_bytes(0) == 0);
    EXPECT(hawkes_mlp_forward(nullptr, nullptr, 1, nullptr, nullptr, nullptr) == HAWKES_EINVAL);
    EXPECT(hawkes_mlp_leapfrog(fake, nullptr, 20, nullptr) == HAWKES_EINVAL);
    EXPECT(hawkes_mlp_adam_step(fake, reinterpret_cast<float *>(fake), 0, 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr) ==
           HAWKES_EINVAL);
    for (int code = 0; code >= -7; --code)
        EXPECT(hawkes_strerror(code) != nullptr && std::strlen(hawkes_strerror(code)) > 0);
    std::printf(fails ? "FAILED %d\n" : "OK\n", fails);
    return fails ? 1 : 0;
}
