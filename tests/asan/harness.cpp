// Host AddressSanitizer harness for the runtime of libfpdlbm (test infrastructure).
//
// Built with AddressSanitizer on the host code only (the device code is the same as in
// the library), it drives the C ABI through the paths that touch host memory: creation and
// validation, stepping and read-back in three storage formats, split steps, checkpoint
// save / load (including a truncated file and a missing one), recording, launch settings,
// a batch with admission, launch / wait and the pending guard, release and the
// allocation-free entry point, plus the error returns for NULL and invalid arguments.  Exit status 0 when every
// call returned what it should; AddressSanitizer aborts on any invalid host access.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <string>
#include <vector>

#include "fpdlbm.h"

#define EXPECT(call, want)                                                               \
    do {                                                                                 \
        const int rc_ = (call);                                                          \
        if (rc_ != (want)) {                                                             \
            fprintf(stderr, "FAIL %s:%d: %s returned %d, expected %d (%s)\n", __FILE__,  \
                    __LINE__, #call, rc_, (int)(want), fpd_last_error());                \
            return 1;                                                                    \
        }                                                                                \
    } while (0)

#define REQUIRE(cond)                                                                    \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);              \
            return 1;                                                                    \
        }                                                                                \
    } while (0)

static fpd_params channel(int storage, int nx, int ny, int n_beads) {
    fpd_params p;
    fpd_params_default(&p);
    p.nx = nx;
    p.ny = ny;
    p.u_wall = 0.02;
    p.nu_f = 0.1;
    p.n_beads = n_beads;
    p.radius = 2.0;
    p.l0 = 4.0;
    p.k_s = 0.05 * 16.0;
    p.k_b = 1e-3;
    p.storage = storage;
    return p;
}

// a straight fiber along x through the channel's centre
static std::vector<double> fiber(const fpd_params& p) {
    std::vector<double> R(2 * (size_t)p.n_beads);
    for (int i = 0; i < p.n_beads; ++i) {
        R[2 * i] = 0.5 * p.nx + (i - 0.5 * (p.n_beads - 1)) * p.l0;
        R[2 * i + 1] = 0.5 * p.ny;
    }
    return R;
}

static std::string temp_path(const char* tag) {
    char buf[256];
    snprintf(buf, sizeof buf, "/tmp/fpd_asan_%s_%d.ckpt", tag, (int)getpid());
    return buf;
}

static int lifecycle(int storage) {
    fpd_params p = channel(storage, 96, 40, 5);
    const size_t nodes = (size_t)p.nx * p.ny;
    fpd_sim* s = nullptr;
    EXPECT(fpd_create(&p, nullptr, &s), FPD_OK);
    std::vector<double> R = fiber(p);
    EXPECT(fpd_step(s, 1), FPD_ESTATE);  // the fiber comes first
    EXPECT(fpd_init_fiber(s, R.data()), FPD_OK);
    EXPECT(fpd_step(s, 40), FPD_OK);
    EXPECT(fpd_sync(s), FPD_OK);
    std::vector<double> f(9 * nodes), rho(nodes), ux(nodes), uy(nodes), eta(nodes);
    std::vector<double> Rb(2 * p.n_beads), V(2 * p.n_beads), F(2 * p.n_beads);
    EXPECT(fpd_read_populations(s, f.data()), FPD_OK);
    EXPECT(fpd_read_fields(s, rho.data(), ux.data(), uy.data(), eta.data()), FPD_OK);
    EXPECT(fpd_read_fields(s, rho.data(), nullptr, nullptr, nullptr), FPD_OK);
    EXPECT(fpd_read_beads(s, Rb.data(), V.data(), F.data()), FPD_OK);
    uint32_t health = 0;
    double strain = 0.0;
    EXPECT(fpd_health(s, &health, &strain), FPD_OK);
    REQUIRE(health == 0);

    // checkpoint: the state after load + 10 steps equals the state after 10 steps
    const std::string ck = temp_path("ok"), cut = temp_path("cut");
    EXPECT(fpd_save(s, ck.c_str()), FPD_OK);
    EXPECT(fpd_step(s, 10), FPD_OK);
    std::vector<double> fa(9 * nodes), fb(9 * nodes);
    EXPECT(fpd_read_populations(s, fa.data()), FPD_OK);
    EXPECT(fpd_load(s, ck.c_str()), FPD_OK);
    int64_t steps = 0;
    EXPECT(fpd_step_count(s, &steps), FPD_OK);
    REQUIRE(steps == 40);
    EXPECT(fpd_step(s, 10), FPD_OK);
    EXPECT(fpd_read_populations(s, fb.data()), FPD_OK);
    REQUIRE(memcmp(fa.data(), fb.data(), fa.size() * sizeof(double)) == 0);
    // a truncated copy and a missing file are refused and leave the simulation as it was
    {
        FILE* in = fopen(ck.c_str(), "rb");
        REQUIRE(in);
        fseek(in, 0, SEEK_END);
        const long n = ftell(in);
        fseek(in, 0, SEEK_SET);
        std::vector<char> bytes((size_t)n);
        REQUIRE(fread(bytes.data(), 1, (size_t)n, in) == (size_t)n);
        fclose(in);
        for (long keep : {0L, 7L, n / 2, n - 1}) {
            FILE* out = fopen(cut.c_str(), "wb");
            REQUIRE(out);
            REQUIRE(fwrite(bytes.data(), 1, (size_t)keep, out) == (size_t)keep);
            fclose(out);
            EXPECT(fpd_load(s, cut.c_str()), FPD_EINVAL);
        }
    }
    EXPECT(fpd_load(s, "/nonexistent/fpd_asan.ckpt"), FPD_EINVAL);
    EXPECT(fpd_step_count(s, &steps), FPD_OK);
    REQUIRE(steps == 50);
    remove(ck.c_str());
    remove(cut.c_str());

    // recording of the fiber ends, launch settings, kernel timing
    EXPECT(fpd_record_start(s, 5, 64), FPD_OK);
    EXPECT(fpd_step(s, 20), FPD_OK);
    std::vector<double> rec(64 * 5);
    int64_t nrec = 0;
    EXPECT(fpd_record_read(s, rec.data(), 64, &nrec), FPD_OK);
    REQUIRE(nrec >= 4);
    EXPECT(fpd_record_stop(s), FPD_OK);
    fpd_launch bad{100, 1, 1, 2, 8};
    EXPECT(fpd_set_launch(s, &bad), FPD_EINVAL);
    fpd_launch good{128, 2, 1, 2, 8};
    EXPECT(fpd_set_launch(s, &good), FPD_OK);
    EXPECT(fpd_set_flags(s, FPD_FLAG_TIME_KERNELS), FPD_OK);
    EXPECT(fpd_reset_kernel_times(s), FPD_OK);
    EXPECT(fpd_step(s, 8), FPD_OK);
    double ms_l = 0.0, ms_b = 0.0;
    int64_t n_l = 0, n_b = 0;
    EXPECT(fpd_kernel_times(s, &ms_l, &n_l, &ms_b, &n_b), FPD_OK);
    REQUIRE(n_l == 8);
    EXPECT(fpd_set_flags(s, 0), FPD_OK);
    EXPECT(fpd_write_populations(s, f.data()), FPD_OK);
    EXPECT(fpd_step(s, 2), FPD_OK);
    fpd_destroy(s);
    return 0;
}

static int invalid_arguments() {
    fpd_params p = channel(FPD_F32, 0, 40, 0);
    fpd_sim* s = nullptr;
    EXPECT(fpd_create(&p, nullptr, &s), FPD_EINVAL);
    REQUIRE(s == nullptr);
    REQUIRE(strlen(fpd_last_error()) > 0);
    p = channel(FPD_F32, 64, 70000, 0);
    EXPECT(fpd_create(&p, nullptr, &s), FPD_EINVAL);
    p = channel(FPD_F32, 64, 32, FPD_MAX_BEADS + 1);
    EXPECT(fpd_create(&p, nullptr, &s), FPD_EINVAL);
    EXPECT(fpd_create(nullptr, nullptr, &s), FPD_EINVAL);
    EXPECT(fpd_step(nullptr, 1), FPD_EINVAL);
    EXPECT(fpd_read_beads(nullptr, nullptr, nullptr, nullptr), FPD_EINVAL);
    EXPECT(fpd_save(nullptr, "/tmp/x"), FPD_EINVAL);
    fpd_params q;
    EXPECT(fpd_params_from_physical(1.5, 0.5, 3.3, 10, 4.0, 100.0, 1.0, 0.01, 4, &q), FPD_OK);
    EXPECT(fpd_params_from_physical(1.5, 0.5, 3.3, 10, 4.0, 100.0, 1.0, 0.5, 4, &q),
           FPD_EINVAL);
    fpd_destroy(nullptr);
    fpd_batch_destroy(nullptr);
    return 0;
}

static int batch() {
    fpd_batch* b = nullptr;
    EXPECT(fpd_batch_create(1ull << 32, 0, FPD_F32, nullptr, &b), FPD_EINVAL);
    EXPECT(fpd_batch_create(1ull << 32, 3, FPD_F32, nullptr, &b), FPD_OK);
    fpd_launch cfg{0, 0, 0, 0, 8};
    EXPECT(fpd_batch_set_launch(b, &cfg), FPD_OK);
    const int sizes[4][3] = {{64, 32, 4}, {96, 40, 5}, {48, 36, 3}, {64, 32, 4}};
    int64_t ids[4] = {0, 0, 0, 0};
    for (int i = 0; i < 3; ++i) {
        fpd_params p = channel(FPD_F32, sizes[i][0], sizes[i][1], sizes[i][2]);
        std::vector<double> R = fiber(p);
        EXPECT(fpd_batch_add(b, &p, R.data(), 30 + 10 * i, &ids[i]), FPD_OK);
    }
    {
        fpd_params p = channel(FPD_F32, sizes[3][0], sizes[3][1], sizes[3][2]);
        std::vector<double> R = fiber(p);
        EXPECT(fpd_batch_add(b, &p, R.data(), 10, &ids[3]), FPD_ENOMEM);  // no free slot
        fpd_params w = channel(FPD_F64, 64, 32, 4);
        EXPECT(fpd_batch_add(b, &w, R.data(), 10, &ids[3]), FPD_EINVAL);  // other storage
    }
    int64_t adv = 0;
    EXPECT(fpd_batch_run(b, 16, &adv), FPD_OK);
    REQUIRE(adv == 16);
    EXPECT(fpd_batch_launch(b, 8, &adv), FPD_OK);
    REQUIRE(adv == 8);
    std::vector<double> R(2 * 5), V(2 * 5), F(2 * 5);
    EXPECT(fpd_batch_read_beads(b, ids[0], R.data(), V.data(), F.data()), FPD_EINVAL);
    EXPECT(fpd_batch_launch(b, 8, &adv), FPD_EINVAL);
    EXPECT(fpd_batch_wait(b), FPD_OK);
    EXPECT(fpd_batch_wait(b), FPD_OK);
    int done = 0;
    for (int round = 0; round < 10 && done < 3; ++round) {
        EXPECT(fpd_batch_run(b, 100, &adv), FPD_OK);
        int64_t got[8];
        int32_t st[8], n = 0;
        EXPECT(fpd_batch_poll(b, got, st, 8, &n), FPD_OK);
        for (int k = 0; k < n; ++k) {
            REQUIRE(st[k] == FPD_SIM_DONE);
            int idx = -1;
            for (int i = 0; i < 3; ++i)
                if (ids[i] == got[k]) idx = i;
            REQUIRE(idx >= 0);
            const size_t nodes = (size_t)sizes[idx][0] * sizes[idx][1];
            std::vector<double> f(9 * nodes), rho(nodes), ux(nodes), uy(nodes), eta(nodes);
            EXPECT(fpd_batch_read_populations(b, got[k], f.data()), FPD_OK);
            EXPECT(fpd_batch_read_fields(b, got[k], rho.data(), ux.data(), uy.data(),
                                         eta.data()),
                   FPD_OK);
            std::vector<double> Rk(2 * sizes[idx][2]), Vk(Rk.size()), Fk(Rk.size());
            EXPECT(fpd_batch_read_beads(b, got[k], Rk.data(), Vk.data(), Fk.data()), FPD_OK);
            int64_t steps = 0;
            int32_t status = 0;
            uint32_t health = 0;
            EXPECT(fpd_batch_sim_info(b, got[k], &steps, &status, &health), FPD_OK);
            REQUIRE(steps == 30 + 10 * idx && health == 0);
            EXPECT(fpd_batch_release(b, got[k]), FPD_OK);
            ++done;
        }
    }
    REQUIRE(done == 3);
    EXPECT(fpd_batch_release(b, 12345), FPD_EINVAL);
    int32_t active = -1, held = -1;
    size_t bytes = 1;
    EXPECT(fpd_batch_stats(b, &active, &held, &bytes), FPD_OK);
    REQUIRE(active == 0 && held == 0 && bytes == 0);
    fpd_batch_destroy(b);
    return 0;
}

static int run_static() {
    fpd_params p = channel(FPD_F32, 96, 40, 5);
    const size_t bytes = fpd_population_bytes(&p);
    REQUIRE(fpd_static_scratch_need(&p) <= FPD_STATIC_SCRATCH_BYTES);
    void *fa = nullptr, *fb = nullptr;
    REQUIRE(hipMalloc(&fa, bytes) == hipSuccess && hipMalloc(&fb, bytes) == hipSuccess);
    std::vector<double> R = fiber(p), Rout(R.size());
    double *dR = nullptr, *dRout = nullptr;
    uint32_t* dh = nullptr;
    REQUIRE(hipMalloc((void**)&dR, R.size() * sizeof(double)) == hipSuccess);
    REQUIRE(hipMalloc((void**)&dRout, R.size() * sizeof(double)) == hipSuccess);
    REQUIRE(hipMalloc((void**)&dh, sizeof(uint32_t)) == hipSuccess);
    REQUIRE(hipMemcpy(dR, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice) ==
            hipSuccess);
    EXPECT(fpd_run_static(&p, nullptr, fa, fb, bytes, 1, dR, dRout, dh, 20), FPD_OK);
    EXPECT(fpd_run_static(&p, nullptr, fa, fb, bytes / 2, 1, dR, dRout, dh, 20), FPD_EINVAL);
    REQUIRE(hipDeviceSynchronize() == hipSuccess);
    REQUIRE(hipMemcpy(Rout.data(), dRout, R.size() * sizeof(double), hipMemcpyDeviceToHost) ==
            hipSuccess);
    for (size_t i = 0; i < R.size(); ++i) REQUIRE(fabs(Rout[i] - R[i]) < 1.0);
    (void)hipFree(fa);
    (void)hipFree(fb);
    (void)hipFree(dR);
    (void)hipFree(dRout);
    (void)hipFree(dh);
    return 0;
}

// split steps (a lattice large enough that the fiber's partition is a small part of it):
// the side stream and events are created on first use and released by fpd_destroy, also
// with split steps still in flight
static int split(int storage) {
    fpd_params p = channel(storage, 1024, 384, 10);
    fpd_sim* s = nullptr;
    EXPECT(fpd_create(&p, nullptr, &s), FPD_OK);
    const std::vector<double> R = fiber(p);
    EXPECT(fpd_init_fiber(s, R.data()), FPD_OK);
    int32_t on = -1;
    EXPECT(fpd_split_active(s, &on), FPD_OK);
    if (on != 1) {
        fprintf(stderr, "FAIL: split steps expected for storage %d\n", storage);
        return 1;
    }
    EXPECT(fpd_split_active(s, nullptr), FPD_EINVAL);
    EXPECT(fpd_split_active(nullptr, &on), FPD_EINVAL);
    fpd_launch c;
    EXPECT(fpd_get_launch(s, &c), FPD_OK);
    c.graph_chunk = 8;
    EXPECT(fpd_set_launch(s, &c), FPD_OK);
    EXPECT(fpd_step(s, 3), FPD_OK);   // a whole first step, then direct split steps
    EXPECT(fpd_capture(s, 16), FPD_OK);
    EXPECT(fpd_step(s, 16), FPD_OK);  // graph replays of split steps
    EXPECT(fpd_step(s, 5), FPD_OK);
    EXPECT(fpd_sync(s), FPD_OK);
    const std::string path = temp_path("split");
    EXPECT(fpd_save(s, path.c_str()), FPD_OK);
    EXPECT(fpd_load(s, path.c_str()), FPD_OK);
    remove(path.c_str());
    EXPECT(fpd_step(s, 4), FPD_OK);
    EXPECT(fpd_set_flags(s, FPD_FLAG_NO_SPLIT), FPD_OK);
    EXPECT(fpd_split_active(s, &on), FPD_OK);
    if (on != 0) {
        fprintf(stderr, "FAIL: FPD_FLAG_NO_SPLIT left split steps on\n");
        return 1;
    }
    EXPECT(fpd_step(s, 4), FPD_OK);
    EXPECT(fpd_set_flags(s, 0), FPD_OK);
    std::vector<double> Rb(2 * (size_t)p.n_beads);
    EXPECT(fpd_read_beads(s, Rb.data(), nullptr, nullptr), FPD_OK);
    EXPECT(fpd_step(s, 6), FPD_OK);  // left running: fpd_destroy waits for both streams
    fpd_destroy(s);
    return 0;
}

int main() {
    const int storages[3] = {FPD_F64, FPD_F32, FPD_F16DEV};
    for (int st : storages) {
        printf("[asan] lifecycle storage %d\n", st);
        fflush(stdout);
        if (lifecycle(st)) return 1;
    }
    const int split_storages[2] = {FPD_F32, FPD_F16DEV};
    for (int st : split_storages) {
        printf("[asan] split steps storage %d\n", st);
        fflush(stdout);
        if (split(st)) return 1;
    }
    printf("[asan] invalid arguments\n");
    fflush(stdout);
    if (invalid_arguments()) return 1;
    printf("[asan] batch\n");
    fflush(stdout);
    if (batch()) return 1;
    printf("[asan] run_static\n");
    fflush(stdout);
    if (run_static()) return 1;
    printf("[asan] all calls returned as expected\n");
    return 0;
}
