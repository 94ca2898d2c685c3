// Runs the simulated-device scenarios of the scheduling core in one
// process, for a build under AddressSanitizer and UndefinedBehaviorSanitizer
// (the tests compile it with g++ and expect exit status 0 and no report).
#include <cstdint>
#include <cstdio>

extern "C" {
void *sim_create(const int64_t *cfg, const double *per, const double *tm);
void sim_destroy(void *h);
int32_t sim_admit(void *h, int64_t src_frames, int32_t host, double start_s, int64_t total_frames);
int sim_run(void *h, double seconds, int64_t *istats, double *dstats);
}

static int scenario(int64_t dump, int64_t ring, int64_t inflight, int64_t slots, int64_t stagger, double frame_us,
                    double launch_us, double t_frame, int n_chans, int host, int64_t total, double seconds)
{
    const int64_t cfg[10] = {256, dump, ring, inflight, slots, stagger, 1000, 100, 1000 * slots + 100 * n_chans, 0};
    const double per[2] = {frame_us, launch_us};
    const double tm[5] = {20.0, 20.0, 50.0, t_frame, 10.0};
    void *h = sim_create(cfg, per, tm);
    for (int c = 0; c < n_chans; ++c) sim_admit(h, 5 + c, host, 0.0001 * c, total);
    int64_t ist[10];
    double dst[4];
    int rc = sim_run(h, seconds, ist, dst);
    if (rc == 0 && ist[6] != 0) rc = 1;   // violations
    if (rc == 0) rc = sim_run(h, seconds / 2, ist, dst);   // a second run continues the first
    if (rc == 0 && ist[6] != 0) rc = 1;
    std::printf("scenario dump=%lld ring=%lld chans=%d: rc=%d done=%lld dropped=%lld\n", (long long)dump,
                (long long)ring, n_chans, rc, (long long)ist[1], (long long)ist[2]);
    sim_destroy(h);
    return rc;
}

int main()
{
    int rc = 0;
    rc |= scenario(16, 8, 2, 4, 0, 655.36, 2000.0, 5.0, 4, 0, 0, 0.2);
    rc |= scenario(16, 8, 2, 4, 1, 655.36, 2000.0, 5.0, 6, 0, 40, 0.2);
    rc |= scenario(32, 8, 1, 1, 0, 100.0, 500.0, 80.0, 1, 1, 600, 0.2);
    rc |= scenario(16, 3, 1, 2, 0, 200.0, 20000.0, 5.0, 3, 1, 48, 0.3);
    return rc;
}
