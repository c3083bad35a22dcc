// A caller of the C ABI with no Python and no torch: device buffers from
// hipMalloc, one context, the list build, density and force passes, ten
// velocity-Verlet steps, the status word, teardown.  Test infrastructure:
// tests/test_gpu_c_abi.py writes the input, runs this program and checks its
// output against the oracle.
//
// Input file (little-endian): int64 N; double L, mass, dt, skin, rc;
// double params[6] (Finnis-Sinclair c d c0 c1 c2 A); double pos[N][3];
// double vel[N][3].  Output file: double f[N][3]; double e_box; double
// pos_after[N][3] (after 10 steps); uint32 flags.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "md.h"

static int fail(const char *what, int code)
{
    std::fprintf(stderr, "%s: %d (%s)\n", what, code, code < 0 ? md_strerror(code) : "hip");
    return 1;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        std::fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
        return 2;
    }
    std::FILE *in = std::fopen(argv[1], "rb");
    if (!in) return fail("open input", 0);
    int64_t n = 0;
    double hdr[5], par[6];
    if (std::fread(&n, sizeof n, 1, in) != 1 || std::fread(hdr, sizeof(double), 5, in) != 5 ||
        std::fread(par, sizeof(double), 6, in) != 6 || n <= 0)
        return fail("read header", 0);
    std::vector<double> pos(3 * n), vel(3 * n);
    if (std::fread(pos.data(), sizeof(double), 3 * n, in) != (size_t)(3 * n) ||
        std::fread(vel.data(), sizeof(double), 3 * n, in) != (size_t)(3 * n))
        return fail("read state", 0);
    std::fclose(in);

    const double L = hdr[0];
    int64_t off[2] = {0, n};
    md_system sys = {};
    sys.n_boxes = 1;
    sys.max_neighbors = 0;
    sys.box_offset = off;
    sys.box_len = &L;
    sys.mass = hdr[1];
    sys.dt = hdr[2];
    sys.skin = hdr[3];
    md_potential pot = {};
    pot.kind = MD_POT_FS;
    pot.n_params = 6;
    pot.rc = hdr[4];
    pot.params = par;

    double *d_pos = nullptr, *d_vel = nullptr, *d_f = nullptr, *d_e = nullptr;
    if (hipMalloc(&d_pos, sizeof(double) * 3 * n) != hipSuccess ||
        hipMalloc(&d_vel, sizeof(double) * 3 * n) != hipSuccess ||
        hipMalloc(&d_f, sizeof(double) * 3 * n) != hipSuccess ||
        hipMalloc(&d_e, sizeof(double)) != hipSuccess)
        return fail("hipMalloc", 0);
    if (hipMemcpy(d_pos, pos.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_vel, vel.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice) != hipSuccess)
        return fail("hipMemcpy in", 0);

    md_ctx *ctx = nullptr;
    int rc;
    if ((rc = md_create(&sys, &pot, &ctx)) != MD_OK) return fail("md_create", rc);
    if ((rc = md_set_state(ctx, d_pos, d_vel, nullptr)) != MD_OK) return fail("md_set_state", rc);
    if ((rc = md_build_neighbors(ctx, nullptr)) != MD_OK) return fail("md_build_neighbors", rc);
    if ((rc = md_density(ctx, nullptr, nullptr)) != MD_OK) return fail("md_density", rc);
    if ((rc = md_forces(ctx, d_f, nullptr, d_e, nullptr)) != MD_OK) return fail("md_forces", rc);
    std::vector<double> f(3 * n), after(3 * n);
    double e_box = 0.0;
    if (hipMemcpy(f.data(), d_f, sizeof(double) * 3 * n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&e_box, d_e, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return fail("hipMemcpy out", 0);
    if ((rc = md_step(ctx, 10, nullptr)) != MD_OK) return fail("md_step", rc);
    if ((rc = md_get_state(ctx, d_pos, nullptr, nullptr)) != MD_OK) return fail("md_get_state", rc);
    if (hipMemcpy(after.data(), d_pos, sizeof(double) * 3 * n, hipMemcpyDeviceToHost) != hipSuccess)
        return fail("hipMemcpy after", 0);
    uint32_t flags = 0;
    int64_t counters[2] = {0, 0};
    if ((rc = md_status(ctx, nullptr, &flags, counters)) != MD_OK) return fail("md_status", rc);
    md_destroy(ctx);
    (void)hipFree(d_pos);
    (void)hipFree(d_vel);
    (void)hipFree(d_f);
    (void)hipFree(d_e);

    std::FILE *out = std::fopen(argv[2], "wb");
    if (!out) return fail("open output", 0);
    std::fwrite(f.data(), sizeof(double), 3 * n, out);
    std::fwrite(&e_box, sizeof(double), 1, out);
    std::fwrite(after.data(), sizeof(double), 3 * n, out);
    std::fwrite(&flags, sizeof flags, 1, out);
    std::fclose(out);
    std::printf("forces_from_c: %lld atoms, E = %.12f eV, flags %u\n", (long long)n, e_box, flags);
    return 0;
}
