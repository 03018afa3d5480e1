// Host-side argument and configuration checks of the C ABI, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side (see
// tests/test_sanitize_cpu.py).  Every call here is rejected or answered
// before any device work, so the program runs without a GPU.  Exits 1 on
// the first unexpected return code.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fpic.h"
#include "fpic_particles.h"

static int failures = 0;

static void expect(int got, int want, const char *what)
{
    if (got != want) {
        std::fprintf(stderr, "%s: got %d, want %d (%s)\n", what, got, want, fpic_last_error());
        ++failures;
    }
}

struct Box {
    std::vector<double> dirs, N, Nb;
    fpic_config c;
    Box(int nx, int ny, int nz, int ndir, double dt = 0.05)
    {
        std::memset(&c, 0, sizeof c);
        for (int d = 0; d < ndir; ++d) {
            const double z = 1.0 - (2.0 * d + 1.0) / ndir, r = std::sqrt(1.0 - z * z);
            const double ph = 2.399963229728653 * d;
            dirs.push_back(r * std::cos(ph));
            dirs.push_back(r * std::sin(ph));
            dirs.push_back(z);
            N.push_back(1.0 / ndir);
            Nb.push_back(0.9 / ndir);
        }
        c.ncell[0] = nx;
        c.ncell[1] = ny;
        c.ncell[2] = nz;
        c.dx[0] = c.dx[1] = c.dx[2] = 0.25;
        c.ndir = ndir;
        c.dirs = dirs.data();
        c.N = N.data();
        c.Nbar = Nb.data();
        c.hvac[0] = 1e-3;
        c.hvac[8] = 2e-3;
        c.hvac[2] = 1e-4;
        c.hvac[6] = 1e-4;  // (0,1) and (1,0): Hermitian
        c.dt = dt;
        c.shape_order = 1;
    }
};

int main()
{
    size_t b = 0;
    // single boxes: 1D, 3D, both shapes, launch shapes
    for (int order : {1, 2}) {
        Box one(1, 1, 70, 26), three(8, 6, 5, 26);
        one.c.shape_order = three.c.shape_order = order;
        expect(fpic_workspace_bytes(&one.c, nullptr, &b), FPIC_OK, "1D box");
        expect(fpic_workspace_bytes(&three.c, nullptr, &b), FPIC_OK, "3D box");
        for (int fused : {0, 1, 2}) {
            fpic_tuning t{8, 3, 4, 0, fused};
            expect(fpic_workspace_bytes(&three.c, &t, &b), FPIC_OK, "3D launch shape");
        }
        for (int waves : {1, 2, 4}) {
            fpic_tuning t{waves, 5, 8, 2, 0};
            expect(fpic_workspace_bytes(&one.c, &t, &b), FPIC_OK, "1D launch shape");
        }
    }
    {
        Box x(1, 1, 64, 6);
        x.c.dt = 5.0;
        expect(fpic_workspace_bytes(&x.c, nullptr, &b), FPIC_EUNSUPPORTED, "dt too large");
        x.c.dt = std::nan("");
        expect(fpic_workspace_bytes(&x.c, nullptr, &b), FPIC_EINVAL, "dt nan");
        x.c.dt = 0.05;
        x.c.hvac[1] = 0.5;
        expect(fpic_workspace_bytes(&x.c, nullptr, &b), FPIC_EINVAL, "hvac not Hermitian");
        x.c.hvac[1] = 0.0;
        x.dirs[0] = 2.0;
        expect(fpic_workspace_bytes(&x.c, nullptr, &b), FPIC_EINVAL, "direction not unit");
        x.dirs[0] = 0.0;
        x.c.ncell[2] = 0;
        expect(fpic_workspace_bytes(&x.c, nullptr, &b), FPIC_EINVAL, "no cells");
        Box wide(130, 2, 2, 6);  // rows longer than a wave: x-segments
        expect(fpic_workspace_bytes(&wide.c, nullptr, &b), FPIC_OK, "3D nx > 64");
        Box wide2(300, 1, 1, 6);
        expect(fpic_workspace_bytes(&wide2.c, nullptr, &b), FPIC_OK, "3D rows of 300 cells");
        fpic_tuning t{3, 0, 0, 0, 0};
        Box y(1, 1, 64, 6);
        expect(fpic_workspace_bytes(&y.c, &t, &b), FPIC_EINVAL, "waves 3");
        fpic_tuning f{0, 0, 0, 0, 7};
        Box z(4, 4, 4, 6);
        expect(fpic_workspace_bytes(&z.c, &f, &b), FPIC_EINVAL, "fused 7");
    }
    expect(fpic_workspace_bytes(nullptr, nullptr, &b), FPIC_EINVAL, "null cfg");
    {
        Box x(1, 1, 64, 6);
        fpic_ctx *ctx = nullptr;
        expect(fpic_create(&x.c, nullptr, nullptr, 0, nullptr, &ctx), FPIC_EINVAL, "no workspace");
        expect(fpic_step(nullptr, 1), FPIC_EINVAL, "step null");
        expect(fpic_set_state(nullptr, nullptr, 0), FPIC_EINVAL, "set_state null");
        expect(fpic_moments(nullptr, nullptr), FPIC_EINVAL, "moments null");
        expect(fpic_domain_averages(nullptr, nullptr, nullptr), FPIC_EINVAL, "domain averages null");
        fpic_destroy(nullptr);
    }
    // batches of uneven boxes
    {
        std::vector<Box> boxes;
        for (int i = 0; i < 5; ++i)
            boxes.emplace_back(1, 1, 40 + 37 * i, i % 2 ? 6 : 26);
        std::vector<fpic_config> cf;
        for (auto &x : boxes)
            cf.push_back(x.c);
        expect(fpic_batch_workspace_bytes((int)cf.size(), cf.data(), nullptr, &b), FPIC_OK, "batch");
        cf[2].shape_order = 2;
        expect(fpic_batch_workspace_bytes((int)cf.size(), cf.data(), nullptr, &b), FPIC_EINVAL,
               "batch of two shape orders");
        Box three(4, 4, 4, 6);
        cf[2] = three.c;
        expect(fpic_batch_workspace_bytes((int)cf.size(), cf.data(), nullptr, &b), FPIC_EINVAL,
               "batch with a 3D box");
        expect(fpic_batch_workspace_bytes(0, cf.data(), nullptr, &b), FPIC_EINVAL, "empty batch");
        fpic_batch *bt = nullptr;
        cf[2] = boxes[2].c;
        expect(fpic_batch_create((int)cf.size(), cf.data(), nullptr, nullptr, 0, nullptr, &bt),
               FPIC_EINVAL, "batch without workspace");
    }
    // the allocation-free entry point rejects before touching a device
    {
        Box x(1, 1, 64, 6), three(4, 4, 4, 6), big(1, 1, 4096, 378);
        double dummy[8];
        expect(fpic_step_noalloc(&x.c, nullptr, nullptr, 0, 1, nullptr), FPIC_EINVAL, "noalloc null state");
        expect(fpic_step_noalloc(&x.c, nullptr, dummy, 0, -1, nullptr), FPIC_EINVAL, "noalloc negative steps");
        expect(fpic_step_noalloc(&three.c, nullptr, dummy, 0, 1, nullptr), FPIC_EUNSUPPORTED, "noalloc 3D");
        expect(fpic_step_noalloc(&big.c, nullptr, dummy, 0, 1, nullptr), FPIC_EINVAL, "noalloc too big");
    }
    // general placement
    {
        fpic_pconfig p;
        std::memset(&p, 0, sizeof p);
        p.ncell[0] = p.ncell[1] = 1;
        p.ncell[2] = 64;
        p.dx[0] = p.dx[1] = 1.0;
        p.dx[2] = 0.2;
        p.npart = 1024;
        p.dt = 0.05;
        p.shape_order = 1;
        expect(fpic_particles_workspace_bytes(&p, &b), FPIC_OK, "particles");
        p.shape_order = 2;
        expect(fpic_particles_workspace_bytes(&p, &b), FPIC_OK, "particles quadratic");
        p.ncell[0] = p.ncell[1] = 8;
        expect(fpic_particles_workspace_bytes(&p, &b), FPIC_OK, "particles 3D");
        p.npart = 0;
        expect(fpic_particles_workspace_bytes(&p, &b), FPIC_EINVAL, "particles none");
        p.npart = 1024;
        p.sort_every = 5000;
        expect(fpic_particles_workspace_bytes(&p, &b), FPIC_EINVAL, "particles sort interval");
        p.sort_every = 0;
        p.hvac[1] = 0.5;
        expect(fpic_particles_workspace_bytes(&p, &b), FPIC_EINVAL, "particles hvac");
        fpic_pctx *pc = nullptr;
        p.hvac[1] = 0.0;
        expect(fpic_particles_create(&p, nullptr, 0, nullptr, &pc), FPIC_EINVAL, "particles no workspace");
    }
    std::printf("%s: %d unexpected return codes\n", failures ? "FAILED" : "passed", failures);
    return failures ? 1 : 0;
}
