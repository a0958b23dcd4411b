// Host-side paths of the C ABI under AddressSanitizer / UBSan (no GPU needed):
// a host-only context (device = -1) through every set_* call with valid and
// invalid arguments, the consistency checks of dct_solve, the status codes and
// messages.  Exit status 0 when every call returns what the header states.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dctsn.h"

static int fails = 0;
#define EXPECT(call, code)                                                                  \
    do {                                                                                    \
        int rc_ = (call);                                                                   \
        if (rc_ != (code)) {                                                                \
            std::printf("FAIL %s:%d: %s -> %d, expected %d\n", __FILE__, __LINE__, #call, rc_, \
                        (int)(code));                                                       \
            ++fails;                                                                        \
        }                                                                                   \
    } while (0)

int main()
{
    dct_ctx *c = nullptr;
    EXPECT(dct_create(nullptr, -1, nullptr), DCT_EINVAL);
    EXPECT(dct_create(&c, -1, nullptr), DCT_OK);
    const int nx = 7, ny = 5, nz = 3, C = nx * ny * nz;
    std::vector<uint8_t> mat(C, 0);
    std::vector<double> rho(C, 1.0);
    const double org[3] = {-2.1, -1.5, -0.9};
    for (int v = 0; v < C; ++v) mat[v] = (uint8_t)(v % 2);
    EXPECT(dct_set_geometry(c, 0, ny, nz, 0.6, 0.6, 0.6, org, mat.data(), rho.data()), DCT_EINVAL);
    EXPECT(dct_set_geometry(c, nx, ny, nz, -0.6, 0.6, 0.6, org, mat.data(), rho.data()), DCT_EINVAL);
    rho[3] = -1.0;
    EXPECT(dct_set_geometry(c, nx, ny, nz, 0.6, 0.6, 0.6, org, mat.data(), rho.data()), DCT_EINVAL);
    rho[3] = NAN;
    EXPECT(dct_set_geometry(c, nx, ny, nz, 0.6, 0.6, 0.6, org, mat.data(), rho.data()), DCT_EINVAL);
    rho[3] = 1.0;
    EXPECT(dct_set_geometry(c, 4096, 4096, 4096, 0.6, 0.6, 0.6, org, mat.data(), rho.data()), DCT_EINVAL);
    EXPECT(dct_set_geometry(c, nx, ny, nz, 0.6, 0.6, 0.6, org, mat.data(), rho.data()), DCT_OK);
    const int G = 2, M = 2, L = 1;
    std::vector<double> st(M * G, 0.3), ss(M * (L + 1) * G * G, 0.0), ka(M * G, 1.0);
    const double edges[3] = {120.0, 65.0, 10.0};
    for (int m = 0; m < M; ++m)
        for (int l = 0; l <= L; ++l) {
            ss[((m * (L + 1) + l) * G + 0) * G + 0] = 0.1 / (l + 1);
            ss[((m * (L + 1) + l) * G + 0) * G + 1] = 0.05 / (l + 1);
            ss[((m * (L + 1) + l) * G + 1) * G + 1] = 0.1 / (l + 1);
        }
    ss[((0 * (L + 1) + 0) * G + 1) * G + 0] = 0.01;   // upscatter: rejected
    EXPECT(dct_set_xs(c, G, edges, M, L, st.data(), ss.data(), ka.data()), DCT_EINVAL);
    ss[((0 * (L + 1) + 0) * G + 1) * G + 0] = 0.0;
    EXPECT(dct_set_xs(c, 0, edges, M, L, st.data(), ss.data(), ka.data()), DCT_EINVAL);
    EXPECT(dct_set_xs(c, G, edges, M, 9, st.data(), ss.data(), ka.data()), DCT_EINVAL);
    EXPECT(dct_set_xs(c, G, edges, M, L, st.data(), ss.data(), ka.data()), DCT_OK);
    // S2: the 8 octant directions (1, 1, 1)/sqrt(3), weight pi / 2
    std::vector<double> dirs, w;
    const double a = 1.0 / std::sqrt(3.0);
    for (int o = 0; o < 8; ++o) {
        dirs.push_back(o & 1 ? -a : a);
        dirs.push_back(o & 2 ? -a : a);
        dirs.push_back(o & 4 ? -a : a);
        w.push_back(M_PI / 2.0);
    }
    EXPECT(dct_set_quadrature(c, 0, dirs.data(), w.data()), DCT_EINVAL);
    EXPECT(dct_set_quadrature(c, 8, dirs.data(), w.data()), DCT_OK);
    const double pos_in[3] = {0.5, 0.3, 0.0}, pos[3] = {0.0, 20.0, 0.0}, pos_axis[3] = {0.0, 0.0, 5.0};
    const double gw[2] = {0.6, 0.4};
    EXPECT(dct_set_source(c, 1, pos, nullptr, 0.0, 10.0, gw), DCT_EINVAL);     // fan 0
    EXPECT(dct_set_source(c, 1, pos_axis, nullptr, 20.0, 10.0, gw), DCT_EINVAL); // no direction toward the z axis
    EXPECT(dct_set_source(c, 1, pos_in, nullptr, 20.0, 10.0, gw), DCT_OK);     // inside: checked by the solve
    dct_opts o;
    std::memset(&o, 0, sizeof(o));
    o.precision = DCT_FP64;
    o.tol = 1e-6;
    o.max_iter = 10;
    o.fixup = 1;
    // host-only context: every check up to the device part runs, then EDEVICE
    EXPECT(dct_solve(c, &o, nullptr), DCT_EDEVICE);
    EXPECT(dct_set_source(c, 1, pos, nullptr, 20.0, 10.0, gw), DCT_OK);
    o.precision = 7;
    EXPECT(dct_solve(c, &o, nullptr), DCT_EDEVICE);
    std::vector<double> dose(C);
    EXPECT(dct_dose(c, dose.data(), 1, nullptr, nullptr), DCT_ESTATE);
    EXPECT(dct_adjoint(c, dose.data(), nullptr, nullptr, nullptr, nullptr, nullptr), DCT_ESTATE);
    const double E[2] = {20.0, 100.0}, f[2] = {1.0, 2.0};
    EXPECT(dct_effective_dose(c, 2, E, f, nullptr, dose.data(), 1), DCT_ESTATE);
    EXPECT(dct_effective_dose_noalloc(c, 2, E, f, nullptr, dose.data(), 1), DCT_EDEVICE);
    if (std::strlen(dct_last_error(c)) == 0) {
        std::printf("FAIL: empty error message\n");
        ++fails;
    }
    EXPECT(dct_destroy(c), DCT_OK);
    EXPECT(dct_destroy(nullptr), DCT_OK);
    std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
