// Drives the host side of libsal through its C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (no device: the launches are stubbed): specs, stencils (shared,
// per-plane, duplicated offsets, the union limit), line templates, fusions of every mode,
// sections and workspace sizes, on valid and invalid arguments alike.
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/sal.h"

static int failures = 0;
#define EXPECT(x)                                                            \
    do {                                                                     \
        if (!(x)) {                                                          \
            std::fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #x, sal_last_error()); \
            failures++;                                                      \
        }                                                                    \
    } while (0)

int main() {
    void* p = (void*)0x100;
    // specs
    for (int n = 0; n <= 20; n++)
        for (int s = 0; s <= n; s++) {
            sal_spec sp = {n, s, 0, 0, 0};
            (void)sal_project((const float*)p, 8, 9, 10, &sp, (float*)p, nullptr);
        }
    // shared stencils: every size up to the limit, with and without weights, literal or not
    std::vector<int32_t> off(3 * 70);
    std::vector<float> w(70, 0.5f);
    for (int k = 0; k < 70; k++) {
        off[3 * k] = 2 * (k % 5) - 4;
        off[3 * k + 1] = 2 * (k % 3);
        off[3 * k + 2] = -2 * (k % 7);
    }
    for (int q = 0; q <= 66; q++)
        for (int lit = 0; lit < 2; lit++) {
            sal_stencil st = {q, off.data(), (q & 1) ? w.data() : nullptr, lit, nullptr};
            sal_status rc = sal_center_surround((const float*)p, 0, 4, 4, 2, &st, (float*)p + 64, nullptr);
            EXPECT((q >= 1 && q <= SAL_MAX_STENCIL && !(q == 1 && off[0] == 0 && off[1] == 0 && off[2] == 0))
                       ? rc == SAL_OK || rc == SAL_ERR_ARG : rc == SAL_ERR_ARG);
        }
    // per-plane stencils from line templates, duplicated offsets, and a union past the limit
    int32_t dirs[3][3] = {{2, 0, 0}, {0, 0, 2}, {2, 0, 2}};
    int32_t toff[3][2 * 32 * 3];
    float tw[3][2 * 32];
    for (int m = 0; m < 3; m++) EXPECT(sal_line_template(dirs[m], 32, 3.0, toff[m], tw[m]) == SAL_OK);
    EXPECT(sal_line_template(dirs[0], 33, 3.0, toff[0], tw[0]) == SAL_ERR_ARG);
    for (int L = 1; L <= 32; L++) {
        sal_stencil planes[3];
        for (int m = 0; m < 3; m++) planes[m] = {2 * L, toff[m], (m == 1) ? nullptr : tw[m], 0, nullptr};
        sal_stencil st = {0, nullptr, nullptr, 0, planes};
        sal_status rc = sal_center_surround((const float*)p, 0, 4, 4, 2, &st, (float*)p + 64, nullptr);
        // the union of the three lines holds 6L distinct offsets
        EXPECT(6 * L <= SAL_MAX_STENCIL ? rc == SAL_OK : rc == SAL_ERR_ARG);
    }
    {
        int32_t dup[12] = {2, 0, 0, 2, 0, 0, -2, 0, 0, -2, 0, 0};
        sal_stencil planes[3] = {{4, dup, nullptr, 0, nullptr}, {4, dup, nullptr, 1, nullptr}, {2, dup, nullptr, 0, nullptr}};
        sal_stencil st = {0, nullptr, nullptr, 0, planes};
        EXPECT(sal_center_surround((const float*)p, 0, 4, 4, 2, &st, (float*)p + 64, nullptr) == SAL_OK);
    }
    // fusions
    for (int mode = 0; mode <= 6; mode++)
        for (int64_t sections = -1; sections <= 3; sections++) {
            sal_fusion f = {mode, {0.2, 0.3, 0.5}, 0.5, sections, 0.1, 1e-6, 0.9, 2};
            (void)sal_fuse_groups(&f, 7);
            size_t ws = sal_fuse_workspace_size(4, 7, 5, &f);
            std::vector<unsigned char> buf(ws + 1);
            (void)sal_fuse((const float*)p, 4, 7, 5, &f, (const float*)p, nullptr, 8, 14, 10, 2, (double*)p,
                           (float*)p, buf.data(), ws, nullptr);
            (void)sal_adapt_weights((const float*)p, 4, 7, 5, &f, (const float*)p, nullptr, (double*)p, (float*)p, 8,
                                    nullptr, buf.data(), ws, nullptr);
        }
    std::printf(failures ? "HOST_SANITIZE_FAILED\n" : "HOST_SANITIZE_OK\n");
    return failures ? 1 : 0;
}
