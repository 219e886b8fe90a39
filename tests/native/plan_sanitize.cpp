// Host-only driver of the library's setup code (plan.cpp, tri.cpp) for an AddressSanitizer /
// UndefinedBehaviorSanitizer build with g++: reads meshes written by the test, runs the plan
// (numbering, geometry, every element order, tiling, colouring, snapping) and prints a digest.
// Usage: plan_sanitize <mesh file>... ; file = int64 nv, ne, nvpe, p; double vxy[2 nv];
// int32 elems[ne * nvpe]; double c2[ne]. Exit status 0 when every plan was built.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../../paper_2104_08416_amd/csrc/plan.h"

int main(int argc, char** argv) {
    for (int f = 1; f < argc; ++f) {
        FILE* fp = std::fopen(argv[f], "rb");
        if (!fp) { std::fprintf(stderr, "cannot open %s\n", argv[f]); return 2; }
        int64_t hdr[4];
        if (std::fread(hdr, sizeof(int64_t), 4, fp) != 4) return 2;
        const int64_t nv = hdr[0], ne = hdr[1], nvpe = hdr[2], p = hdr[3];
        std::vector<double> vxy(2 * nv), c2(ne);
        std::vector<int32_t> el(ne * nvpe);
        if (std::fread(vxy.data(), sizeof(double), vxy.size(), fp) != vxy.size()) return 2;
        if (std::fread(el.data(), sizeof(int32_t), el.size(), fp) != el.size()) return 2;
        if (std::fread(c2.data(), sizeof(double), c2.size(), fp) != c2.size()) return 2;
        std::fclose(fp);
        sem::MeshIn m;
        m.nv = nv;
        m.ne = ne;
        m.vxy = vxy.data();
        m.quad = el.data();
        m.c2 = c2.data();
        m.nvpe = (int)nvpe;
        for (int order = 0; order <= 5; ++order) {
            for (int split = 0; split <= 1; ++split) {
                sem::PlanOptions o;
                o.p = (int)p;
                o.elem_order = order;
                o.tile_items = 40;
                o.max_owned = split ? 64 : 1 << 30;
                o.split_single = split != 0;
                sem::Plan P;
                int code = 0;
                const std::string err = sem::build_plan(m, o, P, code);
                if (!err.empty()) { std::fprintf(stderr, "%s: %s\n", argv[f], err.c_str()); return 1; }
                const double pts[6] = {vxy[0] + 0.3, vxy[1] + 0.2, -1e6, 3e6, vxy[2], vxy[3]};
                int32_t near[3];
                sem::nearest_nodes(P, 3, pts, near);
                const int32_t node = near[0];
                std::printf("%s order %d split %d: nodes %lld tiles %zu halo %zu colours %d node %d\n", argv[f],
                            order, split, (long long)P.nn, P.tile_eb.size() - 1, P.halo.size(), P.n_colours, node);
            }
        }
    }
    return 0;
}
