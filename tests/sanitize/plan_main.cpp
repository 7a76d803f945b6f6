// Host-side sanitizer harness: builds the plan (mesh preprocessing, fused-FV tiles,
// workspace layout) and runs hlbm_workspace_size and hlbm_validate for each input
// file written by dump_inputs.py; run.sh builds it with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code.
#include <cstdio>
#include <cstring>
#include <vector>
#include "hlbm_internal.h"

int main(int argc, char** argv) {
    for (int a = 1; a < argc; ++a) {
        FILE* f = fopen(argv[a], "rb");
        if (!f) return 2;
        int gl, z; double zd, ell[4], chord;
        if (fread(&gl, 4, 1, f) != 1 || fread(&z, 4, 1, f) != 1 || fread(&zd, 8, 1, f) != 1 ||
            fread(ell, 8, 4, f) != 4 || fread(&chord, 8, 1, f) != 1) return 3;
        if (gl != int(sizeof(hlbm_grid))) { printf("grid size %d vs %zu\n", gl, sizeof(hlbm_grid)); return 4; }
        hlbm_grid g;
        if (fread(&g, gl, 1, f) != 1) return 5;
        int nn, nt;
        if (fread(&nn, 4, 1, f) != 1 || fread(&nt, 4, 1, f) != 1) return 6;
        std::vector<double> xy(2 * size_t(nn));
        std::vector<int32_t> tri(3 * size_t(nt));
        std::vector<uint8_t> kind(nn);
        double tau;
        if (fread(xy.data(), 8, xy.size(), f) != xy.size() || fread(tri.data(), 4, tri.size(), f) != tri.size() ||
            fread(kind.data(), 1, kind.size(), f) != kind.size() || fread(&tau, 8, 1, f) != 1) return 7;
        fclose(f);
        hlbm_mesh m;
        std::memset(&m, 0, sizeof(m));
        m.n_nodes = nn; m.n_tris = nt; m.xy = xy.data(); m.tri = tri.data(); m.kind = kind.data();
        m.chord = chord;
        for (int i = 0; i < 4; ++i) m.inner_ellipse[i] = ell[i];
        hlbm::Plan p;
        std::string err;
        const int rc = hlbm::build_plan(&g, &m, 0.0, tau, p, err);
        size_t ws = 0;
        const int rc2 = hlbm_workspace_size(&g, &m, 0.0, tau, &ws);
        const int rc3 = hlbm_validate(&g, &m, 0.0, tau);
        printf("%s: rc %d %d %d nn %d fuse %d tiles %d tile %d maxl %d maxw %d threads %d ws %zu %s\n", argv[a], rc,
               rc2, rc3, p.nn, p.fv_fuse, p.n_tiles, p.fv_tile, p.fv_maxl, p.fv_maxw, p.fv_threads, ws,
               err.c_str());
    }
    return 0;
}
