// Host run of the library's FP64 refinement traversal (exact_traverse.h): prints
// every nonzero of A for one frame as "ray voxel length", with the public
// layouts (ray = (view * nv + iv) * nu + iu, voxel = (iz * ny + iy) * nx + ix),
// so the test can compare it with the FP64 oracle's matrix.
// Usage: exact_rows nx ny nz nu nv du dv src_iso src_det off_u off_v angle...
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "exact_traverse.h"

int main(int argc, char **argv)
{
    if (argc < 13) return 2;
    ExactArgs A{};
    A.nx = atoi(argv[1]); A.ny = atoi(argv[2]); A.nz = atoi(argv[3]);
    A.nu = atoi(argv[4]); A.nv = atoi(argv[5]); A.nf = 1;
    A.du = atof(argv[6]); A.dv = atof(argv[7]); A.rs = atof(argv[8]); A.rsd = atof(argv[9]);
    A.offu = atof(argv[10]); A.offv = atof(argv[11]);
    std::vector<double2> cs;
    for (int k = 12; k < argc; ++k) {
        const double t = atof(argv[k]);
        cs.push_back(double2{std::cos(t), std::sin(t)});
    }
    A.cs = cs.data();
    A.n_views = (int64_t)cs.size();
    A.nvox = (int64_t)A.nx * A.ny * A.nz;
    for (int64_t view = 0; view < A.n_views; ++view)
        for (int iv = 0; iv < A.nv; ++iv)
            for (int iu = 0; iu < A.nu; ++iu) {
                double S[3], d[3];
                ray_of(A, view, iu, iv, S, d);
                const int64_t ray = (view * A.nv + iv) * A.nu + iu;
                traverse(A, S, d, [&](int64_t vox, double len) {
                    const int64_t iz = vox % A.nz, c = vox / A.nz;
                    const int64_t ix = c % A.nx, iy = c / A.nx;
                    printf("%lld %lld %.17g\n", (long long)ray, (long long)((iz * A.ny + iy) * A.nx + ix), len);
                });
            }
    return 0;
}
