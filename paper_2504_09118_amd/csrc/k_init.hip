// Seeded random initial state generated on the device.
//
// The cavity workloads start from a "random initial state" (Fig. 1b, Sec. 4)
// with PEC walls. E components are drawn from SplitMix64 (Steele, Lea and
// Flood, OOPSLA 2014) used counter-style: output c of seed s is
// mix64(s + (c + 1) * 0x9E3779B97F4A7C15 mod 2^64), u = (output >> 11) 2^-53,
// value 2u - 1 computed in FP64 and rounded once to the storage type (FP32
// first for 16-bit storage). The counter of component f (0, 1, 2 for Ex, Ey,
// Ez) at the x-fastest linear index l of its staggered array is (f << 40) + l.
// Wall-tangential E is 0 (PEC) and H = 0. Generating on the device avoids a
// host round trip when requests are admitted at a high rate.
#include "fdtd_internal.h"
#include "storage.h"

namespace fdtd {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ unsigned long long mix64(unsigned long long z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_random(Geom g, int field, int X, int Y, long long n,
                                                        unsigned long long seed, T *dst, T *dst2, double scale)
{
    const long long l = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    const int i = (int)(l % X);
    const long long r = l / X;
    const int j = (int)(r % Y);
    const int k = (int)(r / Y);
    typename Store<T>::C v = 0;
    if (field < 3) {
        bool wall;
        if (field == 0)
            wall = j == 0 || j == g.ny || k == 0 || k == g.nz;
        else if (field == 1)
            wall = i == 0 || i == g.nx || k == 0 || k == g.nz;
        else
            wall = i == 0 || i == g.nx || j == 0 || j == g.ny;
        if (!wall) {
            const unsigned long long c = ((unsigned long long)field << 40) + (unsigned long long)l;
            const unsigned long long z = mix64(seed + (c + 1ull) * 0x9E3779B97F4A7C15ull);
            const double u = (double)(z >> 11) * 0x1.0p-53;
            v = to_compute<T>((2.0 * u - 1.0) * scale);  // exact for scale 1
        }
    }
    const long long o = g.at(i, j, k);
    put_elem(dst, g.lo_rec(field), o, v);
    if (dst2)
        put_elem(dst2, g.lo_rec(field), o, v);
}

}  // namespace

template <typename T>
hipError_t launch_init_random(const Geom &g, unsigned long long seed, T *const a[6], T *const b[6], hipStream_t s,
                              const double *scale)
{
    for (int f = 0; f < 6; ++f) {
        int X, Y, Z;
        extents(g, f, X, Y, Z);
        const long long n = (long long)X * Y * Z;
        hipLaunchKernelGGL((k_init_random<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g,
                           f, X, Y, n, seed, a[f], b[f], scale ? scale[f % 3] : 1.0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template hipError_t launch_init_random<float>(const Geom &, unsigned long long, float *const[6], float *const[6],
                                              hipStream_t, const double *);
template hipError_t launch_init_random<double>(const Geom &, unsigned long long, double *const[6],
                                               double *const[6], hipStream_t, const double *);
template hipError_t launch_init_random<f16>(const Geom &, unsigned long long, f16 *const[6], f16 *const[6],
                                            hipStream_t, const double *);
template hipError_t launch_init_random<f16c>(const Geom &, unsigned long long, f16c *const[6], f16c *const[6],
                                             hipStream_t, const double *);
template hipError_t launch_init_random<bf16c>(const Geom &, unsigned long long, bf16c *const[6], bf16c *const[6],
                                              hipStream_t, const double *);
template hipError_t launch_init_random<bf16>(const Geom &, unsigned long long, bf16 *const[6], bf16 *const[6],
                                             hipStream_t, const double *);

}  // namespace fdtd
