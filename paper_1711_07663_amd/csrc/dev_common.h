// Device helpers: outward FP32 rounding, order-preserving float keys, bins,
// wave-level utilities.  Included by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "oc_internal.h"

namespace oc {

constexpr double kTolHit = OC_TOL_HIT;

// Checked builds (OC_CHECKED): the CSR walks validate every index they read
// against the size of the array it indexes; a violation sets a bit of the
// context's check word (oc_check_word) and the access is skipped, so a bad
// offset is reported instead of faulting.  Product builds trust the indices
// (the check folds away).
enum : uint32_t {
    kChkSurfBin = 1u,    // a surface bin's entry range outside the batch's records
    kChkSurfFace = 2u,   // a surface bin record naming a face outside its cut
    kChkDonorBin = 4u,   // a donor bin's entry range outside the grid's records
    kChkDonorElem = 8u,  // a donor bin record naming an element outside the grid
    kChkPairElem = 16u   // a (point, element) pair naming an element outside the grid
};
__device__ inline bool chk(bool ok, uint32_t *word, uint32_t code)
{
#ifdef OC_CHECKED
    if (!ok && word) atomicOr(word, code);
    return ok;
#else
    (void)ok;
    (void)word;
    (void)code;
    return true;
#endif
}
// a size read from device memory for the checks (checked builds only)
__device__ inline int64_t chk_size(const int32_t *p)
{
#ifdef OC_CHECKED
    return *p;
#else
    (void)p;
    return INT64_MAX;
#endif
}

// Round an FP64 value to the nearest FP32 value not above / not below it.
__host__ __device__ inline float f32_down(double v)
{
    float f = (float)v;
    if ((double)f > v) f = nextafterf(f, -INFINITY);
    return f;
}
__host__ __device__ inline float f32_up(double v)
{
    float f = (float)v;
    if ((double)f < v) f = nextafterf(f, INFINITY);
    return f;
}

// Order-preserving map float <-> int (min / max of floats taken on ints).
__device__ inline int f2ord(float f)
{
    int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ inline float ord2f(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

// Monotone bin index (see BinGrid).  Separate FP32 subtract and multiply,
// no contraction, clamp before the integer conversion.
__device__ inline int bin_of(float v, float o, float inv, int n)
{
    float t = __fmul_rn(__fsub_rn(v, o), inv);
    t = fminf(fmaxf(t, 0.0f), (float)(n - 1));
    return (int)t;
}

struct d3 {
    double x, y, z;
};
__device__ inline d3 mk(double x, double y, double z) { return d3{x, y, z}; }
__device__ inline d3 operator-(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline d3 operator+(d3 a, d3 b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline d3 operator*(d3 a, double s) { return d3{a.x * s, a.y * s, a.z * s}; }
__device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline d3 cross(d3 a, d3 b)
{
    return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__device__ inline d3 pose_apply(const Pose &p, d3 x)
{
    return d3{p.r[0] * x.x + p.r[1] * x.y + p.r[2] * x.z + p.t[0],
              p.r[3] * x.x + p.r[4] * x.y + p.r[5] * x.z + p.t[1],
              p.r[6] * x.x + p.r[7] * x.y + p.r[8] * x.z + p.t[2]};
}
// x = R^T (y - t)
__device__ inline d3 pose_inverse(const Pose &p, d3 y)
{
    d3 q = d3{y.x - p.t[0], y.y - p.t[1], y.z - p.t[2]};
    return d3{p.r[0] * q.x + p.r[3] * q.y + p.r[6] * q.z, p.r[1] * q.x + p.r[4] * q.y + p.r[7] * q.z,
              p.r[2] * q.x + p.r[5] * q.y + p.r[8] * q.z};
}

// Lattice node of boundary face f (order -xi,+xi,-eta,+eta,-zeta,+zeta) at
// face-lattice position (u, v) in {0,1,2}^2.
__device__ inline int elem_face_node(int f, int u, int v)
{
    const int base[6] = {0, 2, 0, 6, 0, 18};
    const int su[6] = {3, 3, 1, 1, 1, 1};
    const int sv[6] = {9, 9, 9, 9, 3, 3};
    return base[f] + su[f] * u + sv[f] * v;
}

// Triangle w (0/1) of lattice quad (m, n): corners p(m,n), p(m+1,n),
// p(m+1,n+1) and p(m,n), p(m+1,n+1), p(m,n+1); returns lattice (u,v) pairs.
__device__ inline void quad_tri_uv(int m, int n, int w, int uv[6])
{
    uv[0] = m;
    uv[1] = n;
    if (w == 0) {
        uv[2] = m + 1; uv[3] = n;
        uv[4] = m + 1; uv[5] = n + 1;
    } else {
        uv[2] = m + 1; uv[3] = n + 1;
        uv[4] = m;     uv[5] = n + 1;
    }
}

}  // namespace oc
