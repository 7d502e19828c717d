// Device helpers shared by several translation units.
#pragma once
#include "common.h"

#include <type_traits>

namespace hts {

// Pointers read out of device-resident descriptors are generic; reading
// through a global-address-space pointer gives global (not flat) loads,
// which do not count against the LDS wait of a barrier.
#define HTS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ static const T HTS_GLOBAL *gptr(const void *p)
{
    return (const T HTS_GLOBAL *)p;
}

struct ColInfo {
    int64_t base;   // instance-local index of the node at k = 0
    int valid;
    int xyc;        // constrained by an x or y face
    int dlo, dhi;   // constrained z range from Dirichlet columns
};

__device__ __forceinline__ static ColInfo col_info(const OpDev &o, int i, int j)
{
    ColInfo c;
    c.valid = (i >= 0 && i < o.NX && j >= 0 && j < o.NY);
    c.base = c.valid ? (int64_t)i + (int64_t)o.NX * j : 0;
    const int m = o.dmask;
    c.xyc = c.valid && (((m & 1) && i == 0) || ((m & 2) && i == o.NX - 1) || ((m & 4) && j == 0) ||
                        ((m & 8) && j == o.NY - 1));
    int packed = (c.valid && o.dcol) ? gptr<int32_t>(o.dcol)[c.base] : DCOL_NONE;
    c.dlo = packed & 0xFFFF;
    c.dhi = (packed >> 16) & 0xFFFF;
    return c;
}

__device__ __forceinline__ static bool constrained(const ColInfo &c, int k, int NZ, int m)
{
    return c.xyc || ((m & 16) && k == 0) || ((m & 32) && k == NZ - 1) || (k >= c.dlo && k <= c.dhi);
}

// Element i of an instance vector through a 32-bit byte offset from a
// uniform base (one vector of an instance stays below 4 GiB: meshes have
// fewer than 2^29 nodes), so the loads and stores take
// the scalar-base plus 32-bit-offset address form without 64-bit address
// arithmetic per lane.
template <typename P>
__device__ __forceinline__ P *at32(P *base, uint32_t i)
{
    using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    return reinterpret_cast<P *>(reinterpret_cast<C *>(base) + i * (uint32_t)sizeof(P));
}
template <typename P>
__device__ __forceinline__ const P HTS_GLOBAL *at32(const P HTS_GLOBAL *base, uint32_t i)
{
    return reinterpret_cast<const P HTS_GLOBAL *>(reinterpret_cast<const char HTS_GLOBAL *>(base) +
                                                  i * (uint32_t)sizeof(P));
}

__device__ __forceinline__ static double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}


// Node (i, j, k) of instance-local index n.
__device__ __forceinline__ static void node_ijk(const OpDev &o, int64_t n, int &i, int &j, int &k)
{
    i = (int)(n % o.NX);
    j = (int)((n / o.NX) % o.NY);
    k = (int)(n / ((int64_t)o.NX * o.NY));
}

__device__ __forceinline__ static bool node_constrained(const OpDev &o, int64_t n)
{
    int i, j, k;
    node_ijk(o, n, i, j, k);
    ColInfo c = col_info(o, i, j);
    return constrained(c, k, o.NZ, o.dmask);
}

}  // namespace hts
