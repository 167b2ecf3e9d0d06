#pragma once
// Reference-element matrices of P1-P4 in constant memory.  Each translation
// unit that launches DG kernels holds its own copy (internal linkage) and
// uploads it with upload_ref before its first launch.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "dg_kernels.h"
#include "refelem.h"

namespace dgt {

static __constant__ RefC<1, double> c_ref1d;
static __constant__ RefC<2, double> c_ref2d;
static __constant__ RefC<3, double> c_ref3d;
static __constant__ RefC<4, double> c_ref4d;
static __constant__ RefC<1, float> c_ref1f;
static __constant__ RefC<2, float> c_ref2f;
static __constant__ RefC<3, float> c_ref3f;
static __constant__ RefC<4, float> c_ref4f;

template <int K, typename T>
__device__ __forceinline__ const RefC<K, T> &R();
template <> __device__ __forceinline__ const RefC<1, double> &R<1, double>() { return c_ref1d; }
template <> __device__ __forceinline__ const RefC<2, double> &R<2, double>() { return c_ref2d; }
template <> __device__ __forceinline__ const RefC<3, double> &R<3, double>() { return c_ref3d; }
template <> __device__ __forceinline__ const RefC<4, double> &R<4, double>() { return c_ref4d; }
template <> __device__ __forceinline__ const RefC<1, float> &R<1, float>() { return c_ref1f; }
template <> __device__ __forceinline__ const RefC<2, float> &R<2, float>() { return c_ref2f; }
template <> __device__ __forceinline__ const RefC<3, float> &R<3, float>() { return c_ref3f; }
template <> __device__ __forceinline__ const RefC<4, float> &R<4, float>() { return c_ref4f; }

template <int K, typename T>
static const void *ref_symbol() {
    if constexpr (std::is_same<T, double>::value) {
        if constexpr (K == 1) return (const void *)&HIP_SYMBOL(c_ref1d);
        if constexpr (K == 2) return (const void *)&HIP_SYMBOL(c_ref2d);
        if constexpr (K == 3) return (const void *)&HIP_SYMBOL(c_ref3d);
        if constexpr (K == 4) return (const void *)&HIP_SYMBOL(c_ref4d);
    } else {
        if constexpr (K == 1) return (const void *)&HIP_SYMBOL(c_ref1f);
        if constexpr (K == 2) return (const void *)&HIP_SYMBOL(c_ref2f);
        if constexpr (K == 3) return (const void *)&HIP_SYMBOL(c_ref3f);
        if constexpr (K == 4) return (const void *)&HIP_SYMBOL(c_ref4f);
    }
    return nullptr;
}

template <int K, typename T>
static void upload_ref(const RefElem &E, hipStream_t st) {
    RefC<K, T> h{};
    constexpr int NP = RefC<K, T>::NP, NFP = RefC<K, T>::NFP;
    for (int i = 0; i < NP * NP; ++i) {
        h.Dr[i] = (T)E.Dr[i];
        h.Ds[i] = (T)E.Ds[i];
        h.M[i] = (T)E.M[i];
    }
    for (int i = 0; i < 3 * NP * NFP; ++i) h.lift[i] = (T)E.lift[i];
    for (int i = 0; i < 3 * NFP; ++i) h.fn[i] = E.fnodes[i];
    for (int q = 0; q < 3; ++q)
        for (int t = 0; t < NFP; ++t)
            DGT_REQUIRE(E.fnodes[q * NFP + t] == fnode(K, q, t), DGT_ESTATE, "facet node numbering mismatch");
    DGT_HIP(hipMemcpyToSymbolAsync(ref_symbol<K, T>(), &h, sizeof(h), 0, hipMemcpyHostToDevice, st));
}

}  // namespace dgt
