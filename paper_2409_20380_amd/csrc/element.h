// element.h -- device code shared by the element-by-element kernels of the
// single-case path (kernels.hip) and the batched path (batch.hip): wavefront
// and workgroup reductions, storage conversions, tetrahedron geometry and the
// matrix-free P2 element operator.
//
// Element operator without element matrices.  The displacement gradient of
// a straight P2 tet is linear, so it is fixed by its values H_k at the four
// vertices:  H_k = sum_{j != k} (4 u_kj - u_j - 3 u_k) (x) grad L_j.
// The stress is linear too, sigma = sum_k L_k sigma_k, and with
// int L_a L_b dV = V (1 + delta_ab) / 20 the internal forces are
//   vertex k:     f_k  = (V/20) (4 sigma_k - S) grad L_k,
//   edge (k, j):  f_kj = (V/5) ((sigma_k + S) grad L_j + (sigma_j + S) grad L_k),
// with S = sum_k sigma_k.  The consistent mass uses the P2 mass table
// (units rho V / 420: vertex diagonal 6, vertex-vertex 1, vertex-edge -4 if
// incident else -6, edge diagonal 32, edges sharing a vertex 16, opposite 8).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"

namespace ebe {

typedef double double4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    // fixed butterfly order over the 64 lanes: deterministic
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// 8 XCDs receive workgroups round-robin; give each XCD a contiguous block of
// patches so neighbouring patches (which share nodes) hit the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    int per = nb >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// Sum of n partials p[0..n) as seen by one lane of nlanes: the lane loads its
// strided share (at most PER values) all at once, then adds in a fixed order.
template <int PER>
__device__ __forceinline__ double lane_partials(const double* __restrict__ p, int n, int lane, int nlanes) {
    double v[PER];
    // loads unconditional (index clamped into [0, n), n >= 1), so that the
    // partials of several arrays are in flight together
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = lane + k * nlanes;
        const double t = p[i < n ? i : n - 1];
        v[k] = i < n ? t : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) s += v[k];
    return s;
}

// Everything the element kernels read (topology, coordinates, materials and
// the input vectors) is read-only for the duration of a launch: those loads go
// through the constant address space.  Uniform ones become scalar loads
// (scalar cache), and the compiler may move all of them across the kernel's
// own stores, so they do not queue behind slot or direction stores in the
// in-order vector-memory counter.
template <class X>
__device__ __forceinline__ X ld_ro(const X* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(4))) X*)p;
#else
    return *p;   // host pass: never executed
#endif
}

struct PatchMeta {
    int pn0, npn, nv, e0, ne;
};
__device__ __forceinline__ PatchMeta patch_meta(const DevPatches& P, int patch) {
    PatchMeta m;
    m.pn0 = ld_ro(P.pn_ptr + patch);
    m.npn = ld_ro(P.pn_ptr + patch + 1) - m.pn0;
    m.nv = ld_ro(P.nv + patch);
    m.e0 = ld_ro(P.el_ptr + patch);
    m.ne = ld_ro(P.el_ptr + patch + 1) - m.e0;
    return m;
}

template <bool B>
using Bool = std::integral_constant<bool, B>;

// Copies the material table (lambda, mu, rho per material) into LDS at lmat.
__device__ __forceinline__ void stage_material_table(const DevPatches& P, double* lmat, int nthreads) {
    for (int i = threadIdx.x; i < 3 * P.n_mat; i += nthreads) lmat[i] = ld_ro(P.mat + i);
}

__device__ __forceinline__ void lds_add(double* p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Storage conversions.  bf16_t holds the upper 16 bits of an IEEE binary32;
// rounding to it is round-to-nearest-even (the native conversion).
template <class T, class S>
__device__ __forceinline__ T from_storage(S v) { return (T)v; }
template <>
__device__ __forceinline__ float from_storage<float, bf16_t>(bf16_t v) {
    return __uint_as_float((uint32_t)v.bits << 16);
}
template <class S, class T>
__device__ __forceinline__ S to_storage(T v) { return (S)v; }
template <>
__device__ __forceinline__ bf16_t to_storage<bf16_t, float>(float v) {
    return bf16_t{__builtin_bit_cast(uint16_t, (__bf16)v)};   // native round to nearest even
}

template <class T>
struct GeoT {
    T g[4][3];
    T V;
};

// Barycentric gradients of a straight tetrahedron: rows of J^{-1} with
// J = [x1-x0, x2-x0, x3-x0]; grad L0 = -(grad L1 + grad L2 + grad L3).
template <class T>
__device__ __forceinline__ void tet_geo(const T* x0, const T* x1, const T* x2, const T* x3, GeoT<T>& G) {
    T a0 = x1[0] - x0[0], a1 = x2[0] - x0[0], a2 = x3[0] - x0[0];
    T b0 = x1[1] - x0[1], b1 = x2[1] - x0[1], b2 = x3[1] - x0[1];
    T c0 = x1[2] - x0[2], c1 = x2[2] - x0[2], c2 = x3[2] - x0[2];
    T m00 = b1 * c2 - b2 * c1, m01 = a2 * c1 - a1 * c2, m02 = a1 * b2 - a2 * b1;
    T m10 = b2 * c0 - b0 * c2, m11 = a0 * c2 - a2 * c0, m12 = a2 * b0 - a0 * b2;
    T m20 = b0 * c1 - b1 * c0, m21 = a1 * c0 - a0 * c1, m22 = a0 * b1 - a1 * b0;
    T det = a0 * m00 + a1 * m10 + a2 * m20;
    T id = T(1) / det;
    G.g[1][0] = m00 * id; G.g[1][1] = m01 * id; G.g[1][2] = m02 * id;
    G.g[2][0] = m10 * id; G.g[2][1] = m11 * id; G.g[2][2] = m12 * id;
    G.g[3][0] = m20 * id; G.g[3][1] = m21 * id; G.g[3][2] = m22 * id;
#pragma unroll
    for (int d = 0; d < 3; ++d) G.g[0][d] = -(G.g[1][d] + G.g[2][d] + G.g[3][d]);
    G.V = det * T(1.0 / 6.0);
}
using Geo = GeoT<double>;

// local edge index (4..9) of the vertex pair (k, j)
__device__ __forceinline__ constexpr int edge_of(int k, int j) {
    const int a = k < j ? k : j, b = k < j ? j : k;
    return a == 0 ? (b == 1 ? 4 : b == 2 ? 6 : 7) : a == 1 ? (b == 2 ? 5 : 8) : 9;
}

// f = mc * Mhat pm + K pk for one element (Mhat: P2 mass table in units of
// rho V / 420, scaled into mc; K with lamV = ck lam V/20, muV = ck mu V/20),
// each node's 3-vector handed to emit(i, f0, f1, f2) as soon as it is formed:
// the 30 outputs are never all live, which keeps register pressure down.
template <class T, class Emit>
__device__ __forceinline__ void element_apply_emit(const T (&pm)[10][3], const T (&pk)[10][3], const GeoT<T>& G,
                                                   T lamV, T muV, T mc, Emit&& emit) {
    T sg[4][6];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j == k) continue;
            const int e = edge_of(k, j);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T d = T(4) * pk[e][c] - pk[j][c] - T(3) * pk[k][c];
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) H[c][dd] = fma(d, G.g[j][dd], H[c][dd]);
            }
        }
        T tr = lamV * (H[0][0] + H[1][1] + H[2][2]);
        T m2 = T(2) * muV;
        sg[k][0] = fma(m2, H[0][0], tr);
        sg[k][1] = fma(m2, H[1][1], tr);
        sg[k][2] = fma(m2, H[2][2], tr);
        sg[k][3] = muV * (H[0][1] + H[1][0]);
        sg[k][4] = muV * (H[0][2] + H[2][0]);
        sg[k][5] = muV * (H[1][2] + H[2][1]);
    }
    T S[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) S[t] = (sg[0][t] + sg[1][t]) + (sg[2][t] + sg[3][t]);
    T Pv[3], Pe[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Pv[c] = (pm[0][c] + pm[1][c]) + (pm[2][c] + pm[3][c]);
        Pe[c] = (pm[4][c] + pm[5][c]) + (pm[6][c] + pm[7][c]) + (pm[8][c] + pm[9][c]);
    }
    // vertices: stiffness (4 sigma_k - S) g_k, mass row 5 p_k + Pv - 6 Pe + 2 (incident edges)
    constexpr int INC[4][3] = {{4, 6, 7}, {4, 5, 8}, {5, 6, 9}, {7, 8, 9}};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T t[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) t[q] = fma(T(4), sg[k][q], -S[q]);
        const T* g = G.g[k];
        T f[3];
        f[0] = t[0] * g[0] + t[3] * g[1] + t[4] * g[2];
        f[1] = t[3] * g[0] + t[1] * g[1] + t[5] * g[2];
        f[2] = t[4] * g[0] + t[5] * g[1] + t[2] * g[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T m = fma(T(5), pm[k][c], Pv[c] - T(6) * Pe[c]) + T(2) * (pm[INC[k][0]][c] + pm[INC[k][1]][c] + pm[INC[k][2]][c]);
            f[c] = fma(mc, m, f[c]);
        }
        emit(k, f[0], f[1], f[2]);
    }
    // edges (k, j): stiffness 4 ((sigma_k + S) g_j + (sigma_j + S) g_k),
    // mass row -6 Pv + 2 (p_k + p_j) + 16 Pe + 16 p_e - 8 p_opposite
    constexpr int EV[6][3] = {{0, 1, 9}, {1, 2, 7}, {0, 2, 8}, {0, 3, 5}, {1, 3, 6}, {2, 3, 4}};
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int k = EV[m][0], j = EV[m][1], o = EV[m][2];
        const T* gj = G.g[j];
        const T* gk = G.g[k];
        T A[6], B[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            A[q] = T(4) * (sg[k][q] + S[q]);
            B[q] = T(4) * (sg[j][q] + S[q]);
        }
        T f[3];
        f[0] = A[0] * gj[0] + A[3] * gj[1] + A[4] * gj[2] + B[0] * gk[0] + B[3] * gk[1] + B[4] * gk[2];
        f[1] = A[3] * gj[0] + A[1] * gj[1] + A[5] * gj[2] + B[3] * gk[0] + B[1] * gk[1] + B[5] * gk[2];
        f[2] = A[4] * gj[0] + A[5] * gj[1] + A[2] * gj[2] + B[4] * gk[0] + B[5] * gk[1] + B[2] * gk[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T mm = fma(T(16), Pe[c], -T(6) * Pv[c]) + T(2) * (pm[k][c] + pm[j][c]) + T(16) * pm[4 + m][c] - T(8) * pm[o][c];
            f[c] = fma(mc, mm, f[c]);
        }
        emit(4 + m, f[0], f[1], f[2]);
    }
}


// z = B^{-1} r for one node, B^{-1} stored as 6 symmetric entries (xx, yy, zz, xy, xz, yz).
template <class T>
__device__ __forceinline__ void apply_binv(const T* B, T r0, T r1, T r2, T& z0, T& z1, T& z2) {
    z0 = B[0] * r0 + B[3] * r1 + B[4] * r2;
    z1 = B[3] * r0 + B[1] * r1 + B[5] * r2;
    z2 = B[4] * r0 + B[5] * r1 + B[2] * r2;
}

// Sum of the ns >= 1 matvec slots of one node starting at slot k0, in slot
// order ((s0 + s1) + s2) + ...  The first two are loaded unconditionally (a
// node with one slot reads its first twice), so that only nodes with three or
// more slots run the loop.  Callers issue their other loads of the node
// before this one: the slot values are the only ones that wait for the slot
// range.
template <class T>
__device__ __forceinline__ void sum_slots(const T* qbuf, int k0, int ns, T (&q)[3]) {
    const T* qs = qbuf + 3 * (int64_t)k0;
    const int o1 = ns > 1 ? 3 : 0;
    T qb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        q[c] = qs[c];
        qb[c] = qs[o1 + c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] = ns > 1 ? q[c] + qb[c] : q[c];
    for (int k = 2; k < ns; ++k) {
        q[0] += qs[3 * k]; q[1] += qs[3 * k + 1]; q[2] += qs[3 * k + 2];
    }
}

// Modes of the element kernels.
enum { MODE_APPLY = 0, MODE_PCG = 1, MODE_RHS = 2 };

// Sum of v over the workgroup (4 wavefronts of 64), fixed order, returned to every thread.
__device__ __forceinline__ double block_bcast_sum(double v) {
    __shared__ double red[4];
    __shared__ double out;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) out = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return out;
}

// Four block sums at once (each in the fixed order of block_bcast_sum, so the
// results are bitwise those of four separate calls), with one pair of barriers.
__device__ __forceinline__ void block_bcast_sum4(double& a, double& b, double& c, double& d) {
    __shared__ double red4[4][4];
    __shared__ double out4[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double s0 = wave_sum(a), s1 = wave_sum(b), s2 = wave_sum(c), s3 = wave_sum(d);
    if (lane == 0) {
        red4[0][w] = s0; red4[1][w] = s1; red4[2][w] = s2; red4[3][w] = s3;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        out4[k] = (red4[k][0] + red4[k][1]) + (red4[k][2] + red4[k][3]);
    }
    __syncthreads();
    a = out4[0]; b = out4[1]; c = out4[2]; d = out4[3];
}

// True-residual check is due when the loop stopped (converged or capped) and
// the check has not run yet.
__device__ __forceinline__ bool check_due(const DevScalars* sc) {
    return (sc->done == DONE_CONVERGED || sc->done == DONE_MAXITER) && !sc->checked;
}

}  // namespace ebe
