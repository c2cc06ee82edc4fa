// seasd_kernels.hip - gfx950 kernels of the Spectral Ewald mobility product.
//
// Pipeline for y = M x (one call):
//   bin      wrap centres into the cell, count spheres per bin (a bin is one
//            8^3 tile of the grid), scan, scatter, order each bin by input
//            index (deterministic), copy moments into binned order
//   pair     real-space pair sum over neighbour bins + self terms (FP64)
//   spread   tile-owner Gaussian spreading: one workgroup owns an 8^3 tile
//            and accumulates every sphere whose window touches it, so no
//            grid point is written by two workgroups (no atomics)
//   fft_x_fwd, fft_y_fwd, fft_z_scale (forward z, k-space multiply, inverse
//            z), fft_y_inv, fft_x_inv: 3-D transforms by line passes through LDS
//   gather   one wavefront per sphere reads its window of the velocity and
//            pressure grids, adds the pair/self part, writes y in input order
//
// Grid layouts (R = float or double):
//   real grid  [z][y][x] of R4 = 4 interleaved real fields
//              forward: (Hx, Hy, Hz, Hs)   inverse: (vx, vy, vz, p)
//   spectrum   [z][y][qx < M/2] of C4 = 4 interleaved complex fields. The
//              x transform of a real field is kept for qx in [0, M/2); the
//              qx = M/2 plane is the Nyquist plane, which the method zeroes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <stdint.h>

#include "seasd_math.h"
#include "seasd_internal.h"

namespace seasd {

template <typename R>
struct alignas(4 * sizeof(R)) R4 {
    R x, y, z, w;
};

template <typename R>
struct C1 {
    R re, im;
};

template <typename R>
__device__ inline C1<R> cmul(C1<R> a, C1<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// ---------------------------------------------------------------------------
// binning

// Bins are numbered along a Morton (Z-order) curve, so that spheres that are
// consecutive in binned order sit in compact 3-D blocks (cache locality for
// the pair sum, spreading and gather). nb is a power of two.
__host__ __device__ inline unsigned spread_bits3(unsigned v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline int bin_id(int bx, int by, int bz) {
    return (int)(spread_bits3((unsigned)bx) | (spread_bits3((unsigned)by) << 1) | (spread_bits3((unsigned)bz) << 2));
}
__host__ __device__ inline unsigned compact_bits3(unsigned v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x000003ffu;
    return v;
}

// Workgroups are handed to the 8 XCDs round-robin; renumber them so that each
// XCD runs one contiguous range of work items (its L2 then sees a compact
// region of the grid and of the sphere data).
__device__ inline int xcd_block(int b, int nblk) {
    const int per = nblk / 8, rem = nblk % 8;
    const int k = b % 8, idx = b / 8;
    return k * per + min(k, rem) + idx;
}

// fractional coordinates of a centre wrapped into [0, 1); the same expression
// gives the bin and the binned copy, so both always agree
__device__ inline void wrap_frac(const Cell& c, const double* p, double* t) {
    cell_frac(c, p[0], p[1], p[2], t);
    for (int d = 0; d < 3; ++d) {
        const double w = t[d] - floor(t[d]);
        t[d] = (w < 1.0 && w >= 0.0) ? w : 0.0;
    }
}

__device__ inline int bin_coord(double t, int nb) {
    const int k = (int)floor(t * nb);
    return k < 0 ? 0 : (k >= nb ? nb - 1 : k);
}

// clears the per-bin counters, the radius maximum and the list statistics
// of a new geometry in one launch
__global__ void k_zero_geometry(int nbins, int* __restrict__ counts, int* __restrict__ fill,
                                unsigned long long* __restrict__ amax_bits,
                                unsigned long long* __restrict__ nstats) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nbins) {
        counts[i] = 0;
        fill[i] = 0;
    }
    if (i == 0) {
        *amax_bits = 0ull;
        nstats[0] = 0ull;
        nstats[1] = 0ull;
    }
}

__global__ __launch_bounds__(256) void k_bin_count(int n, const double* __restrict__ pos, const double* __restrict__ rad,
                            Cell cell, int nb, int* __restrict__ bin_of,
                            int* __restrict__ counts, unsigned long long* __restrict__ amax_bits,
                            int* __restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0;   // radii are positive: 0 is neutral for the maximum
    if (i < n) {
        double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        a = rad[i];
        bool bad = !(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) && isfinite(a)) || !(a > 0.0);
        if (bad) {
            atomicOr(err, kErrNonfinite);
            p[0] = p[1] = p[2] = 0.0;
            a = 1.0;
        }
        double t[3];
        wrap_frac(cell, p, t);
        int bin = bin_id(bin_coord(t[0], nb), bin_coord(t[1], nb), bin_coord(t[2], nb));
        bin_of[i] = bin;
        atomicAdd(&counts[bin], 1);
    }
    // largest radius: one atomic per workgroup
    __shared__ double wmax[4];
    for (int off = 32; off > 0; off >>= 1) a = fmax(a, __shfl_xor(a, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        if (m > 0.0) atomicMax(amax_bits, (unsigned long long)__double_as_longlong(m));
    }
}

// Device-wide exclusive scan of int counts: each workgroup of 256 threads
// owns 2048 consecutive entries (coalesced loads through LDS); block sums are
// scanned by one workgroup and added back. out has n + 1 entries (total last).
constexpr int kScanItems = 8;
constexpr int kScanChunk = 256 * kScanItems;

__device__ inline int block_exclusive_scan(int v, int* sh, int& total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int u = (t >= o) ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += u;
        __syncthreads();
    }
    total = sh[255];
    const int incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(int n, const int* __restrict__ in, int* __restrict__ partial) {
    __shared__ int sh[256];
    const int base = blockIdx.x * kScanChunk;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
    int total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(int nb, int* __restrict__ partial) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    int s = 0;
    for (int b = b0; b < b1; ++b) s += partial[b];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = (t >= o) ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int b = b0; b < b1; ++b) {
        const int v = partial[b];
        partial[b] = run;
        run += v;
    }
    if (t == 1023) partial[nb] = part[t];
}

__global__ __launch_bounds__(256) void k_scan_apply(int n, const int* __restrict__ in, const int* __restrict__ partial,
                                                    int* __restrict__ out) {
    __shared__ int tile[kScanChunk];
    __shared__ int sh[256];
    const int base = blockIdx.x * kScanChunk;
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k * 256 + threadIdx.x;
        tile[k * 256 + threadIdx.x] = (i < n) ? in[i] : 0;
    }
    __syncthreads();
    int v[kScanItems], s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = tile[threadIdx.x * kScanItems + k];
        s += v[k];
    }
    int total;
    int run = block_exclusive_scan(s, sh, total) + partial[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        tile[threadIdx.x * kScanItems + k] = run;
        run += v[k];
    }
    __syncthreads();
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k * 256 + threadIdx.x;
        if (i < n) out[i] = tile[k * 256 + threadIdx.x];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = partial[gridDim.x];
}

static int launch_scan(int n, const int* in, int* out, int* partial, hipStream_t st) {
    const int nb = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(256), 0, st, n, in, partial);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, nb, partial);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, st, n, in, partial, out);
    return 0;
}

__global__ void k_bin_scatter(int n, const int* __restrict__ bin_of, const int* __restrict__ start,
                              int* __restrict__ fill, int* __restrict__ perm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = bin_of[i];
    perm[start[b] + atomicAdd(&fill[b], 1)] = i;
}

// order each bin by input index so that every later sum runs in a fixed order
__global__ void k_bin_order(int nbins, const int* __restrict__ start, int* __restrict__ perm) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    int s0 = start[b], s1 = start[b + 1];
    for (int i = s0 + 1; i < s1; ++i) {
        int v = perm[i], j = i - 1;
        while (j >= s0 && perm[j] > v) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

// binned copies: wrapped centres (fractional and Cartesian), radii and moments (FP64)
__device__ __forceinline__ void bin_gather_body(int n, const int* __restrict__ perm, const double* __restrict__ pos,
                                                const double* __restrict__ rad, const double* __restrict__ x,
                                                Cell cell, int compressible, double* __restrict__ sp, double* __restrict__ stf,
                                                double* __restrict__ sa, double* __restrict__ sx,
                                                int* __restrict__ err, int bid) {
    int s = bid * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
    double p[3];
    for (int d = 0; d < 3; ++d) {
        p[d] = pos[3 * i + d];
        if (!isfinite(p[d])) p[d] = 0.0;
    }
    double t[3], r[3];
    wrap_frac(cell, p, t);
    cell_cart(cell, t[0], t[1], t[2], r);
    for (int d = 0; d < 3; ++d) {
        stf[3 * s + d] = t[d];
        sp[3 * s + d] = r[d];
    }
    double a = rad[i];
    sa[s] = (isfinite(a) && a > 0.0) ? a : 1.0;
    bool bad = false;
    for (int c = 0; c < 12; ++c) {
        double v = x[12 * (size_t)i + c];
        if (!isfinite(v)) {
            bad = true;
            v = 0.0;
        }
        if (c == 11 && !compressible) v = 0.0;
        sx[12 * (size_t)s + c] = v;
    }
    if (bad) atomicOr(err, kErrNonfinite);
}

__global__ void k_bin_gather(int n, const int* __restrict__ perm, const double* __restrict__ pos,
                             const double* __restrict__ rad, const double* __restrict__ x,
                             Cell cell, int compressible, double* __restrict__ sp, double* __restrict__ stf,
                             double* __restrict__ sa, double* __restrict__ sx,
                             int* __restrict__ err) {
    bin_gather_body(n, perm, pos, rad, x, cell, compressible, sp, stf, sa, sx, err, blockIdx.x);
}

// ---------------------------------------------------------------------------
// real-space pair sum and self terms (FP64)
//
// Pass 1 counts, per sphere, the sources (sphere j and lattice image) within
// r_c = rc_factor (a_i + a_j); pass 2, after a scan, writes them as
// (j, image code) entries; pass 3 evaluates the couplings along each list, so
// no lane spends the heavy pair arithmetic on a candidate outside the cut-off.

// below this many spheres the neighbour list and the pair sum use one
// wavefront per sphere (one thread per sphere would leave most CUs idle);
// larger suspensions search with a wavefront per bin and sum with a thread
// per sphere (a wavefront per sphere when the lists are uneven)
constexpr int kWaveSpheres = 32768;

__device__ inline int floordiv(int c, int nb) { return (c >= 0) ? c / nb : -((-c + nb - 1) / nb); }

// Neighbour-bin geometry: the cell and, per lattice direction, the bins per
// unit length across its faces (nb / height). A source within r of a centre
// lies at most ceil(r nb / height_d) bins away along direction d.
struct NbrGeom {
    Cell cell;
    double rpl[3];
};

__device__ inline int image_code(int wx, int wy, int wz) { return ((wz + 512) << 20) | ((wy + 512) << 10) | (wx + 512); }
__device__ inline void image_of(int code, int& wx, int& wy, int& wz) {
    wx = (code & 1023) - 512;
    wy = ((code >> 10) & 1023) - 512;
    wz = ((code >> 20) & 1023) - 512;
}
// lattice translation wx a1 + wy a2 + wz a3
__device__ inline void image_shift(const Cell& c, int wx, int wy, int wz, double* o) {
    cell_cart(c, (double)wx, (double)wy, (double)wz, o);
}

// bin reach of cut-off r along each direction; flags (and clamps) a reach
// beyond about three cell lengths
__device__ inline void bin_reach(const NbrGeom& g, double r, int nb, int* reach, int* __restrict__ err, bool flag) {
    for (int d = 0; d < 3; ++d) {
        reach[d] = (int)ceil(r * g.rpl[d]);
        if (reach[d] > 3 * nb + 2) {
            if (flag) atomicOr(err, kErrCutoff);
            reach[d] = 3 * nb + 2;
        }
    }
}

// visit every (j, image) within the cut-off of binned sphere s, bins in the
// order x fastest, then y, then z; f(j, code) per hit
template <typename F>
__device__ inline void for_each_neighbour(int s, const double* __restrict__ sp, const double* __restrict__ stf,
                                          const double* __restrict__ sa, const int* __restrict__ start, int nb,
                                          const NbrGeom& g, double rc_factor, double amax, int checks,
                                          int* __restrict__ err, F&& f) {
    const double px = sp[3 * s], py = sp[3 * s + 1], pz = sp[3 * s + 2];
    const double ai = sa[s];
    int reach[3];
    bin_reach(g, rc_factor * (ai + amax), nb, reach, err, true);
    const int bx = bin_coord(stf[3 * s], nb), by = bin_coord(stf[3 * s + 1], nb), bz = bin_coord(stf[3 * s + 2], nb);
    for (int oz = -reach[2]; oz <= reach[2]; ++oz) {
        int cz = bz + oz;
        const int wz = floordiv(cz, nb);
        cz -= wz * nb;
        for (int oy = -reach[1]; oy <= reach[1]; ++oy) {
            int cy = by + oy;
            const int wy = floordiv(cy, nb);
            cy -= wy * nb;
            for (int ox = -reach[0]; ox <= reach[0]; ++ox) {
                int cx = bx + ox;
                const int wx = floordiv(cx, nb);
                cx -= wx * nb;
                const int bin = bin_id(cx, cy, cz);
                const int code = image_code(wx, wy, wz);
                double o[3];
                image_shift(g.cell, wx, wy, wz, o);
                for (int j = start[bin]; j < start[bin + 1]; ++j) {
                    if (j == s && wx == 0 && wy == 0 && wz == 0) continue;
                    const double dx = px - (sp[3 * j] + o[0]);
                    const double dy = py - (sp[3 * j + 1] + o[1]);
                    const double dz = pz - (sp[3 * j + 2] + o[2]);
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double aj = sa[j];
                    const double rc = rc_factor * (ai + aj);
                    if (r2 >= rc * rc) continue;
                    if (checks && r2 < (ai + aj) * (ai + aj) * (1.0 - 1e-12)) atomicOr(err, kErrOverlap);
                    f(j, code);
                }
            }
        }
    }
}

// The list with a group of G lanes per sphere (G = 64: a wavefront, for
// suspensions too small to fill the chip with one thread per sphere): lane l
// of the group takes bins l, l + G, ... of the neighbour bins in the visiting
// order of for_each_neighbour, counts its hits, a prefix sum over the group
// gives every lane its first slot and a second sweep over the lane's bin
// writes the entries, so the list comes out in the same order as the serial
// search. Every sphere lists into its own slot of `cap` entries and stores
// the full count; when the largest count exceeds cap the host grows cap and
// repeats the pass.
template <int G>
__global__ __launch_bounds__(256) void k_pair_fill_group(int n, const double* __restrict__ sp,
                                                        const double* __restrict__ stf,
                                                        const double* __restrict__ sa, const int* __restrict__ start,
                                                        int nb, NbrGeom g, double rc_factor,
                                                        const unsigned long long* __restrict__ amax_bits, int checks,
                                                        int cap, int* __restrict__ ncount,
                                                        int2* __restrict__ list, int* __restrict__ err) {
    const int lane = threadIdx.x & (G - 1);
    const int s = xcd_block(blockIdx.x, gridDim.x) * (256 / G) + threadIdx.x / G;
    if (s >= n) return;   // whole groups only; the kernel has no barrier
    const double amax = __longlong_as_double((long long)*amax_bits);
    const double px = sp[3 * s], py = sp[3 * s + 1], pz = sp[3 * s + 2];
    const double ai = sa[s];
    int reach[3];
    bin_reach(g, rc_factor * (ai + amax), nb, reach, err, lane == 0);
    const int sx = 2 * reach[0] + 1, sy = 2 * reach[1] + 1, sz = 2 * reach[2] + 1;
    const int nbins = sx * sy * sz;
    const int bx = bin_coord(stf[3 * s], nb), by = bin_coord(stf[3 * s + 1], nb), bz = bin_coord(stf[3 * s + 2], nb);
    int2* dst = list + (size_t)cap * s;
    int total = 0;
    for (int base = 0; base < nbins; base += G) {
        const int q = base + lane;
        int j0 = 0, j1 = 0, code = 0;
        double o[3] = {0.0, 0.0, 0.0};
        bool self_bin = false;
        if (q < nbins) {
            const int kx = q % sx - reach[0], ky = (q / sx) % sy - reach[1], kz = q / (sx * sy) - reach[2];
            int cx = bx + kx, cy = by + ky, cz = bz + kz;
            const int wx = floordiv(cx, nb), wy = floordiv(cy, nb), wz = floordiv(cz, nb);
            cx -= wx * nb;
            cy -= wy * nb;
            cz -= wz * nb;
            const int bin = bin_id(cx, cy, cz);
            j0 = start[bin];
            j1 = start[bin + 1];
            code = image_code(wx, wy, wz);
            image_shift(g.cell, wx, wy, wz, o);
            self_bin = wx == 0 && wy == 0 && wz == 0;
        }
        int cnt = 0;
        for (int j = j0; j < j1; ++j) {
            if (j == s && self_bin) continue;
            const double dx = px - (sp[3 * j] + o[0]), dy = py - (sp[3 * j + 1] + o[1]), dz = pz - (sp[3 * j + 2] + o[2]);
            const double r2 = dx * dx + dy * dy + dz * dz, aj = sa[j];
            const double rc = rc_factor * (ai + aj);
            if (r2 >= rc * rc) continue;
            if (checks && r2 < (ai + aj) * (ai + aj) * (1.0 - 1e-12)) atomicOr(err, kErrOverlap);
            ++cnt;
        }
        int incl = cnt;
        for (int off = 1; off < G; off <<= 1) {
            const int v = __shfl_up(incl, off, G);
            if (lane >= off) incl += v;
        }
        int k = total + incl - cnt;
        if (cnt > 0) {
            for (int j = j0; j < j1; ++j) {
                if (j == s && self_bin) continue;
                const double dx = px - (sp[3 * j] + o[0]), dy = py - (sp[3 * j + 1] + o[1]),
                             dz = pz - (sp[3 * j + 2] + o[2]);
                const double r2 = dx * dx + dy * dy + dz * dz, aj = sa[j];
                const double rc = rc_factor * (ai + aj);
                if (r2 >= rc * rc) continue;
                if (k < cap) dst[k] = make_int2(j, code);
                ++k;
            }
        }
        total += __shfl(incl, G - 1, G);
    }
    if (lane == 0) {
        ncount[s] = total;
    }
}

// The same lists with one wavefront per bin (large suspensions). The
// wavefront holds the spheres of its bin, 64 at a time, one per lane ("home"
// spheres), and walks the neighbour bins in the visiting order of
// for_each_neighbour, reach taken from the largest home radius: 64 bins at a
// time give their sphere ranges (one bin per lane) and a wavefront prefix sum;
// the candidates of those bins are listed in LDS in visiting order and taken
// into registers 64 kFillSlots at a time (slot r of lane l: candidate 64 r + l),
// then every home sphere is tested against them in order, a ballot giving
// each hit its slot. A bin beyond a sphere's own reach holds no sphere within
// its cut-off, so each list is exactly the one the serial search writes; the
// candidate loads are coalesced and shared by all spheres of the bin.
constexpr int kFillSlots = 4;   // candidate slots per lane and pass

__device__ inline int lanes_below(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}
// value of lane l (l uniform across the wavefront)
__device__ inline int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
// orders the LDS accesses of one wavefront before and after it
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void k_pair_fill_bin(int n, const double* __restrict__ sp,
                                                      const double* __restrict__ sa, const int* __restrict__ start,
                                                      int nb, NbrGeom g, double rc_factor,
                                                      const unsigned long long* __restrict__ amax_bits, int checks,
                                                      int cap, int* __restrict__ ncount,
                                                      int2* __restrict__ list, int* __restrict__ err) {
    constexpr int W = kFillSlots * 64;
    constexpr int kOwn = (512 << 20) | (512 << 10) | 512;   // image code of the unshifted sphere
    __shared__ int2 cand_lds[4][W];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int2* cl = cand_lds[wv];
    const int nbins = nb * nb * nb;
    const int b = xcd_block(blockIdx.x, gridDim.x) * 4 + wv;
    if (b >= nbins) return;   // whole wavefronts only; the kernel has no workgroup barrier
    const int h0 = start[b], h1 = start[b + 1];
    const double amax = __longlong_as_double((long long)*amax_bits);
    const int bx = (int)compact_bits3((unsigned)b), by = (int)compact_bits3((unsigned)b >> 1),
              bz = (int)compact_bits3((unsigned)b >> 2);
    for (int hb = h0; hb < h1; hb += 64) {
        const int nh = min(64, h1 - hb);
        double hx = 0.0, hy = 0.0, hz = 0.0, ha = 0.0;
        if (lane < nh) {
            hx = sp[3 * (hb + lane)];
            hy = sp[3 * (hb + lane) + 1];
            hz = sp[3 * (hb + lane) + 2];
            ha = sa[hb + lane];
        }
        double amx = 0.0;
        for (int h = 0; h < nh; ++h) amx = fmax(amx, lane_value(ha, h));
        int reach[3];
        bin_reach(g, rc_factor * (amx + amax), nb, reach, err, lane == 0);
        const int sx = 2 * reach[0] + 1, sy = 2 * reach[1] + 1, sz = 2 * reach[2] + 1;
        const int nnb = sx * sy * sz;
        int cnt = 0;   // lane h: entries of home sphere hb + h so far
        for (int q0 = 0; q0 < nnb; q0 += 64) {
            int j0 = 0, len = 0, code = 0;
            {   // lane u: neighbour bin q0 + u
                const int q = q0 + lane;
                if (q < nnb) {
                    int cx = bx + q % sx - reach[0], cy = by + (q / sx) % sy - reach[1],
                        cz = bz + q / (sx * sy) - reach[2];
                    const int wx = floordiv(cx, nb), wy = floordiv(cy, nb), wz = floordiv(cz, nb);
                    cx -= wx * nb;
                    cy -= wy * nb;
                    cz -= wz * nb;
                    const int bin = bin_id(cx, cy, cz);
                    j0 = start[bin];
                    len = start[bin + 1] - j0;
                    code = image_code(wx, wy, wz);
                }
            }
            int incl = len;
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            const int excl = incl - len;
            const int tot = lane_value(incl, 63);
            for (int w0 = 0; w0 < tot; w0 += W) {
                const int wlen = min(W, tot - w0);
                {   // list this window's candidates in LDS, in visiting order
                    const int lo = max(excl, w0), hi = min(excl + len, w0 + wlen);
                    for (int c = lo; c < hi; ++c) cl[c - w0] = make_int2(j0 + (c - excl), code);
                }
                wave_sync();
                double cx[kFillSlots], cy[kFillSlots], cz[kFillSlots], ca[kFillSlots];
                int cj[kFillSlots], cc[kFillSlots];
#pragma unroll
                for (int r = 0; r < kFillSlots; ++r) {
                    const int c = 64 * r + lane;
                    cj[r] = -1;
                    cc[r] = 0;
                    cx[r] = cy[r] = cz[r] = ca[r] = 0.0;
                    if (c < wlen) {
                        const int2 e = cl[c];
                        int wx, wy, wz;
                        image_of(e.y, wx, wy, wz);
                        double o[3];
                        image_shift(g.cell, wx, wy, wz, o);
                        cj[r] = e.x;
                        cc[r] = e.y;
                        cx[r] = sp[3 * e.x] + o[0];
                        cy[r] = sp[3 * e.x + 1] + o[1];
                        cz[r] = sp[3 * e.x + 2] + o[2];
                        ca[r] = sa[e.x];
                    }
                }
                wave_sync();   // the LDS list is read before the next window overwrites it
                const int nslots = (wlen + 63) / 64;
                for (int h = 0; h < nh; ++h) {
                    const double px = lane_value(hx, h), py = lane_value(hy, h), pz = lane_value(hz, h);
                    const double ai = lane_value(ha, h);
                    const int sh = hb + h;
                    int base = lane_value(cnt, h);
#pragma unroll
                    for (int r = 0; r < kFillSlots; ++r) {
                        if (r >= nslots) break;
                        bool hit = false;
                        if (cj[r] >= 0 && !(cj[r] == sh && cc[r] == kOwn)) {
                            const double dx = px - cx[r], dy = py - cy[r], dz = pz - cz[r];
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            const double rc = rc_factor * (ai + ca[r]);
                            hit = r2 < rc * rc;
                            if (hit && checks && r2 < (ai + ca[r]) * (ai + ca[r]) * (1.0 - 1e-12))
                                atomicOr(err, kErrOverlap);
                        }
                        const unsigned long long m = __ballot(hit);
                        const int k = base + lanes_below(m);
                        if (hit && k < cap) list[(size_t)cap * sh + k] = make_int2(cj[r], cc[r]);
                        base += __popcll(m);
                    }
                    if (lane == h) cnt = base;
                }
            }
        }
        if (lane < nh) ncount[hb + lane] = cnt;
    }
}

// Largest and total list length (one atomic pair per workgroup, at most 64
// workgroups; the statistics are cleared with the geometry): the host reads
// them with the overflow check to choose how the pair sum spreads the lists
// over lanes.
constexpr int kStatsBlocks = 64;

__global__ __launch_bounds__(256) void k_count_stats(int n, const int* __restrict__ ncount,
                                                    unsigned long long* __restrict__ stats) {
    __shared__ unsigned long long ssum[256];
    __shared__ int smax[256];
    unsigned long long sum = 0;
    int mx = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const int c = ncount[i];
        sum += (unsigned long long)c;
        mx = max(mx, c);
    }
    ssum[threadIdx.x] = sum;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            ssum[threadIdx.x] += ssum[threadIdx.x + o];
            smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&stats[0], (unsigned long long)smax[0]);
        atomicAdd(&stats[1], ssum[0]);
    }
}

__device__ __forceinline__ void pair_eval_body(int n, const double* __restrict__ sp,
                                               const double* __restrict__ sa, const double* __restrict__ sx,
                                               const int* __restrict__ ncount, int cap, const int2* __restrict__ list,
                                               Cell cell, double xi, double inv_eta, int parts,
                                               double* __restrict__ ybuf, int bid) {
    const int s = bid * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double px = sp[3 * s], py = sp[3 * s + 1], pz = sp[3 * s + 2];
    const double ai = sa[s];
    double y[12];
    for (int c = 0; c < 12; ++c) y[c] = 0.0;
    if (parts & kPartsReal) {
        const int k0 = cap * s, k1 = k0 + min(ncount[s], cap);
        for (int k = k0; k < k1; ++k) {
            const int2 e = list[k];
            const int j = e.x;
            int wx, wy, wz;
            image_of(e.y, wx, wy, wz);
            double o[3];
            image_shift(cell, wx, wy, wz, o);
            const double dx = px - (sp[3 * j] + o[0]);
            const double dy = py - (sp[3 * j + 1] + o[1]);
            const double dz = pz - (sp[3 * j + 2] + o[2]);
            double xj[12];
            for (int c = 0; c < 12; ++c) xj[c] = sx[12 * (size_t)j + c];
            pair_coupling<double>(dx, dy, dz, ai, sa[j], xi, inv_eta, xj, y);
        }
    }
    if (parts & kPartsSelf) {
        double d4[4];
        self_diag<double>(ai, xi, 1.0 / inv_eta, d4);
        const double* xs = sx + 12 * (size_t)s;
        for (int c = 0; c < 3; ++c) y[c] += d4[0] * xs[c];
        for (int c = 3; c < 6; ++c) y[c] += d4[1] * xs[c];
        for (int c = 6; c < 11; ++c) y[c] += d4[2] * xs[c];
        y[11] += d4[3] * xs[11];
    }
    for (int c = 0; c < 12; ++c) ybuf[12 * (size_t)s + c] = y[c];
}

__global__ __launch_bounds__(128) void k_pair_eval(int n, const double* __restrict__ sp,
                                                   const double* __restrict__ sa, const double* __restrict__ sx,
                                                   const int* __restrict__ ncount, int cap, const int2* __restrict__ list,
                                                   Cell cell, double xi, double inv_eta, int parts,
                                                   double* __restrict__ ybuf) {
    pair_eval_body(n, sp, sa, sx, ncount, cap, list, cell, xi, inv_eta, parts, ybuf,
                   xcd_block(blockIdx.x, gridDim.x));
}

// Pair sum with a group of G lanes per sphere: lane l of the group evaluates
// list entries l, l + G, ..., and the 12 partial sums are reduced across the
// group in a fixed butterfly order. G = 64 (a wavefront) serves suspensions
// too small to fill the chip with one thread per sphere; for large ones a few
// lanes per sphere read runs of consecutive neighbours together, which cuts
// the cache lines each load instruction touches.
template <int G>
__device__ __forceinline__ void pair_eval_group_body(int n, const double* __restrict__ sp,
                                                     const double* __restrict__ sa,
                                                     const double* __restrict__ sx,
                                                     const int* __restrict__ ncount, int cap,
                                                     const int2* __restrict__ list, Cell cell, double xi,
                                                     double inv_eta, int parts, double* __restrict__ ybuf, int bid) {
    const int lane = threadIdx.x & (G - 1);
    const int s = bid * (256 / G) + threadIdx.x / G;
    if (s >= n) return;   // whole groups only; the kernel has no barrier
    const double px = sp[3 * s], py = sp[3 * s + 1], pz = sp[3 * s + 2];
    const double ai = sa[s];
    double y[12];
    for (int c = 0; c < 12; ++c) y[c] = 0.0;
    if (parts & kPartsReal) {
        const int k0 = cap * s, k1 = k0 + min(ncount[s], cap);
        for (int k = k0 + lane; k < k1; k += G) {
            const int2 e = list[k];
            const int j = e.x;
            int wx, wy, wz;
            image_of(e.y, wx, wy, wz);
            double o[3];
            image_shift(cell, wx, wy, wz, o);
            const double dx = px - (sp[3 * j] + o[0]);
            const double dy = py - (sp[3 * j + 1] + o[1]);
            const double dz = pz - (sp[3 * j + 2] + o[2]);
            double xj[12];
            for (int c = 0; c < 12; ++c) xj[c] = sx[12 * (size_t)j + c];
            pair_coupling<double>(dx, dy, dz, ai, sa[j], xi, inv_eta, xj, y);
        }
        for (int off = G / 2; off > 0; off >>= 1)
            for (int c = 0; c < 12; ++c) y[c] += __shfl_xor(y[c], off, G);
    }
    if (lane != 0) return;
    if (parts & kPartsSelf) {
        double d4[4];
        self_diag<double>(ai, xi, 1.0 / inv_eta, d4);
        const double* xs = sx + 12 * (size_t)s;
        for (int c = 0; c < 3; ++c) y[c] += d4[0] * xs[c];
        for (int c = 3; c < 6; ++c) y[c] += d4[1] * xs[c];
        for (int c = 6; c < 11; ++c) y[c] += d4[2] * xs[c];
        y[11] += d4[3] * xs[11];
    }
    for (int c = 0; c < 12; ++c) ybuf[12 * (size_t)s + c] = y[c];
}

template <int G>
__global__ __launch_bounds__(256) void k_pair_eval_group(int n, const double* __restrict__ sp,
                                                         const double* __restrict__ sa,
                                                         const double* __restrict__ sx,
                                                         const int* __restrict__ ncount, int cap,
                                                         const int2* __restrict__ list, Cell cell, double xi,
                                                         double inv_eta, int parts, double* __restrict__ ybuf) {
    pair_eval_group_body<G>(n, sp, sa, sx, ncount, cap, list, cell, xi, inv_eta, parts, ybuf,
                            xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// neighbour graph of the learned preconditioner: directed edges s -> j between
// binned spheres closer than cut (a_s + a_j), rows in binned order, each row
// in the (deterministic) visiting order of for_each_neighbour

__global__ __launch_bounds__(256) void k_edge_count(int n, const double* __restrict__ sp, const double* __restrict__ stf,
                                                    const double* __restrict__ sa, const int* __restrict__ start,
                                                    int nb, NbrGeom g, double cut,
                                                    const unsigned long long* __restrict__ amax_bits,
                                                    int* __restrict__ deg, int* __restrict__ err) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double amax = __longlong_as_double((long long)*amax_bits);
    int k = 0;
    for_each_neighbour(s, sp, stf, sa, start, nb, g, cut, amax, 0, err, [&](int, int) { ++k; });
    deg[s] = k;
}

__global__ __launch_bounds__(256) void k_edge_fill(int n, const double* __restrict__ sp, const double* __restrict__ stf,
                                                   const double* __restrict__ sa, const int* __restrict__ start,
                                                   int nb, NbrGeom g, double cut,
                                                   const unsigned long long* __restrict__ amax_bits,
                                                   const int* __restrict__ rowptr, int* __restrict__ esrc,
                                                   int* __restrict__ edst, float4* __restrict__ geo,
                                                   float* __restrict__ fe, int* __restrict__ err) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double amax = __longlong_as_double((long long)*amax_bits);
    const double px = sp[3 * s], py = sp[3 * s + 1], pz = sp[3 * s + 2], ai = sa[s];
    int e = rowptr[s];
    const int e1 = rowptr[s + 1];
    for_each_neighbour(s, sp, stf, sa, start, nb, g, cut, amax, 0, err, [&](int j, int code) {
        if (e >= e1) return;   // the count pass bounds the row
        int wx, wy, wz;
        image_of(code, wx, wy, wz);
        double o[3];
        image_shift(g.cell, wx, wy, wz, o);
        const double dx = sp[3 * j] + o[0] - px, dy = sp[3 * j + 1] + o[1] - py, dz = sp[3 * j + 2] + o[2] - pz;
        const double r = sqrt(dx * dx + dy * dy + dz * dz), aj = sa[j];
        const double rho = r / (ai + aj);
        esrc[e] = s;
        edst[e] = j;
        geo[e] = make_float4((float)(dx / r), (float)(dy / r), (float)(dz / r), (float)r);
        float* f = fe + 16 * (size_t)e;
        f[0] = (float)rho;
        f[1] = (float)(1.0 / rho);
        f[2] = (float)(1.0 / (rho * rho * rho));
        f[3] = (float)log(aj / ai);
        f[4] = (float)(aj / (ai + aj));
        for (int k = 5; k < 16; ++k) f[k] = 0.f;
        ++e;
    });
}

// reverse edge (j -> s) of every edge s -> j, and the node features
__global__ __launch_bounds__(256) void k_edge_rev(int n, const double* __restrict__ sa, const int* __restrict__ rowptr,
                                                  const int* __restrict__ edst, const float4* __restrict__ geo,
                                                  int* __restrict__ erev, float* __restrict__ fn,
                                                  int* __restrict__ err) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int e0 = rowptr[s], e1 = rowptr[s + 1];
    const double ai = sa[s];
    double sr3 = 0.0, sl3 = 0.0, slog = 0.0;
    for (int e = e0; e < e1; ++e) {
        const int j = edst[e];
        int rev = -1;
        for (int q = rowptr[j]; q < rowptr[j + 1]; ++q)
            if (edst[q] == s) {
                rev = q;
                break;
            }
        if (rev < 0) atomicOr(err, kErrCutoff);
        erev[e] = rev < 0 ? e : rev;
        const double aj = sa[j], rho = (double)geo[e].w / (ai + aj), lam = aj / ai;
        sr3 += 1.0 / (rho * rho * rho);
        sl3 += lam * lam * lam;
        slog += log(lam);
    }
    const int deg = e1 - e0;
    float* f = fn + 16 * (size_t)s;
    f[0] = (float)(deg / 16.0);
    f[1] = (float)(sr3 / 16.0);
    f[2] = (float)(log1p(sl3) / 4.0);
    f[3] = (float)(deg > 0 ? slog / deg : 0.0);
    for (int k = 4; k < 16; ++k) f[k] = 0.f;
}

// ---------------------------------------------------------------------------
// window records
//
// The window is the Gaussian h = C exp(-beta |u|^2) of eq. shape, with u the
// offset from the sphere centre in grid units of the fractional grid (the
// cell's M^3 grid points t = k/M), beta = 2 m^2/P^2 from eq. theta-param
// (h falls to exp(-m^2/2) at |u| = P/2). It is evaluated on P points per
// dimension: for even P the points floor(u) - P/2 + 1 .. floor(u) + P/2, for
// odd P the points round(u) -+ (P - 1)/2, so that the window is centred on
// the sphere either way (the printed range [-P/2, P/2] of eq. fgg-exp holds
// P + 1 points when P is even). One record per sphere (binned order) holds
// i0, the offset delta = i0 - u, the 1-D factors exp(-beta (delta + k)^2),
// the moments and the Faxen constants of the sphere (WinGeom); spreading and
// gather both read it. The factors use fast Gaussian gridding (eq. fgg-exp),
// anchored at the window centre so the recurrences run over at most P/2
// steps, in FP64.

constexpr int kMaxP = 32;
// record layout (R units): [0..2] i0 (int bits), [3] d1, [4..6] delta, [7] a^2,
// [8..10] F, [11..13] T, [14..19] S (xx yy zz xy xz yz), [20] sqrt3 s6,
// [21] c0, [22] c1, [23] e0, [24 ..] factors x[P], y[P], z[P].
static_assert(kRecHead == 24, "record header layout above");

// first of the P window points of a centre at grid coordinate u
__host__ __device__ inline int first_window_point(double u, int P) {
    return (P & 1) ? (int)floor(u + 0.5) - (P - 1) / 2 : (int)floor(u) - P / 2 + 1;
}

template <typename O>
__device__ inline void fgg_factors(double d0, double h, double alpha, int P, O* out) {
    const int kc = (P - 1) / 2;   // d0 + kc h in (-h, 0] (even P) or [-h/2, h/2) (odd P)
    const double dc = d0 + kc * h;
    const double e0 = exp(-alpha * dc * dc);
    const double up = exp(-2.0 * alpha * dc * h);  // exp(-2 alpha dc h)^j
    const double q = exp(-alpha * h * h);          // exp(-alpha h^2)^(j^2)
    const double q2 = q * q;
    double v = e0, stp = up * q;
    out[kc] = (O)e0;
    for (int k = kc + 1; k < P; ++k) {
        v *= stp;
        stp *= q2;
        out[k] = (O)v;
    }
    v = e0;
    stp = q / up;
    for (int k = kc - 1; k >= 0; --k) {
        v *= stp;
        stp *= q2;
        out[k] = (O)v;
    }
}

template <typename R>
__device__ inline int rec_i0(const R* rec, int d) {
    if constexpr (sizeof(R) == 4) return __float_as_int(rec[d]);
    else return (int)__double_as_longlong(rec[d]);
}

// One workgroup builds the records of 64 consecutive spheres in LDS (four
// threads per sphere: the header, and the anchor, offset and factors of one
// dimension each) and writes them out as one contiguous block, so every
// record line is written whole.
constexpr int kWinSpheres = 64;

template <typename R>
__device__ __forceinline__ void window_body(int n, const double* __restrict__ stf, const double* __restrict__ sa,
                                            const double* __restrict__ sx, int P, int M, double beta, double bq,
                                            double bz, R* __restrict__ rec_out, int bid) {
    __shared__ __attribute__((aligned(16))) R buf[kWinSpheres * ((kRecHead + 3 * kMaxP + 3) & ~3)];
    const int RS = rec_stride(P);
    const int s0 = bid * kWinSpheres;
    const int ns = min(kWinSpheres, n - s0);
    const int t = threadIdx.x;
    const int q = t >> 2, piece = t & 3;
    if (q < ns) {
        const int s = s0 + q;
        R* rec = buf + q * RS;
        if (piece > 0) {
            const int d = piece - 1;
            const double u = stf[3 * s + d] * M;   // exact: M is a power of two
            const int i0 = first_window_point(u, P);
            const double delta = i0 - u;
            if constexpr (sizeof(R) == 4) rec[d] = __int_as_float(i0);
            else rec[d] = __longlong_as_double((long long)i0);
            rec[4 + d] = (R)delta;
            fgg_factors(delta, 1.0, beta, P, rec + kRecHead + d * P);   // straight into the LDS record
        } else {
            const double a = sa[s];
            const double a2 = a * a;
            const double* xs = sx + 12 * (size_t)s;
            rec[3] = (R)(0.8 * a2);
            rec[7] = (R)a2;
            rec[21] = (R)(1.0 - a2 * bq / 3.0);
            rec[22] = (R)(2.0 / 3.0 * a2);
            rec[23] = (R)(2.0 - 0.4 * a2 * bq - 0.8 * a2 * bz);
            for (int d = 0; d < 3; ++d) {
                rec[8 + d] = (R)xs[d];
                rec[11 + d] = (R)xs[3 + d];
            }
            double S[6];
            s5_to_sym<double>(xs + 6, S);
            for (int d = 0; d < 6; ++d) rec[14 + d] = (R)S[d];
            rec[20] = (R)(kSqrt3 * xs[11]);
            for (int k = kRecHead + 3 * P; k < RS; ++k) rec[k] = R(0);   // padding
        }
    }
    __syncthreads();
    // records are multiples of 16 bytes and the block starts on a record
    using V = typename std::conditional<sizeof(R) == 4, float4, double2>::type;
    constexpr int PV = 16 / sizeof(R);
    const V* src = reinterpret_cast<const V*>(buf);
    V* dst = reinterpret_cast<V*>(rec_out + (size_t)s0 * RS);
    for (int e = t; e < ns * RS / PV; e += 256) dst[e] = src[e];
}

template <typename R>
__global__ __launch_bounds__(256) void k_window(int n, const double* __restrict__ stf, const double* __restrict__ sa,
                                                const double* __restrict__ sx, int P, int M, double beta, double bq,
                                                double bz, R* __restrict__ rec_out) {
    window_body<R>(n, stf, sa, sx, P, M, beta, bq, bz, rec_out, blockIdx.x);
}

// ---------------------------------------------------------------------------
// spreading: one workgroup of 256 threads owns one 8^3 tile. The spheres that
// can reach the tile are listed once in LDS and their records staged 16 at a
// time. Lane l of every wavefront owns the tile's (x, y) column l and its 8
// z-points; the wavefronts take different spheres (w, w + 4, ...), so a
// sphere costs one wavefront pass: its column coefficients once per lane,
// then 13 multiply-adds per z-point inside its window. The four wavefronts'
// partial tiles are summed in FP64 at the end, and each grid point is written
// by exactly one thread, with no atomics.

// spheres staged per round
constexpr int kStage = 16;
constexpr int kMaxCand = 2048; // candidate list held in LDS

template <typename R>
__device__ inline void neumaier(R& acc, R& cmp, R v) {
    const R sum = acc + v;
    cmp += (fabs(acc) >= fabs(v)) ? ((acc - sum) + v) : ((v - sum) + acc);
    acc = sum;
}

// wavefronts per workgroup of an 8^3 tile (each lane owns 8 / kSpreadWaves points)
constexpr int kSpreadWaves = 4;
constexpr int kTile = 8;   // spreading tile = bin edge in grid points

// gradient-vector coefficients of the window on the fractional grid (WinGeom)
struct SpreadGeom {
    double Gxx, Gyx, Gyy, Gzz;   // g = (Gxx u_x, Gyx u_x + Gyy u_y, Gzz u_z)
    double Qxx, Qxy, Qyy;        // x-y part of the sheared-cell stresslet term
    double cw;                   // window weight (spreading C, gather C V / M^3)
};

template <typename R, bool SHEAR>
__device__ __forceinline__ void spread_body(
    int n, const R* __restrict__ recs, const int* __restrict__ start, int nb, int M, int P, SpreadGeom sg,
    R4<R>* __restrict__ grid, int bid) {
    constexpr int TILE = kTile;
    constexpr int NW = kSpreadWaves;        // wavefronts
    constexpr int NT = 64 * NW;             // threads per workgroup
    static_assert(TILE * TILE == 64, "a lane owns one (x, y) column of the tile");
    constexpr int MAXB = 125;               // (2 reach + 1)^3 for reach <= 2 (P <= 32)
    constexpr int STAGE = kStage;
    constexpr int MAXC = kMaxCand;
    // staged records and their z bases; the closing cross-wavefront sum
    // reuses the same bytes
    constexpr int kStBytes = STAGE * (kRecHead + 3 * kMaxP) * (int)sizeof(R);
    constexpr int kZbBytes = STAGE * kMaxP * (int)sizeof(R4<R>);
    constexpr int kRedBytes = NW * 2 * 64 * (int)sizeof(R4<R>);   // two z-planes at a time
    constexpr int kSmem = (kStBytes + kZbBytes) > kRedBytes ? (kStBytes + kZbBytes) : kRedBytes;
    static_assert(kStBytes % 16 == 0, "z bases start on 16 bytes");
    __shared__ __attribute__((aligned(16))) unsigned char smem[kSmem];
    R* st = reinterpret_cast<R*>(smem);
    R4<R>* zb = reinterpret_cast<R4<R>*>(smem + kStBytes);   // [STAGE][kMaxP]: f_z g_z^k, k = 0..3
    R4<R>* red = reinterpret_cast<R4<R>*>(smem);             // [NW][2][64]
    __shared__ int cand[MAXC];
    __shared__ int bins[MAXB], pre[MAXB + 1];
    __shared__ int nbins_used;
    const int t = threadIdx.x;
    // the wavefront index is uniform: kept in a scalar register, the sphere
    // loop below and its z-plane tests run on the scalar unit
    const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const unsigned tcode = (unsigned)bid;   // Morton code of the tile
    const int tx = (int)compact_bits3(tcode), ty = (int)compact_bits3(tcode >> 1), tz = (int)compact_bits3(tcode >> 2);
    const int gx = tx * TILE + (lane & 7), gy = ty * TILE + (lane >> 3), gz0 = tz * TILE;
    const int mask = M - 1;
    const int RS = rec_stride(P);

    // a window reaches ceil(P/2) points above and ceil(P/2) - 1 below the
    // grid point at or below its centre
    const int reach = ((P + 1) / 2 + TILE - 1) / TILE;
    const int span = min(2 * reach + 1, nb);
    // neighbour bins and their sizes in parallel, then one running sum in LDS
    const int nused = span * span * span;
    for (int k = t; k < nused; k += NT) {
        const int kx = k % span, ky = (k / span) % span, kz = k / (span * span);
        const int bx = (span == nb) ? kx : ((tx - reach + kx) % nb + nb) % nb;
        const int by = (span == nb) ? ky : ((ty - reach + ky) % nb + nb) % nb;
        const int bz = (span == nb) ? kz : ((tz - reach + kz) % nb + nb) % nb;
        const int b = bin_id(bx, by, bz);
        bins[k] = b;
        pre[k + 1] = start[b + 1] - start[b];
    }
    __syncthreads();
    if (t == 0) {
        nbins_used = nused;
        int run = 0;
        pre[0] = 0;
        for (int k = 1; k <= nused; ++k) {
            run += pre[k];
            pre[k] = run;
        }
    }
    __syncthreads();
    const int ncand = pre[nbins_used];
    const R Gxx = (R)sg.Gxx, Gyx = (R)sg.Gyx, Gyy = (R)sg.Gyy, Gzz = (R)sg.Gzz, cwr = (R)sg.cw;
    const R Qxx = (R)sg.Qxx, Qxy = (R)sg.Qxy, Qyy = (R)sg.Qyy;
    // this wavefront's sums over its spheres at the 8 points of the lane's column
    R part[TILE][4];
#pragma unroll
    for (int p = 0; p < TILE; ++p)
        for (int c = 0; c < 4; ++c) part[p][c] = R(0);

    for (int cbase = 0; cbase < ncand; cbase += MAXC) {
        const int clen = min(MAXC, ncand - cbase);
        for (int k = t; k < nbins_used; k += NT) {
            const int b0 = max(pre[k], cbase), b1 = min(pre[k + 1], cbase + clen);
            const int s0 = start[bins[k]] + (b0 - pre[k]);
            for (int c = b0; c < b1; ++c) cand[c - cbase] = s0 + (c - b0);
        }
        __syncthreads();
        for (int c0 = 0; c0 < clen; c0 += STAGE) {
            const int cnt = min(STAGE, clen - c0);
            {   // records are multiples of 16 bytes: copy them in 16-byte pieces
                constexpr int V = 16 / sizeof(R);
                const int RV = RS / V;
                using V4 = typename std::conditional<sizeof(R) == 4, float4, double2>::type;
                V4* stv = reinterpret_cast<V4*>(st);
                const V4* rv = reinterpret_cast<const V4*>(recs);
                for (int e = t; e < cnt * RV; e += NT) {
                    const int q = e / RV, k = e - q * RV;
                    stv[q * RV + k] = rv[(size_t)RV * cand[c0 + q] + k];
                }
            }
            __syncthreads();
            for (int e = t; e < cnt * P; e += NT) {
                const int q = e / P, kz = e - q * P;
                const R* rc = st + q * RS;
                const R fz = rc[kRecHead + 2 * P + kz];
                const R g = Gzz * (rc[6] + (R)kz);
                zb[q * kMaxP + kz] = R4<R>{fz, fz * g, fz * g * g, fz * g * g * g};
            }
            __syncthreads();
            // wavefront wv takes staged spheres wv, wv + 4, ...
            for (int q = wv; q < cnt; q += NW) {
                const R* rc = static_cast<const R*>(__builtin_assume_aligned(st + q * RS, 16));
                const int i0x = rec_i0(rc, 0), i0y = rec_i0(rc, 1), i0z = rec_i0(rc, 2);
                // window index of the tile's first z-plane (the same in every lane)
                const int kz0 = __builtin_amdgcn_readfirstlane((gz0 - i0z) & mask);
                bool anyz = false;
#pragma unroll
                for (int p = 0; p < TILE; ++p) anyz = anyz || (((kz0 + p) & mask) < P);
                if (!anyz) continue;
                const int kx = (gx - i0x) & mask, ky = (gy - i0y) & mask;
                const bool inxy = (kx < P) && (ky < P);
                if (!__any(inxy)) continue;
                if (!inxy) continue;
                // The window is f_x f_y f_z and the Faxen polynomials are
                // cubic in g_z = Gzz u_z, so the column's contribution at
                // window z-index kz is sum_k C_k f_z g_z^k per component.
                const R F0 = rc[8], F1 = rc[9], F2 = rc[10], T0 = rc[11], T1 = rc[12], T2 = rc[13];
                const R S0 = rc[14], S1 = rc[15], S2 = rc[16], S3 = rc[17], S4 = rc[18], S5 = rc[19];
                const R sq = rc[20], c0 = rc[21], c1 = rc[22], e0 = rc[23], d1 = rc[3];
                const R* fa = rc + kRecHead;
                const R ux = rc[4] + (R)kx, uy = rc[5] + (R)ky;
                const R gX = Gxx * ux, gY = Gyx * ux + Gyy * uy;
                const R wxy = cwr * fa[kx] * fa[P + ky];
                const R gxy2 = gX * gX + gY * gY;
                const R a0 = c0 + c1 * gxy2, b0 = e0 + d1 * gxy2;
                const R Sx = S0 * gX + S3 * gY, Sy = S3 * gX + S1 * gY, Sz = S4 * gX + S5 * gY;
                const R tzz = gX * T1 - gY * T0;
                R u0 = F0 * a0 - gY * T2 + b0 * Sx, u1 = F1 * a0 + gX * T2 + b0 * Sy, u2 = F2 * a0 - tzz + b0 * Sz;
                if constexpr (SHEAR) {   // S . (-(4/5) a^2 Qt g_xy)
                    const R ex = -d1 * (Qxx * gX + Qxy * gY), ey = -d1 * (Qxy * gX + Qyy * gY);
                    u0 += S0 * ex + S3 * ey;
                    u1 += S3 * ex + S1 * ey;
                    u2 += S4 * ex + S5 * ey;
                }
                const R C0 = wxy * u0, C1 = wxy * (T1 + b0 * S4);
                const R C2 = wxy * (F0 * c1 + d1 * Sx), C3 = wxy * (d1 * S4);
                const R C4 = wxy * u1, C5 = wxy * (b0 * S5 - T0);
                const R C6 = wxy * (F1 * c1 + d1 * Sy), C7 = wxy * (d1 * S5);
                const R C8 = wxy * u2, C9 = wxy * (b0 * S2);
                const R C10 = wxy * (F2 * c1 + d1 * Sz), C11 = wxy * (d1 * S2);
                const R C12 = wxy * sq;
                const R4<R>* zq = zb + q * kMaxP;
#pragma unroll
                for (int p = 0; p < TILE; ++p) {
                    const int kz = (kz0 + p) & mask;
                    if (kz >= P) continue;   // the same in every lane
                    const R4<R> z = zq[kz];
                    // one fused multiply-add per term, straight into the sums
                    part[p][0] = fma(C3, z.w, fma(C2, z.z, fma(C1, z.y, fma(C0, z.x, part[p][0]))));
                    part[p][1] = fma(C7, z.w, fma(C6, z.z, fma(C5, z.y, fma(C4, z.x, part[p][1]))));
                    part[p][2] = fma(C11, z.w, fma(C10, z.z, fma(C9, z.y, fma(C8, z.x, part[p][2]))));
                    part[p][3] = fma(C12, z.x, part[p][3]);
                }
            }
            __syncthreads();   // the next stage overwrites the records
        }
    }
    // Sum of the four wavefronts' partial sums in FP64, in a fixed order, two
    // z-planes at a time: each grid point is written once, with no atomics.
#pragma unroll
    for (int p0 = 0; p0 < TILE; p0 += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
            red[(wv * 2 + h) * 64 + lane] = R4<R>{part[p0 + h][0], part[p0 + h][1], part[p0 + h][2], part[p0 + h][3]};
        __syncthreads();
        if (t < 128) {
            const int h = t >> 6, l = t & 63;
            double ox = 0.0, oy = 0.0, oz = 0.0, ow = 0.0;
            for (int w = 0; w < NW; ++w) {
                const R4<R> v = red[(w * 2 + h) * 64 + l];
                ox += (double)v.x;
                oy += (double)v.y;
                oz += (double)v.z;
                ow += (double)v.w;
            }
            const int x = tx * TILE + (l & 7), y = ty * TILE + (l >> 3), z = gz0 + p0 + h;
            grid[((size_t)z * M + y) * M + x] = R4<R>{(R)ox, (R)oy, (R)oz, (R)ow};
        }
        __syncthreads();
    }
}

template <typename R, bool SHEAR>
__global__ __launch_bounds__(64 * kSpreadWaves) void k_spread(
    int n, const R* __restrict__ recs, const int* __restrict__ start, int nb, int M, int P, SpreadGeom sg,
    R4<R>* __restrict__ grid) {
    spread_body<R, SHEAR>(n, recs, start, nb, M, P, sg, grid, xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// FFT building block: Stockham autosort transform over `nlines` lines of
// length M held in LDS (line-major), ping-ponging between a and b: one
// radix-2 stage when log2 M is odd, then radix-4 stages. tw[j] =
// exp(sgn 2 pi i j/M), j < M. Returns the buffer that holds the result.

template <typename R>
__device__ inline C1<R> cadd(C1<R> a, C1<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ inline C1<R> csub(C1<R> a, C1<R> b) { return {a.re - b.re, a.im - b.im}; }
// multiply by sgn*i
template <typename R>
__device__ inline C1<R> cmuli(C1<R> a, int sgn) { return sgn > 0 ? C1<R>{-a.im, a.re} : C1<R>{a.im, -a.re}; }

template <typename R, int M>
__device__ inline C1<R>* lds_fft(C1<R>* a, C1<R>* b, int nlines, const C1<R>* tw, int sgn) {
    constexpr int LOG = (M <= 1) ? 0 : 31 - __builtin_clz(M);
    int p = 1;
    if (LOG & 1) {  // radix-2 stage
        constexpr int H = M / 2;
        for (int e = threadIdx.x; e < nlines * H; e += blockDim.x) {
            const int line = e / H, j = e - line * H;
            const C1<R> x0 = a[line * M + j];
            const C1<R> x1 = a[line * M + j + H];
            C1<R>* o = b + line * M + 2 * j;
            o[0] = cadd(x0, x1);
            o[1] = csub(x0, x1);
        }
        __syncthreads();
        C1<R>* tmp = a; a = b; b = tmp;
        p = 2;
    }
    constexpr int Q = M / 4;
    for (; p < M; p <<= 2) {
        const int tstride = M / (4 * p);
        for (int e = threadIdx.x; e < nlines * Q; e += blockDim.x) {
            const int line = e / Q, j = e - line * Q;
            const int k = j & (p - 1);
            const C1<R>* in = a + line * M + j;
            const C1<R> x0 = in[0];
            const C1<R> x1 = cmul(tw[(k * tstride) & (M - 1)], in[Q]);
            const C1<R> x2 = cmul(tw[(2 * k * tstride) & (M - 1)], in[2 * Q]);
            const C1<R> x3 = cmul(tw[(3 * k * tstride) & (M - 1)], in[3 * Q]);
            const C1<R> s02 = cadd(x0, x2), d02 = csub(x0, x2);
            const C1<R> s13 = cadd(x1, x3), d13 = cmuli(csub(x1, x3), sgn);
            C1<R>* o = b + line * M + 4 * (j - k) + k;
            o[0] = cadd(s02, s13);
            o[p] = cadd(d02, d13);
            o[2 * p] = csub(s02, s13);
            o[3 * p] = csub(d02, d13);
        }
        __syncthreads();
        C1<R>* tmp = a; a = b; b = tmp;
    }
    return a;
}

template <typename R, int M>
__device__ inline void load_twiddles(C1<R>* tw, const double* __restrict__ twg, int sgn) {
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        tw[j].re = (R)twg[2 * j];
        tw[j].im = (R)(sgn * twg[2 * j + 1]);
    }
}

template <typename T, typename R>
__device__ inline C1<T> up(C1<R> a) { return C1<T>{(T)a.re, (T)a.im}; }

// x pass, forward, real -> half spectrum. Two real fields share one complex
// transform (A = f0 + i f1), separated with A(-q) = conj of the partner.
template <typename R, int M, int LPB>
__device__ __forceinline__ void fft_x_fwd_body(const R4<R>* __restrict__ in, C1<R>* __restrict__ out,
                                               const double* __restrict__ twg, int bid) {
    using T = R;
    __shared__ C1<T> buf[2][2 * LPB * M];
    __shared__ C1<T> tw[M];
    load_twiddles<T, M>(tw, twg, +1);
    const size_t line0 = (size_t)bid * LPB;
    for (int e = threadIdx.x; e < LPB * M; e += blockDim.x) {
        const int l = e / M, x = e - l * M;
        const R4<R> v = in[(line0 + l) * M + x];
        buf[0][(2 * l) * M + x] = {(T)v.x, (T)v.y};
        buf[0][(2 * l + 1) * M + x] = {(T)v.z, (T)v.w};
    }
    __syncthreads();
    C1<T>* r = lds_fft<T, M>(buf[0], buf[1], 2 * LPB, tw, +1);
    for (int e = threadIdx.x; e < LPB * (M / 2); e += blockDim.x) {
        const int l = e / (M / 2), q = e - l * (M / 2);
        const int qn = (M - q) & (M - 1);
        C1<R> o[4];
        for (int g = 0; g < 2; ++g) {
            const C1<T> A = r[(2 * l + g) * M + q];
            const C1<T> B = r[(2 * l + g) * M + qn];  // A(-q)
            // f0 = (A(q) + conj A(-q))/2,  f1 = -i (A(q) - conj A(-q))/2
            o[2 * g] = {(R)(T(0.5) * (A.re + B.re)), (R)(T(0.5) * (A.im - B.im))};
            o[2 * g + 1] = {(R)(T(0.5) * (A.im + B.im)), (R)(T(-0.5) * (A.re - B.re))};
        }
        C1<R>* dst = out + ((line0 + l) * (M / 2) + q) * 4;
        for (int c = 0; c < 4; ++c) dst[c] = o[c];
    }
}

template <typename R, int M, int LPB>
__global__ __launch_bounds__(256) void k_fft_x_fwd(const R4<R>* __restrict__ in, C1<R>* __restrict__ out,
                                                   const double* __restrict__ twg) {
    fft_x_fwd_body<R, M, LPB>(in, out, twg, blockIdx.x);
}

// x pass, inverse, half spectrum -> real. The qx = M/2 plane is zero.
template <typename R, int M, int LPB>
__device__ __forceinline__ void fft_x_inv_body(const C1<R>* __restrict__ in, R4<R>* __restrict__ out,
                                               const double* __restrict__ twg, int bid) {
    using T = R;
    __shared__ C1<T> buf[2][2 * LPB * M];
    __shared__ C1<T> tw[M];
    load_twiddles<T, M>(tw, twg, -1);
    const size_t line0 = (size_t)bid * LPB;
    // thread (l, q) reads the four spectra at q once and fills x = q and M - q:
    // G0 + i G1 at q, conj G0 + i conj G1 at M - q, zero at the Nyquist plane
    for (int e = threadIdx.x; e < LPB * (M / 2); e += blockDim.x) {
        const int l = e / (M / 2), q = e - l * (M / 2);
        const C1<R>* sp = in + ((line0 + l) * (M / 2) + q) * 4;
        C1<R> S[4];
        for (int c = 0; c < 4; ++c) S[c] = sp[c];
        for (int g = 0; g < 2; ++g) {
            const C1<R> a = S[2 * g], b = S[2 * g + 1];
            C1<T>* ln = buf[0] + (2 * l + g) * M;
            if (q == 0) {
                ln[0] = {(T)a.re, (T)b.re};
                ln[M / 2] = {T(0), T(0)};
            } else {
                ln[q] = {(T)a.re - (T)b.im, (T)a.im + (T)b.re};
                ln[M - q] = {(T)a.re + (T)b.im, (T)b.re - (T)a.im};
            }
        }
    }
    __syncthreads();
    C1<T>* r = lds_fft<T, M>(buf[0], buf[1], 2 * LPB, tw, -1);
    for (int e = threadIdx.x; e < LPB * M; e += blockDim.x) {
        const int l = e / M, x = e - l * M;
        const C1<T> A = r[(2 * l) * M + x], B = r[(2 * l + 1) * M + x];
        out[(line0 + l) * M + x] = {(R)A.re, (R)A.im, (R)B.re, (R)B.im};
    }
}

template <typename R, int M, int LPB>
__global__ __launch_bounds__(256) void k_fft_x_inv(const C1<R>* __restrict__ in, R4<R>* __restrict__ out,
                                                   const double* __restrict__ twg) {
    fft_x_inv_body<R, M, LPB>(in, out, twg, blockIdx.x);
}

// y pass (either direction) on the half spectrum: a block owns W columns of
// qx at one z; 4 fields per element -> 4W lines of length M.
template <typename R, int M, int W>
__device__ __forceinline__ void fft_y_body(C1<R>* __restrict__ data, const double* __restrict__ twg,
                                           int sgn, int bid) {
    using T = R;
    __shared__ C1<T> buf[2][4 * W * M];
    __shared__ C1<T> tw[M];
    load_twiddles<T, M>(tw, twg, sgn);
    constexpr int HX = M / 2;
    const int x0 = (bid % (HX / W)) * W;
    const int z = bid / (HX / W);
    for (int e = threadIdx.x; e < W * M * 4; e += blockDim.x) {
        const int c = e & 3, w = (e >> 2) % W, y = (e >> 2) / W;
        buf[0][(w * 4 + c) * M + y] = up<T>(data[(((size_t)z * M + y) * HX + x0 + w) * 4 + c]);
    }
    __syncthreads();
    C1<T>* r = lds_fft<T, M>(buf[0], buf[1], 4 * W, tw, sgn);
    for (int e = threadIdx.x; e < W * M * 4; e += blockDim.x) {
        const int c = e & 3, w = (e >> 2) % W, y = (e >> 2) / W;
        const C1<T> v = r[(w * 4 + c) * M + y];
        data[(((size_t)z * M + y) * HX + x0 + w) * 4 + c] = C1<R>{(R)v.re, (R)v.im};
    }
}

template <typename R, int M, int W>
__global__ __launch_bounds__(256) void k_fft_y(C1<R>* __restrict__ data, const double* __restrict__ twg,
                                               int sgn) {
    fft_y_body<R, M, W>(data, twg, sgn, blockIdx.x);
}

// ---------------------------------------------------------------------------
// 256-point lines as 16 x 16 (four-step): each line is owned by 16 threads;
// thread t holds x[16 n1 + t], n1 = 0..15, transforms over n1 in registers,
// applies the twiddle w^(t k1), exchanges through LDS once and transforms
// over the other index. One LDS buffer (padded rows of 17, lines of 273) and
// 16 complex lines per workgroup in FP32, 8 in FP64 (Fft16Lines), so a
// workgroup reads whole 128-byte rows.

template <typename R>
struct Fft16Lines {
    static constexpr int value = sizeof(R) == 4 ? 16 : 8;
};

// 4-point DFT in place, exponent sign sgn: Y_k = sum_n a_n (sgn i)^(n k)
template <typename T>
__device__ inline void dft4(C1<T>& a0, C1<T>& a1, C1<T>& a2, C1<T>& a3, int sgn) {
    const C1<T> s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const C1<T> s13 = cadd(a1, a3), d13 = cmuli(csub(a1, a3), sgn);
    a0 = cadd(s02, s13);
    a1 = cadd(d02, d13);
    a2 = csub(s02, s13);
    a3 = csub(d02, d13);
}

// 16-point DFT in registers (4 x 4); tw is the table of wM^j (same sign)
// for lines of M points, so w16^j = tw[(M / 16) j]. On return X_k sits in
// v[4 (k % 4) + k / 4].
template <typename T, int M = 256>
__device__ inline void dft16(C1<T>* v, const C1<T>* tw, int sgn) {
#pragma unroll
    for (int m2 = 0; m2 < 4; ++m2) dft4(v[m2], v[4 + m2], v[8 + m2], v[12 + m2], sgn);
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
        for (int m2 = 1; m2 < 4; ++m2)
            v[4 * k1 + m2] = cmul(tw[((M / 16) * m2 * k1) & (M - 1)], v[4 * k1 + m2]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3], sgn);
}

constexpr int kL16Row = 17;               // padded row of the 16 x 16 exchange
constexpr int kL16Line = 16 * 17 + 1;     // padded line (273 complex)

// v[n1] = x[16 n1 + t] of one line in, X[16 k2 + t] = v[4 (k2 % 4) + k2 / 4] out
template <typename T>
__device__ inline void fft256_line(C1<T>* v, C1<T>* ln, const C1<T>* tw, int t, int sgn) {
    dft16(v, tw, sgn);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1)
        ln[k1 * kL16Row + t] = cmul(tw[(t * k1) & 255], v[4 * (k1 & 3) + (k1 >> 2)]);
    __syncthreads();
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) v[n2] = ln[t * kL16Row + n2];
    dft16(v, tw, sgn);
}

// y pass for M = 256: a workgroup owns LN / 4 qx columns at one z, LN lines
// (columns x 4 fields), 16 threads per line.
template <typename R>
__global__ __launch_bounds__(256) void k_fft_y256(C1<R>* __restrict__ data, const double* __restrict__ twg,
                                                  int sgn) {
    constexpr int M = 256, HX = 128, LN = Fft16Lines<R>::value, W = LN / 4;
    __shared__ C1<R> buf[LN * kL16Line];
    __shared__ C1<R> tw[M];
    load_twiddles<R, M>(tw, twg, sgn);
    const int l = threadIdx.x % LN, t = threadIdx.x / LN;   // consecutive lanes: consecutive lines
    // The forward pass takes the z-planes from last to first: the x pass has
    // just written them first to last, and the planes it wrote last are the
    // ones still in the memory-side cache (the spectrum is slightly larger
    // than that cache; measured 95 -> 83 us at FP32).
    const int bq = sgn > 0 ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
    const int x0 = (bq % (HX / W)) * W;
    const int z = bq / (HX / W);
    C1<R>* base = data + ((size_t)z * M * HX + x0) * 4 + l;   // + (y HX) * 4
    C1<R> v[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = base[(size_t)(16 * n1 + t) * HX * 4];
    __syncthreads();   // twiddles
    fft256_line(v, buf + l * kL16Line, tw, t, sgn);
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) base[(size_t)(16 * k2 + t) * HX * 4] = v[4 * (k2 & 3) + (k2 >> 2)];
}

// x pass, forward, M = 256: LN / 2 real lines per workgroup (8 in FP32, 4 in
// FP64), each a pair of complex transforms (x + i y fields, z + i w fields),
// then the same half-spectrum unpacking as k_fft_x_fwd.
template <typename R>
__global__ __launch_bounds__(256) void k_fft_x_fwd256(const R4<R>* __restrict__ in, C1<R>* __restrict__ out,
                                                      const double* __restrict__ twg) {
    constexpr int M = 256, LN = Fft16Lines<R>::value, RL = LN / 2;
    __shared__ C1<R> buf[LN * kL16Line];
    __shared__ C1<R> tw[M];
    load_twiddles<R, M>(tw, twg, +1);
    const int l16 = threadIdx.x >> 4, t = threadIdx.x & 15;   // complex line, thread in line
    const int line = l16 >> 1, g = l16 & 1;
    const size_t line0 = (size_t)blockIdx.x * RL;
    // the lanes of fields (x, y) and (z, w) of one line sit side by side in a
    // wavefront, so each load instruction covers whole 256-byte rows once
    const C1<R>* src = reinterpret_cast<const C1<R>*>(in) + ((line0 + line) * M + t) * 2 + g;
    C1<R> v[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = src[32 * n1];
    __syncthreads();   // twiddles
    C1<R>* ln = buf + l16 * kL16Line;
    fft256_line(v, ln, tw, t, +1);
    // Half-spectrum unpacking in registers: the thread holds X[16 k2 + t] in
    // v[4 (k2 % 4) + k2 / 4]; X[M - q] of q = 16 k2 + t (t > 0) sits in lane
    // 16 - t of the same line at k2' = 15 - k2, and for t = 0 in the thread
    // itself at k2' = (16 - k2) mod 16.
    const int pl = (int)(threadIdx.x & 63 & ~15) | ((16 - t) & 15);   // partner lane
    C1<R>* dst = out + (line0 + line) * (M / 2) * 4 + 2 * g;
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const int q = 16 * k2 + t;
        const C1<R> A = v[4 * (k2 & 3) + (k2 >> 2)];
        const int kp = 15 - k2, k0 = (16 - k2) & 15;
        const C1<R> Bp = v[4 * (kp & 3) + (kp >> 2)];
        const C1<R> Bs = {__shfl(Bp.re, pl), __shfl(Bp.im, pl)};
        const C1<R> B = t == 0 ? v[4 * (k0 & 3) + (k0 >> 2)] : Bs;
        dst[4 * q] = {R(0.5) * (A.re + B.re), R(0.5) * (A.im - B.im)};
        dst[4 * q + 1] = {R(0.5) * (A.im + B.im), R(-0.5) * (A.re - B.re)};
    }
}

// x pass, inverse, M = 256: half spectrum -> LN / 2 real lines per workgroup
template <typename R>
__global__ __launch_bounds__(256) void k_fft_x_inv256(const C1<R>* __restrict__ in, R4<R>* __restrict__ out,
                                                      const double* __restrict__ twg) {
    constexpr int M = 256, LN = Fft16Lines<R>::value, RL = LN / 2;
    __shared__ C1<R> buf[LN * kL16Line];
    __shared__ C1<R> tw[M];
    load_twiddles<R, M>(tw, twg, -1);
    // lines last to first: the inverse y pass wrote the planes first to last,
    // so this pass starts on the ones still in the memory-side cache (101 ->
    // 99 us at FP32)
    const size_t line0 = (size_t)(gridDim.x - 1 - blockIdx.x) * RL;
    const int l16 = threadIdx.x >> 4, t = threadIdx.x & 15;   // complex line, thread in line
    const int line = l16 >> 1, g = l16 & 1;
    // complex line g of real line `line` packs fields 2g (real part) and
    // 2g + 1 (imaginary part): its element x comes from the two half spectra
    // at q = x (x < M/2) or at q = M - x (conjugated); x = M/2 is zero. The
    // two spectra sit side by side, one 16-byte load per element.
    const R4<R>* sp = reinterpret_cast<const R4<R>*>(in + (line0 + line) * (M / 2) * 4) + g;
    C1<R> v[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
        const int x = 16 * n1 + t;
        const int q = n1 < 8 ? x : (x == M / 2 ? 0 : M - x);
        const R4<R> ab = sp[2 * q];
        if (n1 < 8) {
            v[n1] = x == 0 ? C1<R>{ab.x, ab.z} : C1<R>{ab.x - ab.w, ab.y + ab.z};
        } else {
            v[n1] = x == M / 2 ? C1<R>{R(0), R(0)} : C1<R>{ab.x + ab.w, ab.z - ab.y};
        }
    }
    C1<R>* ln = buf + l16 * kL16Line;
    __syncthreads();   // twiddles
    fft256_line(v, ln, tw, t, -1);
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) ln[16 * k2 + t] = v[4 * (k2 & 3) + (k2 >> 2)];
    __syncthreads();
    for (int e = threadIdx.x; e < RL * M; e += 16 * LN) {
        const int l = e >> 8, x = e & 255;
        const C1<R> A = buf[(2 * l) * kL16Line + x], B = buf[(2 * l + 1) * kL16Line + x];
        out[(line0 + l) * M + x] = {A.re, A.im, B.re, B.im};
    }
}

// k-space multiply (eq. wave-result): k = B q with B = 2 pi A^-T (for the
// supported cells kx = bxx qx, ky = byx qx + byy qy, kz = bzz qz), the
// deconvolution of the two windows exp(kdeconv |q|^2) with q the integer
// wave vector (the fractional-grid Gaussian of eq. shape), the screened
// Stokes and Laplace kernels and the grid normalisation.
struct KScale {
    double bxx, byx, byy, bzz;
    double inv4xi2;        // 1 / (4 xi^2)
    double kdeconv;        // 2 pi^2 / (beta M^2)
    double norm;           // 1/M^3 : grid-sum normalisation of forward x inverse
    double inv_eta;
};

__device__ inline double kscale_factor(const KScale& ks, int qx, int qy, int qz, double& kx, double& ky,
                                       double& kz, double& k2) {
    kx = ks.bxx * qx;
    ky = ks.byx * qx + ks.byy * qy;
    kz = ks.bzz * qz;
    k2 = kx * kx + ky * ky + kz * kz;
    const double q2 = (double)qx * qx + (double)qy * qy + (double)qz * qz;
    return exp(ks.kdeconv * q2 - k2 * ks.inv4xi2) * ks.norm / k2;
}

// z pass: forward z transform, k-space multiply (eq. wave-result with the
// periodic Stokes propagator, the source flow and the pressure), inverse z
// transform. A block owns W columns of qx at one qy.
template <typename R, int M, int W>
__device__ __forceinline__ void fft_z_scale_body(C1<R>* __restrict__ data,
                                                 const double* __restrict__ twg, KScale ks, int bid) {
    using T = R;
    __shared__ C1<T> buf[2][4 * W * M];
    __shared__ C1<T> twf[M], twi[M];
    load_twiddles<T, M>(twf, twg, +1);
    load_twiddles<T, M>(twi, twg, -1);
    constexpr int HX = M / 2;
    const int x0 = (bid % (HX / W)) * W;
    const int y = bid / (HX / W);
    const size_t zstride = (size_t)M * HX * 4;
    for (int e = threadIdx.x; e < W * M * 4; e += blockDim.x) {
        const int c = e & 3, w = (e >> 2) % W, z = (e >> 2) / W;
        buf[0][(w * 4 + c) * M + z] = up<T>(data[z * zstride + ((size_t)y * HX + x0 + w) * 4 + c]);
    }
    __syncthreads();
    C1<T>* a = lds_fft<T, M>(buf[0], buf[1], 4 * W, twf, +1);
    C1<T>* b = (a == buf[0]) ? buf[1] : buf[0];
    const int qy = (y < M / 2) ? y : y - M;
    for (int e = threadIdx.x; e < W * M; e += blockDim.x) {
        const int w = e % W, z = e / W;
        const int qx = x0 + w;
        const int qz = (z < M / 2) ? z : z - M;
        C1<T>* f0 = a + (w * 4 + 0) * M + z;
        C1<T>* f1 = a + (w * 4 + 1) * M + z;
        C1<T>* f2 = a + (w * 4 + 2) * M + z;
        C1<T>* f3 = a + (w * 4 + 3) * M + z;
        const bool zero = (qx == 0 && qy == 0 && qz == 0) || (y == M / 2) || (z == M / 2);
        if (zero) {
            *f0 = *f1 = *f2 = *f3 = {T(0), T(0)};
            continue;
        }
        double kx, ky, kz, k2;
        const double ex = kscale_factor(ks, qx, qy, qz, kx, ky, kz, k2);
        const T st = (T)(ks.inv_eta * (1.0 + k2 * ks.inv4xi2) * ex);   // Stokes, incl. 1/k^2
        const T lp = (T)ex;                                              // Laplace 1/k^2
        const T rkx = (T)kx, rky = (T)ky, rkz = (T)kz, ik2 = (T)(1.0 / k2);
        const C1<T> h0 = *f0, h1 = *f1, h2 = *f2, h3 = *f3;
        // k.f and the transverse projection
        const C1<T> kf = {rkx * h0.re + rky * h1.re + rkz * h2.re, rkx * h0.im + rky * h1.im + rkz * h2.im};
        const C1<T> pk = {kf.re * ik2, kf.im * ik2};
        const T sq = T(0.25) * (T)ks.inv_eta * lp;   // source flow (i k)/(4 eta k^2)
        // v = st (f - k (k.f)/k^2) + sq i k h3 ; i k h3 = k (-h3.im, h3.re)
        *f0 = {st * (h0.re - rkx * pk.re) - sq * rkx * h3.im, st * (h0.im - rkx * pk.im) + sq * rkx * h3.re};
        *f1 = {st * (h1.re - rky * pk.re) - sq * rky * h3.im, st * (h1.im - rky * pk.im) + sq * rky * h3.re};
        *f2 = {st * (h2.re - rkz * pk.re) - sq * rkz * h3.im, st * (h2.im - rkz * pk.im) + sq * rkz * h3.re};
        // p = i (k.f) / k^2
        *f3 = {-lp * kf.im, lp * kf.re};
    }
    __syncthreads();
    C1<T>* r = lds_fft<T, M>(a, b, 4 * W, twi, -1);
    for (int e = threadIdx.x; e < W * M * 4; e += blockDim.x) {
        const int c = e & 3, w = (e >> 2) % W, z = (e >> 2) / W;
        const C1<T> v = r[(w * 4 + c) * M + z];
        data[z * zstride + ((size_t)y * HX + x0 + w) * 4 + c] = C1<R>{(R)v.re, (R)v.im};
    }
}

template <typename R, int M, int W>
__global__ __launch_bounds__(256) void k_fft_z_scale(C1<R>* __restrict__ data,
                                                     const double* __restrict__ twg, KScale ks) {
    fft_z_scale_body<R, M, W>(data, twg, ks, blockIdx.x);
}

// z pass of the hybrid size approach (Sec. 3.2): as k_fft_z_scale, and in
// addition the velocity spectrum times -|k|^2/6 (the Faxen Laplacian of the
// read-out, lap/6, taken in k space: G'' of eq. wave-only-compute-2 with the
// grid-space H of eq. grid-space) into the second spectrum as (Lvx, Lvy,
// Lvz, 0). LDS lines are field-major (line c W + w for field c of column w):
// the forward transform runs over the 4 W input lines, the inverse over all
// 8 W lines.
template <typename R, int M, int W>
__global__ __launch_bounds__(256) void k_fft_z_scale_hyb(C1<R>* __restrict__ data, C1<R>* __restrict__ data2,
                                                         const double* __restrict__ twg, KScale ks) {
    using T = R;
    __shared__ C1<T> buf[2][8 * W * M];
    __shared__ C1<T> twf[M], twi[M];
    load_twiddles<T, M>(twf, twg, +1);
    load_twiddles<T, M>(twi, twg, -1);
    constexpr int HX = M / 2;
    const int x0 = (blockIdx.x % (HX / W)) * W;
    const int y = blockIdx.x / (HX / W);
    const size_t zstride = (size_t)M * HX * 4;
    for (int e = threadIdx.x; e < W * M * 4; e += blockDim.x) {
        const int c = e & 3, w = (e >> 2) % W, z = (e >> 2) / W;
        buf[0][(c * W + w) * M + z] = data[z * zstride + ((size_t)y * HX + x0 + w) * 4 + c];
    }
    __syncthreads();
    C1<T>* a = lds_fft<T, M>(buf[0], buf[1], 4 * W, twf, +1);
    C1<T>* b = (a == buf[0]) ? buf[1] : buf[0];
    const int qy = (y < M / 2) ? y : y - M;
    for (int e = threadIdx.x; e < W * M; e += blockDim.x) {
        const int w = e % W, z = e / W;
        const int qx = x0 + w;
        const int qz = (z < M / 2) ? z : z - M;
        C1<T>* f[8];
        for (int c = 0; c < 8; ++c) f[c] = a + (c * W + w) * M + z;
        const bool zero = (qx == 0 && qy == 0 && qz == 0) || (y == M / 2) || (z == M / 2);
        if (zero) {
            for (int c = 0; c < 8; ++c) *f[c] = {T(0), T(0)};
            continue;
        }
        double kx, ky, kz, k2;
        const double ex = kscale_factor(ks, qx, qy, qz, kx, ky, kz, k2);
        const T st = (T)(ks.inv_eta * (1.0 + k2 * ks.inv4xi2) * ex);
        const T lp = (T)ex;
        const T rkx = (T)kx, rky = (T)ky, rkz = (T)kz, ik2 = (T)(1.0 / k2);
        const T lap6 = (T)(-k2 / 6.0);
        const C1<T> h0 = *f[0], h1 = *f[1], h2 = *f[2], h3 = *f[3];
        const C1<T> kf = {rkx * h0.re + rky * h1.re + rkz * h2.re, rkx * h0.im + rky * h1.im + rkz * h2.im};
        const C1<T> pk = {kf.re * ik2, kf.im * ik2};
        const T sq = T(0.25) * (T)ks.inv_eta * lp;
        const C1<T> v0 = {st * (h0.re - rkx * pk.re) - sq * rkx * h3.im, st * (h0.im - rkx * pk.im) + sq * rkx * h3.re};
        const C1<T> v1 = {st * (h1.re - rky * pk.re) - sq * rky * h3.im, st * (h1.im - rky * pk.im) + sq * rky * h3.re};
        const C1<T> v2 = {st * (h2.re - rkz * pk.re) - sq * rkz * h3.im, st * (h2.im - rkz * pk.im) + sq * rkz * h3.re};
        *f[0] = v0;
        *f[1] = v1;
        *f[2] = v2;
        *f[3] = {-lp * kf.im, lp * kf.re};
        *f[4] = {lap6 * v0.re, lap6 * v0.im};
        *f[5] = {lap6 * v1.re, lap6 * v1.im};
        *f[6] = {lap6 * v2.re, lap6 * v2.im};
        *f[7] = {T(0), T(0)};
    }
    __syncthreads();
    C1<T>* r = lds_fft<T, M>(a, b, 8 * W, twi, -1);
    for (int e = threadIdx.x; e < W * M * 8; e += blockDim.x) {
        const int c = e & 7, w = (e >> 3) % W, z = (e >> 3) / W;
        const C1<T> v = r[(c * W + w) * M + z];
        C1<R>* dst = c < 4 ? data : data2;
        dst[z * zstride + ((size_t)y * HX + x0 + w) * 4 + (c & 3)] = v;
    }
}

// z pass for M = 256 (FP32 storage): forward z transform, k-space multiply
// (as in k_fft_z_scale), inverse z transform; a workgroup owns 4 qx columns
// at one qy.
template <typename R>
__global__ __launch_bounds__(256) void k_fft_z256(C1<R>* __restrict__ data, const double* __restrict__ twg,
                                                  KScale ks) {
    constexpr int M = 256, HX = 128, LN = Fft16Lines<R>::value, W = LN / 4;
    __shared__ C1<R> buf[LN * kL16Line];
    __shared__ C1<R> twf[M], twi[M];
    load_twiddles<R, M>(twf, twg, +1);
    load_twiddles<R, M>(twi, twg, -1);
    const int l = threadIdx.x % LN, t = threadIdx.x / LN;
    const int x0 = (blockIdx.x % (HX / W)) * W;
    const int y = blockIdx.x / (HX / W);
    const size_t zstride = (size_t)M * HX * 4;
    C1<R>* base = data + ((size_t)y * HX + x0) * 4 + l;   // + z zstride
    C1<R>* ln = buf + l * kL16Line;
    C1<R> v[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = base[(size_t)(16 * n1 + t) * zstride];
    __syncthreads();   // twiddles
    fft256_line(v, ln, twf, t, +1);
    __syncthreads();   // every thread has read its exchange row
    // spectrum of this line in natural order: element qz at ln[qz]
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) ln[16 * k2 + t] = v[4 * (k2 & 3) + (k2 >> 2)];
    __syncthreads();
    const int qy = (y < M / 2) ? y : y - M;
    for (int e = threadIdx.x; e < W * M; e += 16 * LN) {
        const int w = e % W, z = e / W;
        const int qx = x0 + w;
        const int qz = (z < M / 2) ? z : z - M;
        C1<R>* f0 = buf + (w * 4 + 0) * kL16Line + z;
        C1<R>* f1 = buf + (w * 4 + 1) * kL16Line + z;
        C1<R>* f2 = buf + (w * 4 + 2) * kL16Line + z;
        C1<R>* f3 = buf + (w * 4 + 3) * kL16Line + z;
        const bool zero = (qx == 0 && qy == 0 && qz == 0) || (y == M / 2) || (z == M / 2);
        if (zero) {
            *f0 = *f1 = *f2 = *f3 = {R(0), R(0)};
            continue;
        }
        double kx, ky, kz, k2;
        const double ex = kscale_factor(ks, qx, qy, qz, kx, ky, kz, k2);
        const R st = (R)(ks.inv_eta * (1.0 + k2 * ks.inv4xi2) * ex);
        const R lp = (R)ex;
        const R rkx = (R)kx, rky = (R)ky, rkz = (R)kz, ik2 = (R)(1.0 / k2);
        const C1<R> h0 = *f0, h1 = *f1, h2 = *f2, h3 = *f3;
        const C1<R> kf = {rkx * h0.re + rky * h1.re + rkz * h2.re, rkx * h0.im + rky * h1.im + rkz * h2.im};
        const C1<R> pk = {kf.re * ik2, kf.im * ik2};
        const R sq = R(0.25) * (R)ks.inv_eta * lp;
        *f0 = {st * (h0.re - rkx * pk.re) - sq * rkx * h3.im, st * (h0.im - rkx * pk.im) + sq * rkx * h3.re};
        *f1 = {st * (h1.re - rky * pk.re) - sq * rky * h3.im, st * (h1.im - rky * pk.im) + sq * rky * h3.re};
        *f2 = {st * (h2.re - rkz * pk.re) - sq * rkz * h3.im, st * (h2.im - rkz * pk.im) + sq * rkz * h3.re};
        *f3 = {-lp * kf.im, lp * kf.re};
    }
    __syncthreads();
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = ln[16 * n1 + t];
    __syncthreads();   // the exchange below reuses the line
    fft256_line(v, ln, twi, t, -1);
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) base[(size_t)(16 * k2 + t) * zstride] = v[4 * (k2 & 3) + (k2 >> 2)];
}

// ---------------------------------------------------------------------------
// 128- and 64-point lines as four-step transforms, FP32 storage: 8 threads
// own a line and thread t holds x[8 n1 + t], n1 = 0..M/8 - 1.
//   M = 128 (16 x 8): a 16-point DFT over n1 in registers, w^(t k1), one LDS
//     exchange, then the rows k1 = t and t + 8 as 8-point DFTs over the
//     former thread index: X[k1 + 16 k2] = sum_t w^(16 t k2) w^(t k1)
//     sum_n1 x[8 n1 + t] w^(8 n1 k1).
//   M = 64 (8 x 8): the same with an 8-point DFT over n1 and one row per
//     thread: X[t + 8 k2].
// 32 lines per workgroup, so the y and z passes read whole 256-byte rows.

constexpr int kL8Row = 9;   // padded row of the exchange (8 entries)

template <int M>
struct Fft8Line {
    static constexpr int NV = M / 8;                    // values per thread
    static constexpr int LINE = NV * kL8Row + 1;        // padded line in LDS
    // position along the line of the thread's j-th output value
    __device__ static int out(int t, int j) { return M == 128 ? t + (j >> 3) * 8 + 16 * (j & 7) : t + 8 * j; }
};

// 8-point DFT of v[0..7] in place (two 4-point DFTs and w8^k = tw[(M/8) k])
template <typename T, int M>
__device__ inline void dft8(C1<T>* v, const C1<T>* tw, int sgn) {
    dft4(v[0], v[2], v[4], v[6], sgn);
    dft4(v[1], v[3], v[5], v[7], sgn);
    C1<T> o[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const C1<T> b = k == 0 ? v[1] : cmul(tw[(M / 8) * k], v[2 * k + 1]);
        o[k] = cadd(v[2 * k], b);
        o[k + 4] = csub(v[2 * k], b);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = o[k];
}

// v[n1] = x[8 n1 + t] of one line in; X[Fft8Line<M>::out(t, j)] = v[j] out.
// Every thread of the workgroup calls it (one barrier inside).
template <typename T, int M>
__device__ inline void fft8_line(C1<T>* v, C1<T>* ln, const C1<T>* tw, int t, int sgn) {
    static_assert(M == 64 || M == 128, "lines of 64 or 128 points");
    constexpr int NV = M / 8;
    if constexpr (M == 128) dft16<T, 128>(v, tw, sgn);
    else dft8<T, 64>(v, tw, sgn);
#pragma unroll
    for (int k1 = 0; k1 < NV; ++k1) {
        // the k1-th output of the first DFT
        const int src = M == 128 ? 4 * (k1 & 3) + (k1 >> 2) : k1;
        ln[k1 * kL8Row + t] = cmul(tw[(t * k1) & (M - 1)], v[src]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NV / 8; ++r)
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) v[8 * r + n2] = ln[(t + 8 * r) * kL8Row + n2];
#pragma unroll
    for (int r = 0; r < NV / 8; ++r) dft8<T, M>(v + 8 * r, tw, sgn);
}

// Lines per workgroup of the four-step passes: 32 in FP32 and 16 in FP64
// (8 threads per line, so 256 and 128 threads; the LDS buffer is the same
// size, and the y and z passes read whole 256-byte rows either way)
template <typename R>
struct Fft8Lines {
    static constexpr int value = sizeof(R) == 4 ? 32 : 16;
};

// y pass, M = 64 or 128: a workgroup owns LN / 4 qx columns at one z
template <typename R, int M>
__device__ __forceinline__ void fft_y8_body(C1<R>* __restrict__ data, const double* __restrict__ twg, int sgn,
                                              int bid) {
    constexpr int LN = Fft8Lines<R>::value, HX = M / 2, W = LN / 4, NV = Fft8Line<M>::NV;
    __shared__ C1<R> buf[LN * Fft8Line<M>::LINE];
    __shared__ C1<R> tw[M];
    load_twiddles<R, M>(tw, twg, sgn);
    const int l = threadIdx.x % LN, t = threadIdx.x / LN;   // consecutive lanes: consecutive lines
    const int x0 = (bid % (HX / W)) * W;
    const int z = bid / (HX / W);
    C1<R>* base = data + ((size_t)z * M * HX + x0) * 4 + l;   // + (y HX) * 4
    C1<R> v[NV];
#pragma unroll
    for (int n1 = 0; n1 < NV; ++n1) v[n1] = base[(size_t)(8 * n1 + t) * HX * 4];
    __syncthreads();   // twiddles
    fft8_line<R, M>(v, buf + l * Fft8Line<M>::LINE, tw, t, sgn);
#pragma unroll
    for (int j = 0; j < NV; ++j) base[(size_t)Fft8Line<M>::out(t, j) * HX * 4] = v[j];
}

template <typename R, int M>
__global__ __launch_bounds__(256) void k_fft_y8(C1<R>* __restrict__ data, const double* __restrict__ twg,
                                                  int sgn) {
    fft_y8_body<R, M>(data, twg, sgn, blockIdx.x);
}

// z pass, M = 64 or 128: forward z transform, k-space multiply (as in
// k_fft_z_scale), inverse z transform; a workgroup owns LN / 4 qx columns at one qy
template <typename R, int M>
__device__ __forceinline__ void fft_z8_body(C1<R>* __restrict__ data, const double* __restrict__ twg, KScale ks,
                                              int bid) {
    constexpr int LN = Fft8Lines<R>::value, HX = M / 2, W = LN / 4, NV = Fft8Line<M>::NV;
    __shared__ C1<R> buf[LN * Fft8Line<M>::LINE];
    __shared__ C1<R> twf[M], twi[M];
    load_twiddles<R, M>(twf, twg, +1);
    load_twiddles<R, M>(twi, twg, -1);
    const int l = threadIdx.x % LN, t = threadIdx.x / LN;   // consecutive lanes: consecutive lines
    const int x0 = (bid % (HX / W)) * W;
    const int y = bid / (HX / W);
    const size_t zstride = (size_t)M * HX * 4;
    C1<R>* base = data + ((size_t)y * HX + x0) * 4 + l;   // + z zstride
    C1<R>* ln = buf + l * Fft8Line<M>::LINE;
    C1<R> v[NV];
#pragma unroll
    for (int n1 = 0; n1 < NV; ++n1) v[n1] = base[(size_t)(8 * n1 + t) * zstride];
    __syncthreads();   // twiddles
    fft8_line<R, M>(v, ln, twf, t, +1);
    __syncthreads();   // every thread has read its exchange rows
    // spectrum of this line in natural order: element qz at ln[qz]
#pragma unroll
    for (int j = 0; j < NV; ++j) ln[Fft8Line<M>::out(t, j)] = v[j];
    __syncthreads();
    const int qy = (y < M / 2) ? y : y - M;
    for (int e = threadIdx.x; e < W * M; e += 8 * LN) {
        const int w = e % W, z = e / W;
        const int qx = x0 + w;
        const int qz = (z < M / 2) ? z : z - M;
        C1<R>* f0 = buf + (w * 4 + 0) * Fft8Line<M>::LINE + z;
        C1<R>* f1 = buf + (w * 4 + 1) * Fft8Line<M>::LINE + z;
        C1<R>* f2 = buf + (w * 4 + 2) * Fft8Line<M>::LINE + z;
        C1<R>* f3 = buf + (w * 4 + 3) * Fft8Line<M>::LINE + z;
        const bool zero = (qx == 0 && qy == 0 && qz == 0) || (y == M / 2) || (z == M / 2);
        if (zero) {
            *f0 = *f1 = *f2 = *f3 = {R(0), R(0)};
            continue;
        }
        double kx, ky, kz, k2;
        const double ex = kscale_factor(ks, qx, qy, qz, kx, ky, kz, k2);
        const R st = (R)(ks.inv_eta * (1.0 + k2 * ks.inv4xi2) * ex);
        const R lp = (R)ex;
        const R rkx = (R)kx, rky = (R)ky, rkz = (R)kz, ik2 = (R)(1.0 / k2);
        const C1<R> h0 = *f0, h1 = *f1, h2 = *f2, h3 = *f3;
        const C1<R> kf = {rkx * h0.re + rky * h1.re + rkz * h2.re, rkx * h0.im + rky * h1.im + rkz * h2.im};
        const C1<R> pk = {kf.re * ik2, kf.im * ik2};
        const R sq = R(0.25) * (R)ks.inv_eta * lp;
        *f0 = {st * (h0.re - rkx * pk.re) - sq * rkx * h3.im, st * (h0.im - rkx * pk.im) + sq * rkx * h3.re};
        *f1 = {st * (h1.re - rky * pk.re) - sq * rky * h3.im, st * (h1.im - rky * pk.im) + sq * rky * h3.re};
        *f2 = {st * (h2.re - rkz * pk.re) - sq * rkz * h3.im, st * (h2.im - rkz * pk.im) + sq * rkz * h3.re};
        *f3 = {-lp * kf.im, lp * kf.re};
    }
    __syncthreads();
#pragma unroll
    for (int n1 = 0; n1 < NV; ++n1) v[n1] = ln[8 * n1 + t];
    __syncthreads();   // the exchange below reuses the line
    fft8_line<R, M>(v, ln, twi, t, -1);
#pragma unroll
    for (int j = 0; j < NV; ++j) base[(size_t)Fft8Line<M>::out(t, j) * zstride] = v[j];
}

template <typename R, int M>
__global__ __launch_bounds__(256) void k_fft_z8(C1<R>* __restrict__ data, const double* __restrict__ twg,
                                                  KScale ks) {
    fft_z8_body<R, M>(data, twg, ks, blockIdx.x);
}

// x pass, forward, M = 64 or 128: LN / 2 real lines per workgroup, each a pair of
// complex transforms (x + i y fields, z + i w fields), then the same
// half-spectrum unpacking as k_fft_x_fwd
template <typename R, int M>
__device__ __forceinline__ void fft_x_fwd8_body(const R4<R>* __restrict__ in, C1<R>* __restrict__ out,
                                                  const double* __restrict__ twg, int bid) {
    constexpr int LN = Fft8Lines<R>::value, RL = LN / 2, NV = Fft8Line<M>::NV;   // RL real lines
    __shared__ C1<R> buf[LN * Fft8Line<M>::LINE];
    __shared__ C1<R> tw[M];
    load_twiddles<R, M>(tw, twg, +1);
    const int l32 = threadIdx.x / 8, t = threadIdx.x % 8;   // complex line, thread in line
    const int line = l32 >> 1, g = l32 & 1;
    const size_t line0 = (size_t)bid * RL;
    // fields (x, y) and (z, w) of one line sit side by side in a wavefront
    const C1<R>* src = reinterpret_cast<const C1<R>*>(in) + ((line0 + line) * M + t) * 2 + g;
    C1<R> v[NV];
#pragma unroll
    for (int n1 = 0; n1 < NV; ++n1) v[n1] = src[16 * n1];
    __syncthreads();   // twiddles
    C1<R>* ln = buf + l32 * Fft8Line<M>::LINE;
    fft8_line<R, M>(v, ln, tw, t, +1);
    // Half-spectrum unpacking in registers, as in k_fft_x_fwd256: element
    // 8 c + t sits in v[jof(c)]; X[M - q] of q = 8 c + t (t > 0) sits in
    // lane 8 - t of the same line at c' = NV - 1 - c, and for t = 0 in the
    // thread itself at c' = (NV - c) mod NV.
    auto jof = [](int c) { return M == 128 ? 8 * (c & 1) + (c >> 1) : c; };
    const int pl = (int)(threadIdx.x & 63 & ~7) | ((8 - t) & 7);   // partner lane
    C1<R>* dst = out + (line0 + line) * (M / 2) * 4 + 2 * g;
#pragma unroll
    for (int c = 0; c < NV / 2; ++c) {
        const int q = 8 * c + t;
        const C1<R> A = v[jof(c)];
        const C1<R> Bp = v[jof(NV - 1 - c)];
        const C1<R> Bs = {__shfl(Bp.re, pl), __shfl(Bp.im, pl)};
        const C1<R> B = t == 0 ? v[jof((NV - c) % NV)] : Bs;
        dst[4 * q] = {R(0.5) * (A.re + B.re), R(0.5) * (A.im - B.im)};
        dst[4 * q + 1] = {R(0.5) * (A.im + B.im), R(-0.5) * (A.re - B.re)};
    }
}

template <typename R, int M>
__global__ __launch_bounds__(256) void k_fft_x_fwd8(const R4<R>* __restrict__ in, C1<R>* __restrict__ out,
                                                      const double* __restrict__ twg) {
    fft_x_fwd8_body<R, M>(in, out, twg, blockIdx.x);
}

// x pass, inverse, M = 64 or 128: half spectrum -> LN / 2 real lines per workgroup
template <typename R, int M>
__device__ __forceinline__ void fft_x_inv8_body(const C1<R>* __restrict__ in, R4<R>* __restrict__ out,
                                                  const double* __restrict__ twg, int bid) {
    constexpr int LN = Fft8Lines<R>::value, RL = LN / 2, NV = Fft8Line<M>::NV;   // RL real lines
    __shared__ C1<R> buf[LN * Fft8Line<M>::LINE];
    __shared__ C1<R> tw[M];
    load_twiddles<R, M>(tw, twg, -1);
    const size_t line0 = (size_t)bid * RL;
    const int l32 = threadIdx.x / 8, t = threadIdx.x % 8;   // complex line, thread in line
    const int line = l32 >> 1, g = l32 & 1;
    // as in k_fft_x_inv256: element x of complex line g from the two half
    // spectra at q = x or M - x, one 16-byte load (two in FP64) per element
    const R4<R>* sp = reinterpret_cast<const R4<R>*>(in + (line0 + line) * (M / 2) * 4) + g;
    C1<R> v[NV];
#pragma unroll
    for (int n1 = 0; n1 < NV; ++n1) {
        const int x = 8 * n1 + t;
        const int q = n1 < NV / 2 ? x : (x == M / 2 ? 0 : M - x);
        const R4<R> ab = sp[2 * q];
        if (n1 < NV / 2) {
            v[n1] = x == 0 ? C1<R>{ab.x, ab.z} : C1<R>{ab.x - ab.w, ab.y + ab.z};
        } else {
            v[n1] = x == M / 2 ? C1<R>{R(0), R(0)} : C1<R>{ab.x + ab.w, ab.z - ab.y};
        }
    }
    C1<R>* ln = buf + l32 * Fft8Line<M>::LINE;
    __syncthreads();   // twiddles
    fft8_line<R, M>(v, ln, tw, t, -1);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) ln[Fft8Line<M>::out(t, j)] = v[j];
    __syncthreads();
    for (int e = threadIdx.x; e < RL * M; e += 8 * LN) {
        const int l = e / M, x = e % M;
        const C1<R> A = buf[(2 * l) * Fft8Line<M>::LINE + x], B = buf[(2 * l + 1) * Fft8Line<M>::LINE + x];
        out[(line0 + l) * M + x] = {A.re, A.im, B.re, B.im};
    }
}

template <typename R, int M>
__global__ __launch_bounds__(256) void k_fft_x_inv8(const C1<R>* __restrict__ in, R4<R>* __restrict__ out,
                                                      const double* __restrict__ twg) {
    fft_x_inv8_body<R, M>(in, out, twg, blockIdx.x);
}

// ---------------------------------------------------------------------------
// gather: one wavefront per sphere (binned order, contiguous per XCD); each
// lane owns some (x, y) columns of the window and sums them over z in R, the
// column sums are added with Neumaier compensation and the wavefront reduces
// in FP64. Adds the pair/self part and writes y in input order.

// G lanes per sphere (64, 32 or 16): a wavefront gathers 64 / G spheres at
// once, each group of G lanes reading its sphere's columns 16 x-points at a
// time, and the 13 sums are reduced over log2(G) butterfly levels. Measured at
// N = 1e5, 256^3: 504 / 579 / 740 us for G = 64 / 32 / 16 (the shorter
// butterfly does not pay for the longer load chain of each lane).
constexpr int kGatherLanes = 64;
// wavefronts per gather workgroup (consecutive spheres of the binned order)
constexpr int kGatherWaves = 4;

// HYB (the hybrid size approach of Sec. 3.2): the Faxen Laplacians of the
// read-out come from the k-space field grid2 = (lap/6) v instead of the
// window, so the window is read plainly (eq. parseval-sum-2): U from
// v + a^2 Lv, Omega from v, E from grad (v + (3/5) a^2 Lv) with grad h = -2 g h.
template <typename R, int G, bool SHEAR, bool HYB>
__device__ __forceinline__ void gather_body(
    int n, const R* __restrict__ recs, const int* __restrict__ perm, const R4<R>* __restrict__ grid,
    const R4<R>* __restrict__ grid2, int M, int P, SpreadGeom sg, double inv_eta, int parts, int compressible,
    const double* __restrict__ ybuf, double* __restrict__ yout, int bid) {
    static_assert(G == 16 || G == 32 || G == 64, "lanes per sphere");
    constexpr int SPB = kGatherWaves * (64 / G);   // spheres per workgroup
    __shared__ R fac[SPB][2 * kMaxP];
    __shared__ R zt[SPB][4][kMaxP + 1];   // f_z(kz) u_z(kz)^k, k = 0..3 (zero past P)
    const int lane = threadIdx.x & (G - 1), sb = threadIdx.x / G;
    const int s0 = bid * SPB + sb;
    const bool active = s0 < n;       // every thread reaches the barrier
    const int s = active ? s0 : n - 1;
    const int mask = M - 1;
    const R* rc = recs + (size_t)rec_stride(P) * s;
    // the z loop loads ZC points of a column at once (many loads in flight
    // per lane); weights past P are zero
    constexpr int ZC = sizeof(R) == 4 ? 4 : 2;
    const int Pe = (P + ZC - 1) / ZC * ZC;
    for (int k = lane; k < 2 * P; k += G) fac[sb][k] = rc[kRecHead + k];
    for (int kz = lane; kz < Pe; kz += G) {
        const R uz = rc[6] + (R)kz, fz = kz < P ? rc[kRecHead + 2 * P + kz] : R(0);
        zt[sb][0][kz] = fz;
        zt[sb][1][kz] = fz * uz;
        zt[sb][2][kz] = fz * uz * uz;
        zt[sb][3][kz] = fz * uz * uz * uz;
    }
    __syncthreads();
    if (!active) return;
    const int4 i0 = make_int4(rec_i0(rc, 0), rec_i0(rc, 1), rec_i0(rc, 2), 0);
    const R d0x = rc[4], d0y = rc[5];
    const R c0 = rc[21], c1 = rc[22], e0 = rc[23], d1 = rc[3];
    const R Gxx = (R)sg.Gxx, Gyx = (R)sg.Gyx, Gyy = (R)sg.Gyy, Gzz = (R)sg.Gzz, Gzz2 = Gzz * Gzz;
    double acc[13];
    for (int c = 0; c < 13; ++c) acc[c] = 0.0;
    if (parts & kPartsWave) {
        R ac[13], cp[13];
        for (int c = 0; c < 13; ++c) ac[c] = cp[c] = R(0);
        const int P2 = P * P;
        // The window factorises into f_x f_y f_z and the Faxen polynomials
        // are cubic in u_z, so each (x, y) column is reduced over z to the
        // moments M_k[c] = sum_z f_z u_z^k g_c (k <= 3) first; the 13 outputs
        // follow from them per column.
        if constexpr (HYB) {
        const R a2 = rc[7], a2e = R(0.6) * rc[7];
        for (int e = lane; e < P2; e += G) {
            const int kx = e % P, ky = e / P;
            const R ux = d0x + (R)kx, uy = d0y + (R)ky;
            const R gX = Gxx * ux, gY = Gyx * ux + Gyy * uy;
            const R wxy = (R)sg.cw * fac[sb][kx] * fac[sb][P + ky];
            const int gx = (i0.x + kx) & mask, gy = (i0.y + ky) & mask;
            // z moments of v (0 and 1), of p (0) and of Lv (0 and 1)
            R m0x = 0, m0y = 0, m0z = 0, m0w = 0, m1x = 0, m1y = 0, m1z = 0;
            R l0x = 0, l0y = 0, l0z = 0, l1x = 0, l1y = 0, l1z = 0;
            // 32-bit offsets (a grid of at most 256^3 points)
            const R4<R>* colp = grid + (gy * M + gx);
            const R4<R>* colq = grid2 + (gy * M + gx);
            const unsigned zs = (unsigned)M * (unsigned)M;
            for (int kc = 0; kc < Pe; kc += ZC) {
                R4<R> gv[ZC], lv[ZC];
#pragma unroll
                for (int j = 0; j < ZC; ++j) {
                    const unsigned o = (unsigned)((i0.z + kc + j) & mask) * zs;
                    gv[j] = colp[o];
                    lv[j] = colq[o];
                }
#pragma unroll
                for (int j = 0; j < ZC; ++j) {
                    const R4<R> g = gv[j], l = lv[j];
                    const R t0 = zt[sb][0][kc + j], t1 = zt[sb][1][kc + j];
                    m0x += t0 * g.x;
                    m0y += t0 * g.y;
                    m0z += t0 * g.z;
                    m0w += t0 * g.w;
                    m1x += t1 * g.x;
                    m1y += t1 * g.y;
                    m1z += t1 * g.z;
                    l0x += t0 * l.x;
                    l0y += t0 * l.y;
                    l0z += t0 * l.z;
                    l1x += t1 * l.x;
                    l1y += t1 * l.y;
                    l1z += t1 * l.z;
                }
            }
            // grad (v + (3/5) a^2 Lv) read with grad h = -2 g h, g_z = Gzz u_z
            const R qx = R(2) * (m0x + a2e * l0x), qy = R(2) * (m0y + a2e * l0y), qz = R(2) * (m0z + a2e * l0z);
            const R sx = R(2) * Gzz * (m1x + a2e * l1x);
            const R sy = R(2) * Gzz * (m1y + a2e * l1y);
            const R sz = R(2) * Gzz * (m1z + a2e * l1z);
            const R hw = R(0.5) * wxy;
            R col[13];
            col[0] = wxy * (m0x + a2 * l0x);
            col[1] = wxy * (m0y + a2 * l0y);
            col[2] = wxy * (m0z + a2 * l0z);
            col[3] = wxy * (gY * m0z - Gzz * m1y);
            col[4] = wxy * (Gzz * m1x - gX * m0z);
            col[5] = wxy * (gX * m0y - gY * m0x);
            col[6] = wxy * (gX * qx);
            col[7] = wxy * (gY * qy);
            col[8] = wxy * sz;
            col[9] = hw * (gY * qx + gX * qy);
            col[10] = hw * (sx + gX * qz);
            col[11] = hw * (sy + gY * qz);
            col[12] = wxy * m0w;
            for (int c = 0; c < 13; ++c) {
                if constexpr (sizeof(R) == 4) neumaier(ac[c], cp[c], col[c]);
                else ac[c] += col[c];
            }
        }
        } else {
        for (int e = lane; e < P2; e += G) {
            const int kx = e % P, ky = e / P;
            const R ux = d0x + (R)kx, uy = d0y + (R)ky;
            const R gX = Gxx * ux, gY = Gyx * ux + Gyy * uy;
            const R wxy = (R)sg.cw * fac[sb][kx] * fac[sb][P + ky];
            const R gxy2 = gX * gX + gY * gY;
            const int gx = (i0.x + kx) & mask, gy = (i0.y + ky) & mask;
            R m0x = 0, m0y = 0, m0z = 0, m0w = 0, m1x = 0, m1y = 0, m1z = 0;
            R m2x = 0, m2y = 0, m2z = 0, m3x = 0, m3y = 0, m3z = 0;
            // 32-bit offsets (a grid of at most 256^3 points); ZC loads in
            // flight per chunk (a point past P has zero weight)
            const R4<R>* colp = grid + (gy * M + gx);
            const unsigned zs = (unsigned)M * (unsigned)M;
            for (int kc = 0; kc < Pe; kc += ZC) {
              R4<R> gv[ZC];
#pragma unroll
              for (int j = 0; j < ZC; ++j) gv[j] = colp[(unsigned)((i0.z + kc + j) & mask) * zs];
#pragma unroll
              for (int j = 0; j < ZC; ++j) {
                const int kz = kc + j;
                const R4<R> g = gv[j];
                const R t0 = zt[sb][0][kz], t1 = zt[sb][1][kz], t2 = zt[sb][2][kz], t3 = zt[sb][3][kz];
                m0x += t0 * g.x;
                m0y += t0 * g.y;
                m0z += t0 * g.z;
                m0w += t0 * g.w;
                m1x += t1 * g.x;
                m1y += t1 * g.y;
                m1z += t1 * g.z;
                m2x += t2 * g.x;
                m2y += t2 * g.y;
                m2z += t2 * g.z;
                m3x += t3 * g.x;
                m3y += t3 * g.y;
                m3z += t3 * g.z;
              }
            }
            // with w = wxy f_z, g_z = Gzz u_z and |g|^2 = gxy2 + Gzz^2 u_z^2:
            //   U = sum w (c0 + c1 |g|^2) v = wxy ((c0 + c1 gxy2) M0 + c1 Gzz^2 M2),
            //   q = sum (w/wxy)(e0 + d1 |g|^2) v, s = the same with one more u_z
            const R cu = c0 + c1 * gxy2, cq = e0 + d1 * gxy2;
            const R ux_ = cu * m0x + c1 * Gzz2 * m2x;
            const R uy_ = cu * m0y + c1 * Gzz2 * m2y;
            const R uz_ = cu * m0z + c1 * Gzz2 * m2z;
            const R qx = cq * m0x + d1 * Gzz2 * m2x;
            const R qy = cq * m0y + d1 * Gzz2 * m2y;
            const R qz = cq * m0z + d1 * Gzz2 * m2z;
            const R sx = Gzz * (cq * m1x + d1 * Gzz2 * m3x);
            const R sy = Gzz * (cq * m1y + d1 * Gzz2 * m3y);
            const R sz = Gzz * (cq * m1z + d1 * Gzz2 * m3z);
            R exx = R(0), exy = R(0);
            if constexpr (SHEAR) {   // -(4/5) a^2 Qt g_xy
                exx = -d1 * ((R)sg.Qxx * gX + (R)sg.Qxy * gY);
                exy = -d1 * ((R)sg.Qxy * gX + (R)sg.Qyy * gY);
            }
            const R hw = R(0.5) * wxy;
            R col[13];
            col[0] = wxy * ux_;
            col[1] = wxy * uy_;
            col[2] = wxy * uz_;
            col[3] = wxy * (gY * m0z - Gzz * m1y);
            col[4] = wxy * (Gzz * m1x - gX * m0z);
            col[5] = wxy * (gX * m0y - gY * m0x);
            col[6] = wxy * (gX * qx + exx * m0x);
            col[7] = wxy * (gY * qy + exy * m0y);
            col[8] = wxy * sz;
            col[9] = hw * (gY * qx + gX * qy + exy * m0x + exx * m0y);
            col[10] = hw * (sx + gX * qz + exx * m0z);
            col[11] = hw * (sy + gY * qz + exy * m0z);
            col[12] = wxy * m0w;
            for (int c = 0; c < 13; ++c) {
                if constexpr (sizeof(R) == 4) neumaier(ac[c], cp[c], col[c]);
                else ac[c] += col[c];   // FP64 sums need no compensation
            }
        }
        }
        for (int c = 0; c < 13; ++c) acc[c] = (double)ac[c] + (double)cp[c];
        for (int off = G / 2; off > 0; off >>= 1)
            for (int c = 0; c < 13; ++c) acc[c] += __shfl_xor(acc[c], off, G);
    }
    if (lane == 0) {
        const int i = perm[s];
        double out[12];
        const double* yb = ybuf + 12 * (size_t)s;
        for (int c = 0; c < 6; ++c) out[c] = yb[c] + acc[c];
        double e5[5];
        sym_to_e5<double>(acc + 6, e5);
        for (int c = 0; c < 5; ++c) out[6 + c] = yb[6 + c] + e5[c];
        out[11] = yb[11] - inv_eta * (kSqrt3 / 4.0) * acc[12];
        if (!compressible) out[11] = 0.0;
        for (int c = 0; c < 12; ++c) yout[12 * (size_t)i + c] = out[c];
    }
}

template <typename R, int G, bool SHEAR, bool HYB>
__global__ __launch_bounds__(64 * kGatherWaves) void k_gather(
    int n, const R* __restrict__ recs, const int* __restrict__ perm, const R4<R>* __restrict__ grid,
    const R4<R>* __restrict__ grid2, int M, int P, SpreadGeom sg, double inv_eta, int parts, int compressible,
    const double* __restrict__ ybuf, double* __restrict__ yout) {
    gather_body<R, G, SHEAR, HYB>(n, recs, perm, grid, grid2, M, P, sg, inv_eta, parts, compressible, ybuf, yout,
                                  xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// host-side launchers (declared in seasd_internal.h)

// The transform chain of one product: forward x, y, the z pass with the
// k-space multiply, inverse y, x. The hybrid size approach (rgrid2, spec2
// non-null) runs the generic kernels, whose z pass also writes the Laplacian
// fields, and inverts both spectra.
template <typename R>
static int launch_fft_chain_M(int M, void* rgrid, void* spec, void* rgrid2, void* spec2, const double* tw,
                              const KScale& ks, hipStream_t st, PhaseTimer* tm);

// Lines per workgroup of the x passes (LPB) and qx columns per workgroup of
// the y and z passes (W) for a grid of edge M.
template <typename R, int M>
struct FftShape {
    static constexpr bool dbl = sizeof(R) == 8;
    static constexpr int LPB = M <= 16 ? 8 : (M <= 64 ? 4 : 2);
    static constexpr int W = M == 8 ? 2 : (M == 256 ? (dbl ? 1 : 2) : (dbl ? 2 : 4));
};

#define FFT_CASE(MM, LPB, W)                                                                              \
    case MM: {                                                                                            \
        constexpr int MM8 = (MM == 64) ? 64 : 128; /* the four-step kernels' M (used when sp8) */        \
        const int lines = MM * MM;                                                                        \
        const bool sp256 = MM == 256 && !hyb;                                                             \
        const bool sp8 = (MM == 128 || MM == 64) && !hyb;                                                 \
        constexpr int LN8 = Fft8Lines<R>::value; /* lines per workgroup of the four-step passes */        \
        constexpr int LN16 = Fft16Lines<R>::value;                                                        \
        tm->begin(kPhaseFftXFwd, st);                                                                     \
        if (sp256)                                                                                        \
            hipLaunchKernelGGL((k_fft_x_fwd256<R>), dim3(lines / (LN16 / 2)), dim3(16 * LN16), 0, st,     \
                               (const R4<R>*)rgrid, (C1<R>*)spec, tw);                                    \
        else if (sp8)                                                                                     \
            hipLaunchKernelGGL((k_fft_x_fwd8<R, MM8>), dim3(lines / (LN8 / 2)), dim3(8 * LN8), 0, st,     \
                               (const R4<R>*)rgrid, (C1<R>*)spec, tw);                                    \
        else                                                                                              \
            hipLaunchKernelGGL((k_fft_x_fwd<R, MM, LPB>), dim3(lines / LPB), dim3(256), 0, st,            \
                               (const R4<R>*)rgrid, (C1<R>*)spec, tw);                                    \
        if (sp256) {                                                                                      \
            const dim3 g16((128 / (LN16 / 4)) * 256), b16(16 * LN16);                                     \
            tm->begin(kPhaseFftYFwd, st);                                                                 \
            hipLaunchKernelGGL((k_fft_y256<R>), g16, b16, 0, st, (C1<R>*)spec, tw, +1);                   \
            tm->begin(kPhaseFftZ, st);                                                                    \
            hipLaunchKernelGGL((k_fft_z256<R>), g16, b16, 0, st, (C1<R>*)spec, tw, ks);                   \
            tm->begin(kPhaseFftYInv, st);                                                                 \
            hipLaunchKernelGGL((k_fft_y256<R>), g16, b16, 0, st, (C1<R>*)spec, tw, -1);                   \
        } else if (sp8) {                                                                                 \
            const dim3 g8((MM8 / 2 / (LN8 / 4)) * MM8), b8(8 * LN8);                                     \
            tm->begin(kPhaseFftYFwd, st);                                                                 \
            hipLaunchKernelGGL((k_fft_y8<R, MM8>), g8, b8, 0, st, (C1<R>*)spec, tw, +1);                  \
            tm->begin(kPhaseFftZ, st);                                                                    \
            hipLaunchKernelGGL((k_fft_z8<R, MM8>), g8, b8, 0, st, (C1<R>*)spec, tw, ks);                  \
            tm->begin(kPhaseFftYInv, st);                                                                 \
            hipLaunchKernelGGL((k_fft_y8<R, MM8>), g8, b8, 0, st, (C1<R>*)spec, tw, -1);                  \
        } else {                                                                                          \
            tm->begin(kPhaseFftYFwd, st);                                                                 \
            hipLaunchKernelGGL((k_fft_y<R, MM, W>), dim3((MM / 2 / W) * MM), dim3(256), 0, st,            \
                               (C1<R>*)spec, tw, +1);                                                     \
            tm->begin(kPhaseFftZ, st);                                                                    \
            if (hyb) {                                                                                    \
                constexpr int WH = (W > 1) ? W / 2 : 1;                                                   \
                hipLaunchKernelGGL((k_fft_z_scale_hyb<R, MM, WH>), dim3((MM / 2 / WH) * MM), dim3(256),   \
                                   0, st, (C1<R>*)spec, (C1<R>*)spec2, tw, ks);                           \
            } else {                                                                                      \
                hipLaunchKernelGGL((k_fft_z_scale<R, MM, W>), dim3((MM / 2 / W) * MM), dim3(256), 0, st,  \
                                   (C1<R>*)spec, tw, ks);                                                 \
            }                                                                                             \
            tm->begin(kPhaseFftYInv, st);                                                                 \
            hipLaunchKernelGGL((k_fft_y<R, MM, W>), dim3((MM / 2 / W) * MM), dim3(256), 0, st,            \
                               (C1<R>*)spec, tw, -1);                                                     \
            if (hyb)                                                                                      \
                hipLaunchKernelGGL((k_fft_y<R, MM, W>), dim3((MM / 2 / W) * MM), dim3(256), 0, st,        \
                                   (C1<R>*)spec2, tw, -1);                                                \
        }                                                                                                 \
        tm->begin(kPhaseFftXInv, st);                                                                     \
        if (sp256)                                                                                        \
            hipLaunchKernelGGL((k_fft_x_inv256<R>), dim3(lines / (LN16 / 2)), dim3(16 * LN16), 0, st,     \
                               (const C1<R>*)spec, (R4<R>*)rgrid, tw);                                    \
        else if (sp8)                                                                                     \
            hipLaunchKernelGGL((k_fft_x_inv8<R, MM8>), dim3(lines / (LN8 / 2)), dim3(8 * LN8), 0, st,     \
                               (const C1<R>*)spec, (R4<R>*)rgrid, tw);                                    \
        else                                                                                              \
            hipLaunchKernelGGL((k_fft_x_inv<R, MM, LPB>), dim3(lines / LPB), dim3(256), 0, st,            \
                               (const C1<R>*)spec, (R4<R>*)rgrid, tw);                                    \
        if (hyb)                                                                                          \
            hipLaunchKernelGGL((k_fft_x_inv<R, MM, LPB>), dim3(lines / LPB), dim3(256), 0, st,            \
                               (const C1<R>*)spec2, (R4<R>*)rgrid2, tw);                                  \
        break;                                                                                            \
    }

template <typename R>
static int launch_fft_chain_M(int M, void* rgrid, void* spec, void* rgrid2, void* spec2, const double* tw,
                              const KScale& ks, hipStream_t st, PhaseTimer* tm) {
    constexpr bool dbl = sizeof(R) == 8;
    const bool hyb = rgrid2 != nullptr && spec2 != nullptr;
    switch (M) {
        FFT_CASE(8, (FftShape<R, 8>::LPB), (FftShape<R, 8>::W))
        FFT_CASE(16, (FftShape<R, 16>::LPB), (FftShape<R, 16>::W))
        FFT_CASE(32, (FftShape<R, 32>::LPB), (FftShape<R, 32>::W))
        FFT_CASE(64, (FftShape<R, 64>::LPB), (FftShape<R, 64>::W))
        FFT_CASE(128, (FftShape<R, 128>::LPB), (FftShape<R, 128>::W))
        FFT_CASE(256, (FftShape<R, 256>::LPB), (FftShape<R, 256>::W))
        default:
            return -1;
    }
    return 0;
}

static NbrGeom nbr_geom(const ApplyArgs& A) {
    NbrGeom g;
    g.cell = A.cell;
    for (int d = 0; d < 3; ++d) g.rpl[d] = A.reach_per_len[d];
    return g;
}

static SpreadGeom spread_geom(const ApplyArgs& A, bool gather) {
    const WinGeom& w = A.win;
    return SpreadGeom{w.Gxx, w.Gyx, w.Gyy, w.Gzz, w.Qxx, w.Qxy, w.Qyy, gather ? w.cwv : w.cw};
}

// FFT twiddle table tw[j] = (cos, sin)(2 pi j / M), j < M (exact argument
// reduction through sincospi)
__global__ void k_twiddles(int M, double* __restrict__ tw) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double sv, cv;
    sincospi(2.0 * (double)j / (double)M, &sv, &cv);
    tw[2 * j] = cv;
    tw[2 * j + 1] = sv;
}

int launch_twiddles(int M, double* tw, hipStream_t st) {
    hipLaunchKernelGGL(k_twiddles, dim3((M + 255) / 256), dim3(256), 0, st, M, tw);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// n ints set to zero by a kernel (a fill that a captured graph may hold)
__global__ void k_clear_ints(int n, int* __restrict__ p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

int launch_clear_ints(int n, int* p, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_clear_ints, dim3((n + 255) / 256), dim3(256), 0, st, n, p);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// binning: bins, their scan, binned copies of centres, radii and moments
int launch_geometry(const ApplyArgs& A, hipStream_t st, PhaseTimer* tm) {
    const int n = (int)A.n;
    const int T = 256;
    const int gb = (n + T - 1) / T;
    const int nbins = A.nb * A.nb * A.nb;
    tm->begin(kPhaseBin, st);
    hipLaunchKernelGGL(k_zero_geometry, dim3((nbins + T - 1) / T), dim3(T), 0, st, nbins, A.counts, A.fill,
                       A.amax_bits, A.nstats);
    hipLaunchKernelGGL(k_bin_count, dim3(gb), dim3(T), 0, st, n, A.pos, A.radius, A.cell, A.nb,
                       A.bin_of, A.counts, A.amax_bits, A.err);
    launch_scan(nbins, A.counts, A.start, A.scan_tmp, st);
    hipLaunchKernelGGL(k_bin_scatter, dim3(gb), dim3(T), 0, st, n, A.bin_of, A.start, A.fill, A.perm);
    hipLaunchKernelGGL(k_bin_order, dim3((nbins + T - 1) / T), dim3(T), 0, st, nbins, A.start, A.perm);
    hipLaunchKernelGGL(k_bin_gather, dim3(gb), dim3(T), 0, st, n, A.perm, A.pos, A.radius, A.x, A.cell,
                       A.compressible, A.sp, A.st, A.sa, A.sx, A.err);
    if (!(A.parts & kPartsReal)) hipMemsetAsync(A.ncount, 0, sizeof(int) * n, st);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// neighbour list into slots of A.cap entries; A.nstats (cleared by
// launch_geometry, or by the caller before a repeated pass) receives the
// largest and the total count (the list is complete when the largest fits A.cap)
int launch_pairlist(const ApplyArgs& A, hipStream_t st) {
    const int n = (int)A.n;
    if (!(A.parts & kPartsReal)) return 0;
    const NbrGeom g = nbr_geom(A);
    if (n < kWaveSpheres)
        hipLaunchKernelGGL((k_pair_fill_group<64>), dim3((n + 3) / 4), dim3(256), 0, st, n, A.sp, A.st, A.sa, A.start,
                           A.nb, g, A.rc_factor, A.amax_bits, A.checks, A.cap, A.ncount, A.list, A.err);
    else
        hipLaunchKernelGGL(k_pair_fill_bin, dim3((A.nb * A.nb * A.nb + 3) / 4), dim3(256), 0, st, n, A.sp, A.sa,
                           A.start, A.nb, g, A.rc_factor, A.amax_bits, A.checks, A.cap, A.ncount, A.list, A.err);
    hipLaunchKernelGGL(k_count_stats, dim3(std::min(kStatsBlocks, (n + 255) / 256)), dim3(256), 0, st, n, A.ncount,
                       A.nstats);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_edge_count(const ApplyArgs& A, double cut, int* deg, int* rowptr, hipStream_t st) {
    const int n = (int)A.n;
    hipLaunchKernelGGL(k_edge_count, dim3((n + 255) / 256), dim3(256), 0, st, n, A.sp, A.st, A.sa, A.start, A.nb,
                       nbr_geom(A), cut, A.amax_bits, deg, A.err);
    launch_scan(n, deg, rowptr, A.scan_tmp, st);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_edge_fill(const ApplyArgs& A, double cut, const int* rowptr, int* esrc, int* edst, int* erev,
                     float4* geo, float* fe, float* fn, hipStream_t st) {
    const int n = (int)A.n;
    hipLaunchKernelGGL(k_edge_fill, dim3((n + 255) / 256), dim3(256), 0, st, n, A.sp, A.st, A.sa, A.start, A.nb,
                       nbr_geom(A), cut, A.amax_bits, rowptr, esrc, edst, geo, fe, A.err);
    hipLaunchKernelGGL(k_edge_rev, dim3((n + 255) / 256), dim3(256), 0, st, n, A.sa, rowptr, edst, geo, erev, fn,
                       A.err);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// moments into binned order (used when the geometry is reused for a new x)
int launch_moments(const ApplyArgs& A, hipStream_t st) {
    const int n = (int)A.n;
    hipLaunchKernelGGL(k_bin_gather, dim3((n + 255) / 256), dim3(256), 0, st, n, A.perm, A.pos, A.radius, A.x,
                       A.cell, A.compressible, A.sp, A.st, A.sa, A.sx, A.err);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

KScale kscale_of(const ApplyArgs& A) {
    // B = 2 pi A^-T: row i of B is 2 pi times column i of A^-1
    const double* ai = A.cell.ainv;
    const double tp = 2.0 * kPi;
    return KScale{tp * ai[0], tp * ai[1], tp * ai[4], tp * ai[8], 1.0 / (4.0 * A.xi * A.xi), A.kdeconv,
                  1.0 / ((double)A.M * A.M * A.M), A.inv_eta};
}

template <typename R>
static void launch_window_spread(const ApplyArgs& A, bool wave, hipStream_t st, PhaseTimer* tm) {
    const int n = (int)A.n;
    const int tiles = A.M / kTile;
    const int gwin = (n + kWinSpheres - 1) / kWinSpheres;
    tm->begin(kPhaseWindow, st);
    hipLaunchKernelGGL((k_window<R>), dim3(gwin), dim3(256), 0, st, n, A.st, A.sa, A.sx, A.P, A.M, A.win.beta,
                       A.win.bq, A.win.bz, (R*)A.wrec);
    tm->begin(kPhaseSpread, st);
    if (!wave) return;
    const SpreadGeom sg = spread_geom(A, false);
    if (A.win.sheared)
        hipLaunchKernelGGL((k_spread<R, true>), dim3(tiles * tiles * tiles), dim3(64 * kSpreadWaves), 0, st, n,
                           (const R*)A.wrec, A.start, A.nb, A.M, A.P, sg, (R4<R>*)A.rgrid);
    else
        hipLaunchKernelGGL((k_spread<R, false>), dim3(tiles * tiles * tiles), dim3(64 * kSpreadWaves), 0, st, n,
                           (const R*)A.wrec, A.start, A.nb, A.M, A.P, sg, (R4<R>*)A.rgrid);
}

// Wave-space part up to the inverse FFT (window records, spreading, the FFT
// chain with the k-space multiply); it reads the binned geometry but not the
// neighbour list.
int launch_wave(const ApplyArgs& A, hipStream_t st, PhaseTimer* tm) {
    const bool wave = (A.parts & kPartsWave) != 0;
    const KScale ks = kscale_of(A);
    if (A.fp32) {
        launch_window_spread<float>(A, wave, st, tm);
        if (wave && launch_fft_chain_M<float>(A.M, A.rgrid, A.spec, A.rgrid2, A.spec2, A.twiddle, ks, st, tm))
            return -1;
    } else {
        launch_window_spread<double>(A, wave, st, tm);
        if (wave && launch_fft_chain_M<double>(A.M, A.rgrid, A.spec, A.rgrid2, A.spec2, A.twiddle, ks, st, tm))
            return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Pair sum (real-space part and self terms, on the neighbour list) into ybuf.
int launch_pair(const ApplyArgs& A, hipStream_t st, PhaseTimer* tm) {
    const int n = (int)A.n;
    tm->begin(kPhasePair, st);
    if (n < kWaveSpheres || A.pair_group == 64)   // small suspensions, or uneven lists
        hipLaunchKernelGGL((k_pair_eval_group<64>), dim3((n + 3) / 4), dim3(256), 0, st, n, A.sp, A.sa, A.sx,
                           A.ncount, A.cap, A.list, A.cell, A.xi, A.inv_eta, A.parts, A.ybuf);
    else
        hipLaunchKernelGGL(k_pair_eval, dim3((n + 127) / 128), dim3(128), 0, st, n, A.sp, A.sa, A.sx, A.ncount,
                           A.cap, A.list, A.cell, A.xi, A.inv_eta, A.parts, A.ybuf);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename R>
static void launch_gather_R(const ApplyArgs& A, hipStream_t st) {
    const int n = (int)A.n;
    constexpr int spb = kGatherWaves * (64 / kGatherLanes);
    constexpr int nt = 64 * kGatherWaves;
    const int gg = (n + spb - 1) / spb;
    const SpreadGeom sg = spread_geom(A, true);
    const R4<R>* g1 = (const R4<R>*)A.rgrid;
    const R4<R>* g2 = (const R4<R>*)A.rgrid2;
    if (A.hybrid)   // the window is read plainly: no sheared-cell Laplacian term
        hipLaunchKernelGGL((k_gather<R, kGatherLanes, false, true>), dim3(gg), dim3(nt), 0, st, n, (const R*)A.wrec,
                           A.perm, g1, g2, A.M, A.P, sg, A.inv_eta, A.parts, A.compressible, A.ybuf, A.y);
    else if (A.win.sheared)
        hipLaunchKernelGGL((k_gather<R, kGatherLanes, true, false>), dim3(gg), dim3(nt), 0, st, n, (const R*)A.wrec,
                           A.perm, g1, g2, A.M, A.P, sg, A.inv_eta, A.parts, A.compressible, A.ybuf, A.y);
    else
        hipLaunchKernelGGL((k_gather<R, kGatherLanes, false, false>), dim3(gg), dim3(nt), 0, st, n, (const R*)A.wrec,
                           A.perm, g1, g2, A.M, A.P, sg, A.inv_eta, A.parts, A.compressible, A.ybuf, A.y);
}

// Gather: the wave-space velocities added to the pair sum, scattered back to
// the caller's order.
int launch_gather(const ApplyArgs& A, hipStream_t st, PhaseTimer* tm) {
    tm->begin(kPhaseGather, st);
    if (A.fp32) launch_gather_R<float>(A, st);
    else launch_gather_R<double>(A, st);
    tm->end(st);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// Batched launches over many suspensions: each phase is one launch per kernel
// variant (precision, sheared or not, pair-sum lanes, FFT size) for the whole
// batch. Workgroup b takes item items[b] = (suspension, block of that
// suspension) and runs the same body as the single-suspension kernel on that
// suspension's arguments, read from a device array. Items are listed
// suspension by suspension, and the XCD renumbering hands each XCD a
// contiguous range of them, so one suspension's grid and spheres stay mostly
// in one L2.

struct MultiSys {
    ApplyArgs A;
    SpreadGeom sgs, sgg;   // window geometry of spreading and of the gather
    KScale ks;
};

enum MultiKind {
    kMkBin, kMkPair1, kMkPair64, kMkWindow, kMkSpread, kMkSpreadShear,
    kMkFftXF, kMkFftY, kMkFftZ, kMkFftXI, kMkGather, kMkGatherShear, kMkCount
};

struct MultiList {
    int kind, M;
    int64_t off;   // first item in the item array
    int count;     // items = workgroups of the launch
};

struct MultiPlan {
    int fp32 = 0;
    DevBuf sys, items;
    std::vector<MultiList> lists;
};

#define MULTI_ITEM()                                              \
    const int2 it = items[xcd_block(blockIdx.x, gridDim.x)];      \
    const MultiSys& S = sys[it.x];                                \
    const ApplyArgs& A = S.A;

__global__ __launch_bounds__(256) void k_bin_gather_multi(const MultiSys* __restrict__ sys,
                                                          const int2* __restrict__ items) {
    MULTI_ITEM();
    bin_gather_body((int)A.n, A.perm, A.pos, A.radius, A.x, A.cell, A.compressible, A.sp, A.st, A.sa, A.sx, A.err,
                    it.y);
}

__global__ __launch_bounds__(128) void k_pair_eval_multi(const MultiSys* __restrict__ sys,
                                                         const int2* __restrict__ items) {
    MULTI_ITEM();
    pair_eval_body((int)A.n, A.sp, A.sa, A.sx, A.ncount, A.cap, A.list, A.cell, A.xi, A.inv_eta, A.parts, A.ybuf,
                   it.y);
}

// lanes per sphere of the batched pair sum for uneven lists (256
// suspensions, lognormal radii: 18.98 / 18.58 / 18.19 ms per batch launch
// with 64 / 32 / 16 lanes; a whole launch fills the GPU, so fewer lanes per
// sphere and shorter reductions pay)
constexpr int kBatchPairLanes = 16;

__global__ __launch_bounds__(256) void k_pair_eval_group_multi(const MultiSys* __restrict__ sys,
                                                               const int2* __restrict__ items) {
    MULTI_ITEM();
    pair_eval_group_body<kBatchPairLanes>((int)A.n, A.sp, A.sa, A.sx, A.ncount, A.cap, A.list, A.cell, A.xi,
                                          A.inv_eta, A.parts, A.ybuf, it.y);
}

template <typename R>
__global__ __launch_bounds__(256) void k_window_multi(const MultiSys* __restrict__ sys,
                                                      const int2* __restrict__ items) {
    MULTI_ITEM();
    window_body<R>((int)A.n, A.st, A.sa, A.sx, A.P, A.M, A.win.beta, A.win.bq, A.win.bz, (R*)A.wrec, it.y);
}

template <typename R, bool SHEAR>
__global__ __launch_bounds__(64 * kSpreadWaves) void k_spread_multi(const MultiSys* __restrict__ sys,
                                                                    const int2* __restrict__ items) {
    MULTI_ITEM();
    spread_body<R, SHEAR>((int)A.n, (const R*)A.wrec, A.start, A.nb, A.M, A.P, S.sgs, (R4<R>*)A.rgrid, it.y);
}

template <typename R, int M, int LPB>
__global__ __launch_bounds__(256) void k_fft_x_fwd_multi(const MultiSys* __restrict__ sys,
                                                         const int2* __restrict__ items) {
    MULTI_ITEM();
    fft_x_fwd_body<R, M, LPB>((const R4<R>*)A.rgrid, (C1<R>*)A.spec, A.twiddle, it.y);
}

template <typename R, int M, int W>
__global__ __launch_bounds__(256) void k_fft_y_multi(const MultiSys* __restrict__ sys, const int2* __restrict__ items,
                                                     int sgn) {
    MULTI_ITEM();
    fft_y_body<R, M, W>((C1<R>*)A.spec, A.twiddle, sgn, it.y);
}

template <typename R, int M, int W>
__global__ __launch_bounds__(256) void k_fft_z_scale_multi(const MultiSys* __restrict__ sys,
                                                           const int2* __restrict__ items) {
    MULTI_ITEM();
    fft_z_scale_body<R, M, W>((C1<R>*)A.spec, A.twiddle, S.ks, it.y);
}

template <typename R, int M, int LPB>
__global__ __launch_bounds__(256) void k_fft_x_inv_multi(const MultiSys* __restrict__ sys,
                                                         const int2* __restrict__ items) {
    MULTI_ITEM();
    fft_x_inv_body<R, M, LPB>((const C1<R>*)A.spec, (R4<R>*)A.rgrid, A.twiddle, it.y);
}

// the four-step passes of FP32 grids of edge 64 and 128
template <typename R, int M>
__global__ __launch_bounds__(256) void k_fft_x_fwd8_multi(const MultiSys* __restrict__ sys,
                                                          const int2* __restrict__ items) {
    MULTI_ITEM();
    fft_x_fwd8_body<R, M>((const R4<R>*)A.rgrid, (C1<R>*)A.spec, A.twiddle, it.y);
}

template <typename R, int M>
__global__ __launch_bounds__(256) void k_fft_y8_multi(const MultiSys* __restrict__ sys,
                                                      const int2* __restrict__ items, int sgn) {
    MULTI_ITEM();
    fft_y8_body<R, M>((C1<R>*)A.spec, A.twiddle, sgn, it.y);
}

template <typename R, int M>
__global__ __launch_bounds__(256) void k_fft_z8_multi(const MultiSys* __restrict__ sys,
                                                      const int2* __restrict__ items) {
    MULTI_ITEM();
    fft_z8_body<R, M>((C1<R>*)A.spec, A.twiddle, S.ks, it.y);
}

template <typename R, int M>
__global__ __launch_bounds__(256) void k_fft_x_inv8_multi(const MultiSys* __restrict__ sys,
                                                          const int2* __restrict__ items) {
    MULTI_ITEM();
    fft_x_inv8_body<R, M>((const C1<R>*)A.spec, (R4<R>*)A.rgrid, A.twiddle, it.y);
}

template <typename R, bool SHEAR>
__global__ __launch_bounds__(64 * kGatherWaves) void k_gather_multi(const MultiSys* __restrict__ sys,
                                                      const int2* __restrict__ items) {
    MULTI_ITEM();
    gather_body<R, kGatherLanes, SHEAR, false>((int)A.n, (const R*)A.wrec, A.perm, (const R4<R>*)A.rgrid,
                                               (const R4<R>*)A.rgrid, A.M, A.P, S.sgg, A.inv_eta, A.parts,
                                               A.compressible, A.ybuf, A.y, it.y);
}

static int fft_lpb(int M, bool dbl) { (void)dbl; return M <= 16 ? 8 : (M <= 64 ? 4 : 2); }
static int fft_w(int M, bool dbl) { return M == 8 ? 2 : (M == 256 ? (dbl ? 1 : 2) : (dbl ? 2 : 4)); }

int multi_plan_build(const ApplyArgs* args, int nsys, MultiPlan** out, hipStream_t st) {
    *out = nullptr;
    if (nsys < 1) return -1;
    auto* P = new MultiPlan();
    P->fp32 = args[0].fp32;
    std::vector<MultiSys> sys(nsys);
    std::vector<std::vector<int2>> per(kMkCount * 9);   // kind x log2(M) - 3 (FFT kinds), else slot 0
    auto slot = [](int kind, int M) {
        const int lm = M > 0 ? 31 - __builtin_clz((unsigned)M) - 3 : 0;
        return kind * 9 + lm;
    };
    auto add = [&](int kind, int M, int k, int nblk) {
        auto& v = per[slot(kind, M)];
        for (int b = 0; b < nblk; ++b) v.push_back(make_int2(k, b));
    };
    for (int k = 0; k < nsys; ++k) {
        const ApplyArgs& A = args[k];
        // one precision, the real-space size approach and both parts
        if (A.fp32 != P->fp32 || A.hybrid || A.parts != (kPartsReal | kPartsWave | kPartsSelf) || A.M < 8 ||
            A.M > 256 || (A.M & (A.M - 1))) {
            delete P;
            return -8;
        }
        sys[k].A = A;
        sys[k].sgs = spread_geom(A, false);
        sys[k].sgg = spread_geom(A, true);
        sys[k].ks = kscale_of(A);
        const int n = (int)A.n, M = A.M;
        const bool dbl = !A.fp32;
        add(kMkBin, 0, k, (n + 255) / 256);
        // the batch fills the GPU however small each suspension is: a group
        // of lanes per sphere only where its lists are uneven
        constexpr int spw = 256 / kBatchPairLanes;   // spheres per workgroup
        if (A.pair_group == 64) add(kMkPair64, 0, k, (n + spw - 1) / spw);
        else add(kMkPair1, 0, k, (n + 127) / 128);
        add(kMkWindow, 0, k, (n + kWinSpheres - 1) / kWinSpheres);
        const int tiles = M / kTile;
        add(A.win.sheared ? kMkSpreadShear : kMkSpread, 0, k, tiles * tiles * tiles);
        // the four-step passes: ln lines per workgroup (32 FP32, 16 FP64)
        const bool f8 = M == 128 || M == 64;
        const int ln = dbl ? Fft8Lines<double>::value : Fft8Lines<float>::value;
        add(kMkFftXF, M, k, f8 ? M * M / (ln / 2) : M * M / fft_lpb(M, dbl));
        add(kMkFftY, M, k, f8 ? (M / 2 / (ln / 4)) * M : (M / 2 / fft_w(M, dbl)) * M);
        add(kMkFftZ, M, k, f8 ? (M / 2 / (ln / 4)) * M : (M / 2 / fft_w(M, dbl)) * M);
        add(kMkFftXI, M, k, f8 ? M * M / (ln / 2) : M * M / fft_lpb(M, dbl));
        constexpr int spb = kGatherWaves * (64 / kGatherLanes);
        add(A.win.sheared ? kMkGatherShear : kMkGather, 0, k, (n + spb - 1) / spb);
    }
    std::vector<int2> all;
    for (int kind = 0; kind < kMkCount; ++kind)
        for (int lm = 0; lm < 9; ++lm) {
            auto& v = per[kind * 9 + lm];
            if (v.empty()) continue;
            const bool fft = kind == kMkFftXF || kind == kMkFftY || kind == kMkFftZ || kind == kMkFftXI;
            P->lists.push_back(MultiList{kind, fft ? (8 << lm) : 0, (int64_t)all.size(), (int)v.size()});
            all.insert(all.end(), v.begin(), v.end());
        }
    if (P->sys.ensure(sizeof(MultiSys) * nsys) || P->items.ensure(sizeof(int2) * all.size())) {
        delete P;
        return -7;
    }
    if (hipMemcpyAsync(P->sys.p, sys.data(), sizeof(MultiSys) * nsys, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(P->items.p, all.data(), sizeof(int2) * all.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        P->sys.release();
        P->items.release();
        delete P;
        return -6;
    }
    *out = P;
    return 0;
}

void multi_plan_free(MultiPlan* P) {
    if (!P) return;
    P->sys.release();
    P->items.release();
    delete P;
}

#define MULTI_LAUNCH(KERNEL, THREADS, ...)                                                                  \
    hipLaunchKernelGGL(KERNEL, dim3(L.count), dim3(THREADS), 0, st, (const MultiSys*)P->sys.p,              \
                       (const int2*)P->items.p + L.off, ##__VA_ARGS__)

int multi_queue_moments(const MultiPlan* P, hipStream_t st) {
    for (const MultiList& L : P->lists)
        if (L.kind == kMkBin) MULTI_LAUNCH(k_bin_gather_multi, 256);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int multi_queue_pair(const MultiPlan* P, hipStream_t st) {
    for (const MultiList& L : P->lists) {
        if (L.kind == kMkPair1) MULTI_LAUNCH(k_pair_eval_multi, 128);
        if (L.kind == kMkPair64) MULTI_LAUNCH(k_pair_eval_group_multi, 256);
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

#define MULTI_FFT_CASE(MM)                                                                                \
    case MM: {                                                                                            \
        constexpr int LPB = FftShape<R, MM>::LPB, W = FftShape<R, MM>::W;                                 \
        if (L.kind == kMkFftXF) MULTI_LAUNCH((k_fft_x_fwd_multi<R, MM, LPB>), 256);                       \
        if (L.kind == kMkFftY) MULTI_LAUNCH((k_fft_y_multi<R, MM, W>), 256, sgn);                          \
        if (L.kind == kMkFftZ) MULTI_LAUNCH((k_fft_z_scale_multi<R, MM, W>), 256);                        \
        if (L.kind == kMkFftXI) MULTI_LAUNCH((k_fft_x_inv_multi<R, MM, LPB>), 256);                       \
        break;                                                                                            \
    }

template <typename R>
static void multi_fft_pass(const MultiPlan* P, int kind, int sgn, hipStream_t st) {
    for (const MultiList& L : P->lists) {
        if (L.kind != kind) continue;
        if (L.M == 128 || L.M == 64) {
            constexpr int b8 = 8 * Fft8Lines<R>::value;
            if (L.M == 128) {
                if (kind == kMkFftXF) MULTI_LAUNCH((k_fft_x_fwd8_multi<R, 128>), b8);
                if (kind == kMkFftY) MULTI_LAUNCH((k_fft_y8_multi<R, 128>), b8, sgn);
                if (kind == kMkFftZ) MULTI_LAUNCH((k_fft_z8_multi<R, 128>), b8);
                if (kind == kMkFftXI) MULTI_LAUNCH((k_fft_x_inv8_multi<R, 128>), b8);
            } else {
                if (kind == kMkFftXF) MULTI_LAUNCH((k_fft_x_fwd8_multi<R, 64>), b8);
                if (kind == kMkFftY) MULTI_LAUNCH((k_fft_y8_multi<R, 64>), b8, sgn);
                if (kind == kMkFftZ) MULTI_LAUNCH((k_fft_z8_multi<R, 64>), b8);
                if (kind == kMkFftXI) MULTI_LAUNCH((k_fft_x_inv8_multi<R, 64>), b8);
            }
            continue;
        }
        switch (L.M) {
            MULTI_FFT_CASE(8)
            MULTI_FFT_CASE(16)
            MULTI_FFT_CASE(32)
            MULTI_FFT_CASE(64)
            MULTI_FFT_CASE(128)
            MULTI_FFT_CASE(256)
            default:
                break;
        }
    }
}

template <typename R>
static void multi_wave_R(const MultiPlan* P, hipStream_t st) {
    for (const MultiList& L : P->lists) {
        if (L.kind == kMkWindow) MULTI_LAUNCH((k_window_multi<R>), 256);
    }
    for (const MultiList& L : P->lists) {
        if (L.kind == kMkSpread) MULTI_LAUNCH((k_spread_multi<R, false>), 64 * kSpreadWaves);
        if (L.kind == kMkSpreadShear) MULTI_LAUNCH((k_spread_multi<R, true>), 64 * kSpreadWaves);
    }
    multi_fft_pass<R>(P, kMkFftXF, 0, st);
    multi_fft_pass<R>(P, kMkFftY, +1, st);
    multi_fft_pass<R>(P, kMkFftZ, 0, st);
    multi_fft_pass<R>(P, kMkFftY, -1, st);
    multi_fft_pass<R>(P, kMkFftXI, 0, st);
}

// window records, spreading and the transform chain of every suspension
int multi_queue_wave(const MultiPlan* P, hipStream_t st) {
    if (P->fp32) multi_wave_R<float>(P, st);
    else multi_wave_R<double>(P, st);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename R>
static void multi_gather_R(const MultiPlan* P, hipStream_t st) {
    for (const MultiList& L : P->lists) {
        if (L.kind == kMkGather) MULTI_LAUNCH((k_gather_multi<R, false>), 64 * kGatherWaves);
        if (L.kind == kMkGatherShear) MULTI_LAUNCH((k_gather_multi<R, true>), 64 * kGatherWaves);
    }
}

int multi_queue_gather(const MultiPlan* P, hipStream_t st) {
    if (P->fp32) multi_gather_R<float>(P, st);
    else multi_gather_R<double>(P, st);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace seasd
