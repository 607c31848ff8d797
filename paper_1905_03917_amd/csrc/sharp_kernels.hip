// sharp_kernels.hip -- gfx950 kernels of the accelerated sharp-interface method
// (Long, Cai & Pan): cut-cell WENO5-LLF finite-volume stages (Sec. 2.1,
// Eq. Eulerdiscrete), level-set geometry, interface interaction, extension,
// mixing, level-set advection and reinitialisation (Sec. 2.2-2.3), and the
// bookkeeping of the accelerated cycle (Sec. 3.1: interpolation, Eq.
// interpolation; interfacial flux correction, Eqs. firstcorrection and
// secondcorrection).
//
// Work is organised in tiles of 256 cells (1-D 256, 2-D 16x16, 3-D 8x8x4).
// Every kernel walks a device-resident tile list with a grid-stride loop over
// the device-side count (the host reads the counts back at its CFL readbacks
// only to size the grids): bulk tiles of one fluid (no interface within reach
// of the stencil) take the lean path, band tiles (the level-set band, dilated
// by one tile) take the cut-cell path, and kernels that touch band-mask cells
// only walk the inner band tiles.  All per-cell state is
// structure-of-arrays FP64 in HBM, x fastest, so a wavefront reads 64
// consecutive doubles of one component.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>

#include <hip/hip_ext.h>

#include "sharp_internal.h"

namespace sharp {

template <int D> struct Tile;
template <> struct Tile<1> { static constexpr int X = 256, Y = 1, Z = 1; };
template <> struct Tile<2> { static constexpr int X = 16, Y = 16, Z = 1; };
template <> struct Tile<3> { static constexpr int X = 8, Y = 8, Z = 4; };

// origin of tile t and the cell handled by this thread; false if outside the domain
template <int D>
__device__ __forceinline__ bool tile_cell(const Dev& g, int t, int tid, int& i, int& j, int& k)
{
    int tx = t % g.nt[0], ty = (t / g.nt[0]) % g.nt[1], tz = t / (g.nt[0] * g.nt[1]);
    i = tx * Tile<D>::X + tid % Tile<D>::X;
    j = ty * Tile<D>::Y + (tid / Tile<D>::X) % Tile<D>::Y;
    k = tz * Tile<D>::Z + tid / (Tile<D>::X * Tile<D>::Y);
    return i < g.n[0] && j < g.n[1] && k < g.n[2];
}

__device__ __forceinline__ int list_count(const Dev& g, int list) { return g.counts[list]; }
__device__ __forceinline__ const int* list_ptr(const Dev& g, int list) { return g.lists + (size_t)list * g.ntiles; }

// XCD-aware assignment of list positions to the blocks of a grid-stride
// loop.  Workgroup b runs on XCD b % 8, and each XCD has its own L2; giving
// every XCD a contiguous range of the (row-major) tile list keeps tiles whose
// halos overlap in the same L2.  Grids that are not a multiple of 8 use the
// plain stride.  (A fused launch starts each simulation's share of 8k blocks
// at a multiple of 8, so blk.b % 8 is still the XCD.)
struct ListRange { int begin, end, step; };
__device__ __forceinline__ ListRange xcd_range(const VB blk, int count)
{
    const int G = blk.n;
    if (G < 8 || (G & 7)) return {blk.b, count, G};
    const int x = blk.b & 7, j = blk.b >> 3, chunk = (count + 7) >> 3;
    const int b = x * chunk;
    return {b + j, min(count, b + chunk), G >> 3};
}

__device__ __forceinline__ void flag_error(const Dev& g, unsigned long long bits)
{
    atomicOr(&g.red[4], bits);
}
// a non-physical state of fluid k in cell c: the flag, and the lowest
// (cell, fluid) code found, which names the cell in the error message
__device__ __forceinline__ void flag_nonphys(const Dev& g, int c, int k)
{
    atomicOr(&g.red[4], (unsigned long long)ERR_NONPHYS);
    atomicMin(&g.red[RED_CELL], ((unsigned long long)(unsigned)c << 1) | (unsigned long long)(k & 1));
}

// ---------------------------------------------------------------------------
// band mask: a cell is in the band when it or an axis neighbour is closer
// than ls_band cells to the interface.  A tile is marked as a core tile when
// a cell is within ls_band + 2 cells.  The level set changes only on inner
// tiles, so a cell of a ring tile can join the band only through its inner
// neighbour, whose |phi| must then fall by the margin within one cycle; the
// interface moves by about CFL < 1 cell per cycle, so two cells keep the
// band off the ring tiles however close to a tile edge it starts.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void b_mask(const VB blk, const Dev& g, int list, int check_ring)
{
    __shared__ int any;
    const int* L = list_ptr(g, list);
    const double R = g.lsb * g.h, Rc = (g.lsb + 2.0) * g.h;
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int t = L[ti];
        if (threadIdx.x == 0) any = 0;
        __syncthreads();
        int i, j, k;
        if (tile_cell<D>(g, t, threadIdx.x, i, j, k)) {
            int c = i + g.n[0] * (j + g.n[1] * k);
            double m = fabs(g.phiP[c]);
#pragma unroll
            for (int d = 0; d < D; d++) {
                m = fmin(m, fabs(g.phiP[nbr(g, c, d, -1)]));
                m = fmin(m, fabs(g.phiP[nbr(g, c, d, 1)]));
            }
            uint8_t in = m < R;
            g.M[c] = in;
            if (m < Rc) any = 1;
            if (in && check_ring && (g.tflag[t] & 4)) flag_error(g, ERR_BAND_OVERFLOW);
        }
        __syncthreads();
        if (threadIdx.x == 0) g.tcore[t] = any;
        __syncthreads();
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_mask(Dev g, int list, int check_ring)
{
    b_mask<D>(VB::grid(), g, list, check_ring);
}

// tile classification: band = within one tile of a core tile, candidate =
// within two, ring = band tile with a non-band neighbour
__device__ __forceinline__ int tile_nbr(const Dev& g, int t, int dx, int dy, int dz)
{
    int tx = t % g.nt[0], ty = (t / g.nt[0]) % g.nt[1], tz = t / (g.nt[0] * g.nt[1]);
    int o[3] = {tx + dx, ty + dy, tz + dz};
    for (int d = 0; d < 3; d++) {
        if (o[d] < 0 || o[d] >= g.nt[d]) {
            if (d < g.D && g.bc[d] == 1) o[d] = (o[d] + g.nt[d]) % g.nt[d];
            else return -1;
        }
    }
    return o[0] + g.nt[0] * (o[1] + g.nt[1] * o[2]);
}

template <int D>
__device__ __forceinline__ void b_tiles1(const VB blk, const Dev& g)
{
    for (int t = blk.b * blockDim.x + threadIdx.x; t < g.ntiles; t += blk.n * blockDim.x) {
        int band = 0, cand = 0;
        int r2y = D > 1 ? 2 : 0, r2z = D > 2 ? 2 : 0;
        for (int dz = -r2z; dz <= r2z; dz++)
            for (int dy = -r2y; dy <= r2y; dy++)
                for (int dx = -2; dx <= 2; dx++) {
                    int u = tile_nbr(g, t, dx, dy, dz);
                    if (u < 0 || !g.tcore[u]) continue;
                    cand = 1;
                    if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) band = 1;
                }
        g.tflag[t] = band | (cand << 1);
        int tx = t % g.nt[0], ty = (t / g.nt[0]) % g.nt[1], tz = t / (g.nt[0] * g.nt[1]);
        int c = tx * Tile<D>::X + g.n[0] * (ty * Tile<D>::Y + g.n[1] * (tz * Tile<D>::Z));
        g.tsign[t] = g.phiP[c] < 0.0 ? 0 : 1;
    }
}
template <int D>
__global__ void k_tiles1(Dev g)
{
    b_tiles1<D>(VB::grid(), g);
}

template <int D>
__device__ __forceinline__ void b_tiles2(const VB blk, const Dev& g)
{
    for (int t = blk.b * blockDim.x + threadIdx.x; t < g.ntiles; t += blk.n * blockDim.x) {
        int f = g.tflag[t];
        if (!(f & 1)) continue;
        int ring = 0;
        int ry = D > 1 ? 1 : 0, rz = D > 2 ? 1 : 0;
        for (int dz = -rz; dz <= rz; dz++)
            for (int dy = -ry; dy <= ry; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int u = tile_nbr(g, t, dx, dy, dz);
                    if (u >= 0 && !(g.tflag[u] & 1)) ring = 1;
                }
        g.tflag[t] = f | (ring << 2);
    }
}
template <int D>
__global__ void k_tiles2(Dev g)
{
    b_tiles2<D>(VB::grid(), g);
}

// cells of tile t inside the domain
__device__ __forceinline__ int tile_cells(const Dev& g, int t)
{
    int tx = t % g.nt[0], ty = (t / g.nt[0]) % g.nt[1], tz = t / (g.nt[0] * g.nt[1]);
    int o[3] = {tx * g.T[0], ty * g.T[1], tz * g.T[2]};
    int n = 1;
    for (int d = 0; d < 3; d++) n *= min(g.T[d], g.n[d] - o[d]);
    return n;
}

// single-block compaction of the tile lists (band, candidate, bulk of each
// fluid, inner) and their cell counts
__device__ __forceinline__ void b_compact(const VB blk, const Dev& g)
{
    constexpr int NL = 5;   // list slot 4 holds LIST_INNER
    __shared__ int cnt[NL][1024];
    __shared__ int ccl[NL][1024];
    int nt = g.ntiles, tid = threadIdx.x, nth = blockDim.x;
    int chunk = (nt + nth - 1) / nth;
    int lo = tid * chunk, hi = min(nt, lo + chunk);
    int c[NL] = {0, 0, 0, 0, 0}, cc[NL] = {0, 0, 0, 0, 0};
    for (int t = lo; t < hi; t++) {
        int f = g.tflag[t], nc = tile_cells(g, t);
        if (f & 1) { c[0]++; cc[0] += nc; }
        if (f & 2) { c[1]++; cc[1] += nc; }
        if (!(f & 1)) { c[2 + g.tsign[t]]++; cc[2 + g.tsign[t]] += nc; }
        if ((f & 1) && !(f & 4)) { c[4]++; cc[4] += nc; }
    }
    for (int l = 0; l < NL; l++) { cnt[l][tid] = c[l]; ccl[l][tid] = cc[l]; }
    __syncthreads();
    for (int off = nth / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int l = 0; l < NL; l++) ccl[l][tid] += ccl[l][tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        for (int l = 0; l < 4; l++) g.counts[8 + l] = ccl[l][0];
        g.counts[8 + LIST_INNER] = ccl[4][0];
    }
    // exclusive scan (Hillis-Steele on a copy)
    for (int off = 1; off < nth; off <<= 1) {
        int v[NL];
        for (int l = 0; l < NL; l++) v[l] = tid >= off ? cnt[l][tid - off] : 0;
        __syncthreads();
        for (int l = 0; l < NL; l++) cnt[l][tid] += v[l];
        __syncthreads();
    }
    int base[NL];
    for (int l = 0; l < NL; l++) base[l] = cnt[l][tid] - c[l];
    if (tid == nth - 1) {
        for (int l = 0; l < 4; l++) g.counts[l] = cnt[l][tid];
        g.counts[LIST_INNER] = cnt[4][tid];
    }
    for (int t = lo; t < hi; t++) {
        int f = g.tflag[t];
        if (f & 1) g.lists[(size_t)LIST_BAND * nt + base[0]++] = t;
        if (f & 2) g.lists[(size_t)LIST_CAND * nt + base[1]++] = t;
        if (!(f & 1)) {
            int l = 2 + g.tsign[t];
            g.lists[(size_t)l * nt + base[l]++] = t;
        }
        if ((f & 1) && !(f & 4)) g.lists[(size_t)LIST_INNER * nt + base[4]++] = t;
    }
}
__global__ void __launch_bounds__(1024) k_compact(Dev g)
{
    b_compact(VB::grid(), g);
}

// ---------------------------------------------------------------------------
// geometry: volume fraction and low-face apertures of every cell of the
// listed tiles (plus the padded high faces on the domain boundary)
// ---------------------------------------------------------------------------
// The geometry is built into a second buffer set while kernels of the
// previous stage may still read the first.  The per-tile |phi| minima of the
// tiles a launch over `list` does not rebuild are carried over into the
// buffer it writes, so both buffers agree outside the rebuilt tiles.
__device__ __forceinline__ void tpm_carry(const VB blk, int nth, const Dev& g, int list, const double* cur,
                                          double* out)
{
    if (list == LIST_ALL || !cur) return;
    for (int t = blk.b * nth + threadIdx.x; t < g.ntiles; t += blk.n * nth) {
        const int f = g.tflag[t];
        const bool built = list == LIST_BAND ? (f & 1) != 0 : ((f & 1) && !(f & 4));
        if (!built) out[t] = cur[t];
    }
}

// the tile's and its halo's level set and vertex values are staged in LDS
template <int D> struct GeoRegion;
template <> struct GeoRegion<1> { static constexpr int X = 256 + 2, Y = 1, Z = 1; };
template <> struct GeoRegion<2> { static constexpr int X = 16 + 2, Y = 16 + 2, Z = 1; };
template <> struct GeoRegion<3> { static constexpr int X = 8 + 2, Y = 8 + 2, Z = 4 + 2; };

template <int D>
__device__ __forceinline__ void b_geom_lds(const VB blk, const Dev& g, int list, const double* cur,
                                           const double* tpm_cur)
{
    constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
    constexpr int CX = GeoRegion<D>::X, CY = GeoRegion<D>::Y, CZ = GeoRegion<D>::Z, CN = CX * CY * CZ;
    constexpr int VX = TX + 1, VY = D > 1 ? TY + 1 : 1, VZ = D > 2 ? TZ + 1 : 1, VN = VX * VY * VZ;
    __shared__ double sP[CN];
    __shared__ double sV[VN];
    __shared__ double sMin[SHARP_WG / 64];
    __shared__ unsigned sSgn[SHARP_WG / 64];
    tpm_carry(blk, SHARP_WG, g, list, tpm_cur, g.tphimin);
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int t = L[ti];
        int ox = (t % g.nt[0]) * TX, oy = ((t / g.nt[0]) % g.nt[1]) * TY, oz = (t / (g.nt[0] * g.nt[1])) * TZ;
        // cells (ox-1 .. ox+TX) x ...; also min |phi| over them (the mixing
        // region of the tile) and which signs occur (bit 0: phi < 0, bit 1:
        // phi >= 0)
        double pmin = INFINITY;
        unsigned sgn = 0;
        for (int r = threadIdx.x; r < CN; r += SHARP_WG) {
            int cx = r % CX, cy = (r / CX) % CY, cz = r / (CX * CY);
            sP[r] = phi_at(g, cur, cidx(g, ox - 1 + cx, D > 1 ? oy - 1 + cy : 0, D > 2 ? oz - 1 + cz : 0));
            pmin = fmin(pmin, fabs(sP[r]));
            sgn |= sP[r] < 0.0 ? 1u : (sP[r] > 0.0 ? 2u : 3u);
        }
        for (int off = 32; off > 0; off >>= 1) pmin = fmin(pmin, __shfl_down(pmin, off, 64));
        const unsigned wsgn = (__ballot(sgn & 1u) ? 1u : 0u) | (__ballot(sgn & 2u) ? 2u : 0u);
        if ((threadIdx.x & 63) == 0) {
            sMin[threadIdx.x >> 6] = pmin;
            sSgn[threadIdx.x >> 6] = wsgn;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < SHARP_WG / 64; w++) pmin = fmin(pmin, sMin[w]);
            g.tphimin[t] = pmin;
        }
        // every cell of the region on one side, none on the level set: all
        // vertices share that sign, so every aperture (and the volume
        // fraction) is exactly 1 (phi < 0) or 0 (phi > 0)
        unsigned tsg = 0;
        for (int w = 0; w < SHARP_WG / 64; w++) tsg |= sSgn[w];
        const bool one_side = tsg == 1u || tsg == 2u;
        const double side_A = tsg == 1u ? 1.0 : 0.0;
        // vertex (vx, vy, vz) <-> corner (ox+vx, ...): mean of cells (vx-1 .. vx) in region offset +1
        for (int r = threadIdx.x; r < VN; r += SHARP_WG) {
            int vx = r % VX, vy = (r / VX) % VY, vz = r / (VX * VY);
            double sum = 0.0;
#pragma unroll
            for (int b = 0; b < (1 << D); b++) {
                int cx = vx + (b & 1);
                int cy = D > 1 ? vy + ((b >> 1) & 1) : 0;
                int cz = D > 2 ? vz + ((b >> 2) & 1) : 0;
                sum += sP[cx + CX * (cy + CY * cz)];
            }
            sV[r] = sum / (double)(1 << D);
        }
        __syncthreads();
        int li = threadIdx.x % TX, lj = (threadIdx.x / TX) % TY, lk = threadIdx.x / (TX * TY);
        int i = ox + li, j = oy + lj, k = oz + lk;
        if (i < g.n[0] && j < g.n[1] && k < g.n[2]) {
            int c = i + g.n[0] * (j + g.n[1] * k);
            auto V = [&](int a, int b2, int c2) { return sV[(li + a) + VX * ((lj + b2) + VY * (lk + c2))]; };
            int ii[3] = {i, j, k};
            double alo[3], ahi[3];
#pragma unroll
            for (int d = 0; d < D; d++) {
#pragma unroll
                for (int side = 0; side < 2; side++) {
                    int sx = d == 0 ? side : 0, sy = d == 1 ? side : 0, sz = d == 2 ? side : 0;
                    double A;
                    if (one_side) {
                        A = side_A;
                    } else if (D == 1) {
                        A = V(sx, 0, 0) < 0.0 ? 1.0 : 0.0;
                    } else if (D == 2) {
                        A = d == 0 ? edge_frac(V(sx, 0, 0), V(sx, 1, 0)) : edge_frac(V(0, sy, 0), V(1, sy, 0));
                    } else {
                        double v[4];
                        if (d == 0) { v[0] = V(sx, 0, 0); v[1] = V(sx, 1, 0); v[2] = V(sx, 1, 1); v[3] = V(sx, 0, 1); }
                        else if (d == 1) { v[0] = V(0, sy, 0); v[1] = V(1, sy, 0); v[2] = V(1, sy, 1); v[3] = V(0, sy, 1); }
                        else { v[0] = V(0, 0, sz); v[1] = V(1, 0, sz); v[2] = V(1, 1, sz); v[3] = V(0, 1, sz); }
                        A = clip_area(v);
                    }
                    if (side == 0) alo[d] = A; else ahi[d] = A;
                }
                g.ap[d][fidx(g, i, j, k)] = alo[d];
                if (ii[d] == g.n[d] - 1) g.ap[d][fidx(g, i + (d == 0), j + (d == 1), k + (d == 2))] = ahi[d];
            }
            double a;
            if (one_side && D <= 2) {
                a = side_A;
            } else if (D == 1) {
                a = edge_frac(V(0, 0, 0), V(1, 0, 0));
            } else if (D == 2) {
                double v[4] = {V(0, 0, 0), V(1, 0, 0), V(1, 1, 0), V(0, 1, 0)};
                a = clip_area(v);
            } else {
                double sumA = 0.0, g2 = 0.0;
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    sumA += alo[d] + ahi[d];
                    double gd = alo[d] - ahi[d];
                    g2 += gd * gd;
                }
                a = (0.5 * sumA + sqrt(g2) * (-sP[(li + 1) + CX * ((lj + 1) + CY * (lk + 1))] / g.h)) / 3.0;
                a = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
            }
            g.alpha[c] = a;
        }
        __syncthreads();
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_geom_lds(Dev g, int list, const double* cur, const double* tpm_cur)
{
    b_geom_lds<D>(VB::grid(), g, list, cur, tpm_cur);
}

// interface segment per unit volume of fluid 0 (points into fluid 1)
template <int D>
__device__ __forceinline__ double iface(const Dev& g, int i, int j, int k, double* gv)
{
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; d++) {
        gv[d] = (g.ap[d][fidx(g, i, j, k)] - g.ap[d][fidx(g, i + (d == 0), j + (d == 1), k + (d == 2))]) / g.h;
        g2 += gv[d] * gv[d];
    }
    return sqrt(g2);
}

__device__ __forceinline__ double alpha_k(const Dev& g, int k, int c)
{
    double a = g.alpha[c];
    return k == 0 ? a : 1.0 - a;
}

template <int D>
__device__ __forceinline__ double grad_phi(const Dev& g, const double* cur, int c, double* gr)
{
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; d++) {
        gr[d] = (phi_at(g, cur, nbr(g, c, d, 1)) - phi_at(g, cur, nbr(g, c, d, -1))) / (2.0 * g.h);
        g2 += gr[d] * gr[d];
    }
    return sqrt(g2);
}

// ---------------------------------------------------------------------------
// elementwise helpers over listed tiles
// ---------------------------------------------------------------------------
// dst = a1 * src1 + a2 * src2 on ncomp components
template <int D>
__device__ __forceinline__ void b_axpby(const VB blk, const Dev& g, int list, double a1, const double* s1, double a2,
                                        const double* s2, double* dst, int ncomp)
{
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, k;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, k)) continue;
        int c = i + g.n[0] * (j + g.n[1] * k);
        for (int q = 0; q < ncomp; q++) {
            size_t e = (size_t)q * g.nc + c;
            dst[e] = s2 ? a1 * s1[e] + a2 * s2[e] : s1[e];
        }
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_axpby(Dev g, int list, double a1, const double* s1, double a2,
                                                    const double* s2, double* dst, int ncomp)
{
    b_axpby<D>(VB::grid(), g, list, a1, s1, a2, s2, dst, ncomp);
}

// ---------------------------------------------------------------------------
// small-cell mixing (Sec. 2.2): increments in gather form
// ---------------------------------------------------------------------------
// A cell is a mixing source of fluid k when its volume fraction alpha_k is
// below alpha_mix, it lies within the source band (|phi| <= mix_band h) and
// the level-set gradient there is non-zero.  Its targets are the cells one
// step away along the normal into fluid k: on each axis the step has the
// sign of that normal component, and each non-empty subset of the axes gives
// one target, weighted |n_d|^2 (one axis), |n_a n_b| (two) or
// |n_x n_y n_z|^(2/3) (three), the weights normalised to sum to one.  The
// two fluids' normals are opposite, so the weights are the same for both;
// only the step signs and the source condition differ.

// Waves per SIMD the mixing kernels are compiled for (at most 128 VGPRs; the
// 3-D source table takes 36 KB of LDS, four blocks per CU).
#define SHARP_MIX_WAVES 4

// The region of a tile that mixing reads: the tile and its one-cell halo.
template <int D> struct MixRegion;
template <> struct MixRegion<1> { static constexpr int X = 256 + 2, Y = 1, Z = 1, N = X; };
template <> struct MixRegion<2> { static constexpr int X = 16 + 2, Y = 16 + 2, Z = 1, N = X * Y; };
template <> struct MixRegion<3> { static constexpr int X = 8 + 2, Y = 8 + 2, Z = 4 + 2, N = X * Y * Z; };

// tile t's origin and the cell of thread `tid` (local coordinates)
template <int D>
__device__ __forceinline__ void tile_origin(const Dev& g, int t, int& ox, int& oy, int& oz)
{
    ox = (t % g.nt[0]) * Tile<D>::X;
    oy = D >= 2 ? ((t / g.nt[0]) % g.nt[1]) * Tile<D>::Y : 0;
    oz = D == 3 ? (t / (g.nt[0] * g.nt[1])) * Tile<D>::Z : 0;
}

// The tile and two cells around it lie inside the grid: every cell the
// mixing of the tile reads (region cells, their level-set neighbours, the
// targets of region cells) is then found by index arithmetic, with no
// boundary images and no cell reached twice.
template <int D>
__device__ __forceinline__ bool mix_interior(const Dev& g, int ox, int oy, int oz)
{
    bool in = ox >= 2 && ox + Tile<D>::X + 2 <= g.n[0];
    if (D >= 2) in = in && oy >= 2 && oy + Tile<D>::Y + 2 <= g.n[1];
    if (D == 3) in = in && oz >= 2 && oz + Tile<D>::Z + 2 <= g.n[2];
    return in;
}

// Source-table code of a region cell: bit k set = source of fluid k; bit
// 2 + 3k + d set = fluid k's step on axis d is -1.
__device__ __forceinline__ int mix_step(int code, int k, int d)
{
    return (code >> (2 + 3 * k + d)) & 1 ? -1 : 1;
}

// Table entry of cell c for both fluids (0: a source of neither); the
// weights of its targets (subset m of the axes at m - 1) go to beta.
// phinb(d, o) is the level set at the neighbour o = +-1 along axis d.
template <int D, typename PhiNb>
__device__ __forceinline__ int mix_entry(const Dev& g, const double* cur, int c, PhiNb phinb, double* beta)
{
    constexpr int NS = (1 << D) - 1;
    const double a = g.alpha[c];
    const bool src0 = a < g.amix, src1 = 1.0 - a < g.amix;
    if (!(src0 || src1) || !(fabs(phi_at(g, cur, c)) <= g.mixb * g.h)) return 0;
    double gr[3];
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; d++) {
        gr[d] = (phinb(d, 1) - phinb(d, -1)) / (2.0 * g.h);
        g2 += gr[d] * gr[d];
    }
    const double gm = sqrt(g2);
    if (!(gm > 0.0)) return 0;
    int code = (src0 ? 1 : 0) | (src1 ? 2 : 0);
    double nrm[3];
#pragma unroll
    for (int d = 0; d < D; d++) {
        const double n0 = -1.0 * gr[d] / gm, n1 = 1.0 * gr[d] / gm;   // fluid 0 / fluid 1 normal
        nrm[d] = fabs(n0);
        if (n0 < 0.0) code |= 1 << (2 + d);
        if (n1 < 0.0) code |= 1 << (5 + d);
    }
    double bsum = 0.0;
    for (int m = 1; m <= NS; m++) {
        int cnt = 0;
        double prod = 1.0;
        for (int d = 0; d < D; d++)
            if (m & (1 << d)) { cnt++; prod *= nrm[d]; }
        // the three-axis weight |n_x n_y n_z|^(2/3) as a cube root of the square
        double b = cnt == 1 ? prod * prod : (cnt == 2 ? prod : cbrt(prod * prod));
        beta[m - 1] = b;
        bsum += b;
    }
    for (int m = 0; m < NS; m++) beta[m] /= bsum;
    return code;
}

// No cell of the tile's mixing region can be a source (|phi| > the source
// band at the last geometry, with two cells of margin for the level set's
// change since then: one stage's advection and reinitialisation move it by
// less than that), so the tile's mixing increments are all zero.  The
// geometry kernels record the per-tile minimum.
__device__ __forceinline__ bool mix_far(const Dev& g, int t)
{
    return g.tphimin[t] > (g.mixb + 2.0) * g.h;
}

// Source table of the tile's region for both fluids (cells outside the grid
// hold the entry of their boundary image): sCode per region cell, and the
// target weights of the sources at sBeta[(m - 1) * N + r].
template <int D>
__device__ __forceinline__ void mix_table(const Dev& g, int ox, int oy, int oz, bool interior, const double* cur,
                                          double* sBeta, int* sCode)
{
    constexpr int NS = (1 << D) - 1;
    constexpr int RX = MixRegion<D>::X, RY = MixRegion<D>::Y, RN = MixRegion<D>::N;
    constexpr int HY = D >= 2 ? 1 : 0, HZ = D == 3 ? 1 : 0;
    const int st[3] = {1, g.n[0], g.n[0] * g.n[1]};
    for (int r = threadIdx.x; r < RN; r += SHARP_WG) {
        const int rx = r % RX, ry = (r / RX) % RY, rz = r / (RX * RY);
        double beta[7];
        int code;
        if (interior) {
            const int c = (ox - 1 + rx) + st[1] * (oy - HY + ry) + st[2] * (oz - HZ + rz);
            code = mix_entry<D>(g, cur, c, [&](int d, int o) { return phi_at(g, cur, c + o * st[d]); }, beta);
        } else {
            const int c = cidx(g, ox - 1 + rx, oy - HY + ry, oz - HZ + rz);
            code = mix_entry<D>(g, cur, c, [&](int d, int o) { return phi_at(g, cur, nbr(g, c, d, o)); }, beta);
        }
        sCode[r] = code;
        if (code)
            for (int m = 0; m < NS; m++) sBeta[m * RN + r] = beta[m];
    }
}

// Mixing increment of fluid k at cell c (grid coordinates i, j, kk; local
// li, lj, lk in the tile) from the tile's source table: c as a source (its
// targets in subset order), then c as a target of each distinct neighbour
// (z, y, x order).  val(q, cell) gives the pre-mixing values.
template <int D, typename Val>
__device__ __forceinline__ void mix_gather(const Dev& g, int k, int c, int i, int j, int kk, int li, int lj, int lk,
                                           bool interior, const double* sBeta, const int* sCode, Val val,
                                           const double* vc, double* dl)
{
    constexpr int NV = D + 2;
    constexpr int NS = (1 << D) - 1;
    constexpr int RX = MixRegion<D>::X, RY = MixRegion<D>::Y, RN = MixRegion<D>::N;
    constexpr int HY = D >= 2 ? 1 : 0, HZ = D == 3 ? 1 : 0;
    const int rc = (li + 1) + RX * ((lj + HY) + RY * (lk + HZ));
    const int kbit = 1 << k;
    const int st[3] = {1, g.n[0], g.n[0] * g.n[1]};
    const double ac = alpha_k(g, k, c);
    const int cc = sCode[rc];
    if (cc & kbit) {
        int sx[3] = {1, 1, 1};
        for (int d = 0; d < D; d++) sx[d] = mix_step(cc, k, d);
        for (int m = 1; m <= NS; m++) {
            const double b = sBeta[(m - 1) * RN + rc];
            int tt;
            if (interior) {
                tt = c;
                for (int d = 0; d < D; d++)
                    if (m & (1 << d)) tt += sx[d] * st[d];
            } else {
                tt = cidx(g, i + ((m & 1) ? sx[0] : 0), j + ((m & 2) ? sx[1] : 0), kk + ((m & 4) ? sx[2] : 0));
            }
            if (!(b > 0.0) || tt == c) continue;
            const double at = alpha_k(g, k, tt);
            if (!(ac + at > 0.0)) continue;
            for (int q = 0; q < NV; q++) dl[q] += b * (val(q, tt) * ac - vc[q] * at) / (ac + at);
        }
    }
    // c as a target: first the mask of neighbours that may reach it (bit
    // (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1) for offset o, so that ascending
    // bits follow z, y, x order), then their contributions in that order.
    const int pos[3] = {i, j, kk};
    int mm[3][3];     // boundary image of c's coordinate + o on each axis
    unsigned mask = 0;
    if (interior) {
        // a neighbour at offset o reaches c through one subset only (the
        // axes where o is non-zero), and only if it steps by -o on each
#pragma unroll
        for (int oz2 = -HZ; oz2 <= HZ; oz2++)
#pragma unroll
            for (int oy2 = -HY; oy2 <= HY; oy2++)
#pragma unroll
                for (int ox2 = -1; ox2 <= 1; ox2++) {
                    if (!ox2 && !oy2 && !oz2) continue;
                    const int code = sCode[rc + ox2 + RX * (oy2 + RY * oz2)];
                    bool hit = (code & kbit) != 0;
                    if (ox2) hit = hit && (mix_step(code, k, 0) == -ox2);
                    if (oy2) hit = hit && (mix_step(code, k, 1) == -oy2);
                    if (oz2) hit = hit && (mix_step(code, k, 2) == -oz2);
                    if (hit) mask |= 1u << ((oz2 + 1) * 9 + (oy2 + 1) * 3 + (ox2 + 1));
                }
    } else {
        // near the grid boundary neighbours are boundary images: a cell
        // reached at several offsets counts once (at the first in z, y, x
        // order) and c itself not at all.  The boundary maps act per axis,
        // so offset o repeats an earlier one exactly when on some axis a
        // smaller offset has the same image, and is c when every axis is.
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int o = -1; o <= 1; o++)
                mm[d][o + 1] = d < D ? bcmap(pos[d] + o, g.n[d], g.bc[d]) : pos[d];
#pragma unroll 1
        for (int oz2 = -HZ; oz2 <= HZ; oz2++)
#pragma unroll 1
            for (int oy2 = -HY; oy2 <= HY; oy2++)
#pragma unroll 1
                for (int ox2 = -1; ox2 <= 1; ox2++) {
                    if (!ox2 && !oy2 && !oz2) continue;
                    const int off[3] = {ox2, oy2, oz2};
                    bool self = true, repeat = false;
#pragma unroll
                    for (int d = 0; d < D; d++) {
                        self = self && mm[d][off[d] + 1] == mm[d][1];
                        for (int o = -1; o < off[d]; o++) repeat = repeat || mm[d][o + 1] == mm[d][off[d] + 1];
                    }
                    if (self || repeat) continue;
                    if (sCode[rc + ox2 + RX * (oy2 + RY * oz2)] & kbit)
                        mask |= 1u << ((oz2 + 1) * 9 + (oy2 + 1) * 3 + (ox2 + 1));
                }
    }
    while (mask) {
        const int e = __builtin_ctz(mask);
        mask &= mask - 1;
        const int ox2 = e % 3 - 1, oy2 = (e / 3) % 3 - 1, oz2 = e / 9 - 1;
        const int rs = rc + ox2 + RX * (oy2 + RY * oz2);
        int sc;
        unsigned msub;   // bit m - 1: subset m of the neighbour's targets reaches c
        if (interior) {
            sc = c + ox2 * st[0] + oy2 * st[1] + oz2 * st[2];
            msub = 1u << (((ox2 ? 1 : 0) | (oy2 ? 2 : 0) | (oz2 ? 4 : 0)) - 1);
        } else {
            const int code = sCode[rs];
            const int off[3] = {ox2, oy2, oz2};
            int sp[3] = {0, 0, 0};
            int onto = 0, held = 0;   // axes that step onto / already hold c's coordinate
            for (int d = 0; d < D; d++) {
                sp[d] = mm[d][off[d] + 1];
                if (bcmap(sp[d] + mix_step(code, k, d), g.n[d], g.bc[d]) == pos[d]) onto |= 1 << d;
                if (sp[d] == pos[d]) held |= 1 << d;
            }
            sc = sp[0] + g.n[0] * (sp[1] + g.n[1] * sp[2]);
            msub = 0;
            for (int m = 1; m <= NS; m++)
                if (((onto & m) | (held & ~m & NS)) == NS) msub |= 1u << (m - 1);
        }
        const double as = alpha_k(g, k, sc);
        if (!(as + ac > 0.0)) continue;
        while (msub) {
            const int m = __builtin_ctz(msub) + 1;
            msub &= msub - 1;
            const double b = sBeta[(m - 1) * RN + rs];
            if (!(b > 0.0)) continue;
            for (int q = 0; q < NV; q++) dl[q] -= b * (vc[q] * as - val(q, sc) * ac) / (as + ac);
        }
    }
}

template <int D>
__device__ __forceinline__ void b_mixdelta_lds(const VB blk, const Dev& g, int list, int k, const double* cons,
                                               const double* cur)
{
    constexpr int NV = D + 2;
    constexpr int NS = (1 << D) - 1;
    constexpr int TX = Tile<D>::X, TY = Tile<D>::Y;
    constexpr int RN = MixRegion<D>::N;
    __shared__ double sBeta[NS * RN];
    __shared__ int sCode[RN];
    const int* L = list_ptr(g, list);
    auto val = [&](int q, int c) { return cons[(size_t)q * g.nc + c]; };
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int ox, oy, oz;
        tile_origin<D>(g, L[ti], ox, oy, oz);
        const bool far = mix_far(g, L[ti]);
        const bool interior = mix_interior<D>(g, ox, oy, oz);
        if (!far) mix_table<D>(g, ox, oy, oz, interior, cur, sBeta, sCode);
        __syncthreads();
        int li = threadIdx.x % TX, lj = (threadIdx.x / TX) % TY, lk = threadIdx.x / (TX * TY);
        int i = ox + li, j = oy + lj, kk = oz + lk;
        if (i < g.n[0] && j < g.n[1] && kk < g.n[2]) {
            int c = i + g.n[0] * (j + g.n[1] * kk);
            if (g.M[c]) {
                double vc[NV], dl[NV];
                for (int q = 0; q < NV; q++) { vc[q] = val(q, c); dl[q] = 0.0; }
                if (!far) mix_gather<D>(g, k, c, i, j, kk, li, lj, lk, interior, sBeta, sCode, val, vc, dl);
                for (int q = 0; q < NV; q++) g.dmix[(size_t)q * g.nc + c] = dl[q];
            }
        }
        __syncthreads();
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG, SHARP_MIX_WAVES) k_mixdelta_lds(Dev g, int list, int k, const double* cons,
                                                           const double* cur)
{
    b_mixdelta_lds<D>(VB::grid(), g, list, k, cons, cur);
}

// Mixed copy of one tile: dst = v + mixing increment of v, where
// v = a1*s1 + a2*s2 (s2 may be null: v = s1) is formed on the fly from
// inputs that are only read, so one pass suffices (the increments use
// pre-mixing values).  Used for the slow fluid's temporary state (Eq.
// interpolation, then mixing with the current geometry) and for the mixing
// of a stage output written out of place.
struct MixPart {
    int k;                // fluid
    double a1;
    const double* s1;
    double a2;
    const double* s2;
    double* dst;
    int do_mix;
    int sched_theta;      // interpolation weight from the device plan: a1 = 1 - th, a2 = th
};

// the part's weights and whether it mixes (a plan-given weight of zero
// leaves the state unmixed)
__device__ __forceinline__ int mix_weights(const Dev& g, const MixPart& P, double& a1, double& a2)
{
    a1 = P.a1;
    a2 = P.a2;
    int do_mix = P.do_mix;
    if (P.sched_theta) {
        double th = g.sched[SCHED_TH1];
        a1 = 1.0 - th;
        a2 = th;
        do_mix = th != 0.0;
    }
    return do_mix;
}

// the part's cells of the tile, from a table built for the tile (when it mixes)
template <int D>
__device__ __forceinline__ void mix_write(const Dev& g, const MixPart& P, double a1, double a2, bool do_mix, int ox,
                                          int oy, int oz, bool interior, const double* sBeta, const int* sCode)
{
    constexpr int NV = D + 2;
    constexpr int TX = Tile<D>::X, TY = Tile<D>::Y;
    const double* s1 = P.s1;
    const double* s2 = P.s2;
    auto val = [&](int q, int c) {
        size_t e = (size_t)q * g.nc + c;
        return s2 ? a1 * s1[e] + a2 * s2[e] : s1[e];
    };
    int li = threadIdx.x % TX, lj = (threadIdx.x / TX) % TY, lk = threadIdx.x / (TX * TY);
    int i = ox + li, j = oy + lj, kk = oz + lk;
    if (i < g.n[0] && j < g.n[1] && kk < g.n[2]) {
        int c = i + g.n[0] * (j + g.n[1] * kk);
        double vc[NV], dl[NV];
        for (int q = 0; q < NV; q++) { vc[q] = val(q, c); dl[q] = 0.0; }
        if (do_mix && g.M[c])
            mix_gather<D>(g, P.k, c, i, j, kk, li, lj, lk, interior, sBeta, sCode, val, vc, dl);
        for (int q = 0; q < NV; q++) P.dst[(size_t)q * g.nc + c] = vc[q] + dl[q];
    }
}

// Several mixed copies of the same tiles in one launch (the parts read no
// buffer another part writes; one source table per tile serves every part),
// and optionally phi_dst = phi_src on the band-mask cells (the mixing reads
// the level set through phi_src).
template <int D>
__device__ __forceinline__ void mix_parts_tiles(const VB blk, const Dev& g, int list, const MixPart& A,
                                                const MixPart& B, int nparts, const double* cur,
                                                const double* phi_src, double* phi_dst)
{
    constexpr int NS = (1 << D) - 1;
    constexpr int TX = Tile<D>::X, TY = Tile<D>::Y;
    constexpr int RN = MixRegion<D>::N;
    __shared__ double sBeta[NS * RN];
    __shared__ int sCode[RN];
    double aA1, aA2, aB1 = 0.0, aB2 = 0.0;
    const int mixA = mix_weights(g, A, aA1, aA2);
    const int mixB = nparts > 1 ? mix_weights(g, B, aB1, aB2) : 0;
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        const int t = L[ti];
        int ox, oy, oz;
        tile_origin<D>(g, t, ox, oy, oz);
        const bool far = mix_far(g, t);
        const bool doA = mixA && !far, doB = mixB && !far;
        const bool interior = mix_interior<D>(g, ox, oy, oz);
        if (doA || doB) mix_table<D>(g, ox, oy, oz, interior, cur, sBeta, sCode);
        __syncthreads();
        mix_write<D>(g, A, aA1, aA2, doA, ox, oy, oz, interior, sBeta, sCode);
        if (nparts > 1) mix_write<D>(g, B, aB1, aB2, doB, ox, oy, oz, interior, sBeta, sCode);
        if (phi_dst) {
            int tid = threadIdx.x;
            int i = ox + tid % TX, j = oy + (tid / TX) % TY, kk = oz + tid / (TX * TY);
            if (i < g.n[0] && j < g.n[1] && kk < g.n[2]) {
                int c = i + g.n[0] * (j + g.n[1] * kk);
                if (g.M[c]) phi_dst[c] = phi_src[c];
            }
        }
        __syncthreads();
    }
}

template <int D>
__device__ __forceinline__ void b_mixinterp_lds(const VB blk, const Dev& g, int list, MixPart P, const double* cur)
{
    mix_parts_tiles<D>(blk, g, list, P, P, 1, cur, nullptr, nullptr);
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG, SHARP_MIX_WAVES) k_mixinterp_lds(Dev g, int list, MixPart P, const double* cur)
{
    b_mixinterp_lds<D>(VB::grid(), g, list, P, cur);
}

template <int D>
__device__ __forceinline__ void b_mix_parts(const VB blk, const Dev& g, int list, MixPart A, MixPart B, int nparts,
                                            const double* cur, const double* phi_src, double* phi_dst)
{
    mix_parts_tiles<D>(blk, g, list, A, B, nparts, cur, phi_src, phi_dst);
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG, SHARP_MIX_WAVES) k_mix_parts(Dev g, int list, MixPart A, MixPart B, int nparts,
                                                        const double* cur, const double* phi_src, double* phi_dst)
{
    b_mix_parts<D>(VB::grid(), g, list, A, B, nparts, cur, phi_src, phi_dst);
}

template <int D>
__device__ __forceinline__ void b_mixapply(const VB blk, const Dev& g, int list, double* cons)
{
    constexpr int NV = D + 2;
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, k;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, k)) continue;
        int c = i + g.n[0] * (j + g.n[1] * k);
        if (!g.M[c]) continue;
        for (int q = 0; q < NV; q++) cons[(size_t)q * g.nc + c] += g.dmix[(size_t)q * g.nc + c];
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_mixapply(Dev g, int list, double* cons)
{
    b_mixapply<D>(VB::grid(), g, list, cons);
}

// ---------------------------------------------------------------------------
// primitive recovery on real band cells (alpha_k >= alpha_mix), both fluids
// in one launch (fluid 0 from src0, fluid 1 from src1)
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void b_prims(const VB blk, const Dev& g, int list, const double* src0,
                                        const double* src1, int wb)
{
    constexpr int NV = D + 2;
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        if (!g.M[c]) continue;
        for (int k = 0; k < 2; k++) {
            const double* src = k == 0 ? src0 : src1;
            double* W = g.Wb[k][wb];
            double a = alpha_k(g, k, c);
            if (a < g.amix) continue;
            double U[NV], w[NV];
            for (int q = 0; q < NV; q++) U[q] = src[(size_t)q * g.nc + c] / a;
            if (!cons2prim<D>(g.gam[k], g.pinf[k], U, w)) flag_nonphys(g, c, k);
            for (int q = 0; q < NV; q++) W[(size_t)q * g.nc + c] = w[q];
        }
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_prims(Dev g, int list, const double* src0, const double* src1, int wb)
{
    b_prims<D>(VB::grid(), g, list, src0, src1, wb);
}

// ---------------------------------------------------------------------------
// 3-D extension stencil lists.  The first sweep of an extension records each
// target (cell, for the primitives also the fluid) with its upwind
// neighbours and weights; the sweeps after it only redo the weighted average
// over the list, with the same arithmetic as the full sweep.  The targets and
// stencils depend on the geometry and the level set only, which do not
// change between the sweeps of one extension.  Each wave of a tile writes
// its targets to slots of its own, ranked by a ballot, and its count; no
// atomics, and the layout does not depend on timing.
// ---------------------------------------------------------------------------
constexpr int WL_WAVE = 128;   // primitive targets per wave: 64 cells x 2 fluids
constexpr int VL_WAVE = 64;

__device__ __forceinline__ void xl_put(int cap, int* lc, int* lup, double* lw, size_t e, int code, const int* up,
                                       const double* w, double wsum)
{
    lc[e] = code;
    for (int d = 0; d < 3; d++) {
        lup[(size_t)d * cap + e] = up[d];
        lw[(size_t)d * cap + e] = w[d];
    }
    lw[(size_t)3 * cap + e] = wsum;
}

// later sweeps of the primitive extension (3-D): both fluids from the list
__device__ __forceinline__ void b_extw_list(const VB blk, const Dev& g, int in, int out)
{
    constexpr int NV = 5;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int ti = blk.b; ti < list_count(g, LIST_INNER); ti += blk.n) {
        const int n = g.wl_n[4 * ti + wv];
        const size_t base = (size_t)(4 * ti + wv) * WL_WAVE;
        for (int r = lane; r < n; r += 64) {
            const size_t e = base + r;
            const int code = g.wl_c[e];
            const int c = code & 0x7fffffff, k = (int)((unsigned)code >> 31);
            const double* Wi = g.Wb[k][in];
            double* Wo = g.Wb[k][out];
            int up[3];
            double w[3];
            for (int d = 0; d < 3; d++) {
                up[d] = g.wl_up[(size_t)d * g.wl_cap + e];
                w[d] = g.wl_w[(size_t)d * g.wl_cap + e];
            }
            const double wsum = g.wl_w[(size_t)3 * g.wl_cap + e];
            for (int q = 0; q < NV; q++) {
                double acc = 0.0;
                for (int d = 0; d < 3; d++) acc += w[d] * Wi[(size_t)q * g.nc + up[d]];
                Wo[(size_t)q * g.nc + c] = acc / wsum;
            }
        }
    }
}
__global__ void __launch_bounds__(SHARP_WG) k_extw_list(Dev g, int in, int out)
{
    b_extw_list(VB::grid(), g, in, out);
}

// later sweeps of the velocity extension (3-D)
__device__ __forceinline__ void b_extv_list(const VB blk, const Dev& g, int in, int out)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int ti = blk.b; ti < list_count(g, LIST_INNER); ti += blk.n) {
        const int n = g.vl_n[4 * ti + wv];
        const size_t base = (size_t)(4 * ti + wv) * VL_WAVE;
        for (int r = lane; r < n; r += 64) {
            const size_t e = base + r;
            const int c = g.vl_c[e];
            int up[3];
            double w[3];
            for (int d = 0; d < 3; d++) {
                up[d] = g.vl_up[(size_t)d * g.vl_cap + e];
                w[d] = g.vl_w[(size_t)d * g.vl_cap + e];
            }
            const double wsum = g.vl_w[(size_t)3 * g.vl_cap + e];
            for (int q = 0; q < 3; q++) {
                double acc = 0.0;
                for (int d = 0; d < 3; d++) acc += w[d] * g.v[in][q][up[d]];
                g.v[out][q][c] = acc / wsum;
            }
        }
    }
}
__global__ void __launch_bounds__(SHARP_WG) k_extv_list(Dev g, int in, int out)
{
    b_extv_list(VB::grid(), g, in, out);
}

// ---------------------------------------------------------------------------
// extension: one Jacobi sweep of the upwind steady state of
// dq/dtau + n.grad q = 0 for both fluids' primitives
// ---------------------------------------------------------------------------
// copy: also copy the cells that are not extended (only the first sweep of a
// call needs to: afterwards both Jacobi buffers hold the same values there)
template <int D>
__device__ __forceinline__ void b_extw(const VB blk, const Dev& g, int list, int in, int out, const double* cur,
                                       int copy)
{
    constexpr int NV = D + 2;
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        // 3-D, after the first sweep: a tile beyond the extension depth (two
        // cells of margin, as for mixing) holds no target
        if (D == 3 && !copy && g.tphimin[L[ti]] > (g.extb + 2.0) * g.h) continue;
        // recording (3-D first sweep): this wave's slots and running count;
        // every wave of the tile writes its count, zero included
        const bool record = D == 3 && copy && list == LIST_INNER;
        int i, j, kk;
        const bool inside = tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk);
        const int c = inside ? i + g.n[0] * (j + g.n[1] * kk) : 0;
        const bool act = inside && g.M[c];
        if (!act && !record) continue;
        double ph = act ? phi_at(g, cur, c) : 0.0;
        double gr[3];
        double gm = -1.0;
        const int lane = threadIdx.x & 63;
        const size_t wbase = (size_t)(4 * ti + (threadIdx.x >> 6)) * WL_WAVE;
        int off = 0;
        for (int k = 0; k < 2; k++) {
            const double* Wi = g.Wb[k][in];
            double* Wo = g.Wb[k][out];
            double sk = k == 0 ? 1.0 : -1.0;
            bool target = act && alpha_k(g, k, c) < g.amix && !(sk * ph > g.extb * g.h);
            if (target && gm < 0.0) gm = grad_phi<D>(g, cur, c, gr);
            int slot = 0;
            if (record) {
                const unsigned long long mk = __ballot(target && gm > 0.0);
                slot = off + __popcll(mk & ((1ull << lane) - 1ull));
                off += __popcll(mk);
            }
            if (!target || !(gm > 0.0)) {
                if (copy && act)
                    for (int q = 0; q < NV; q++) Wo[(size_t)q * g.nc + c] = Wi[(size_t)q * g.nc + c];
                continue;
            }
            int up[3];
            double w[3], wsum = 0.0;
            for (int d = 0; d < D; d++) {
                double nd = sk * gr[d] / gm;
                up[d] = nbr(g, c, d, nd > 0.0 ? -1 : 1);
                w[d] = fabs(nd);
                wsum += w[d];
            }
            for (int q = 0; q < NV; q++) {
                double acc = 0.0;
                for (int d = 0; d < D; d++) acc += w[d] * Wi[(size_t)q * g.nc + up[d]];
                Wo[(size_t)q * g.nc + c] = acc / wsum;
            }
            if (record)
                xl_put(g.wl_cap, g.wl_c, g.wl_up, g.wl_w, wbase + slot, (int)((unsigned)c | ((unsigned)k << 31)), up,
                       w, wsum);
        }
        if (record && lane == 0) g.wl_n[4 * ti + (threadIdx.x >> 6)] = off;
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_extw(Dev g, int list, int in, int out, const double* cur, int copy)
{
    b_extw<D>(VB::grid(), g, list, in, out, cur, copy);
}

// level-set velocity: from the cut cells to the rest of the band
template <int D>
__device__ __forceinline__ void b_extv(const VB blk, const Dev& g, int list, int in, int out, const double* cur,
                                       int copy)
{
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        // recording (3-D first sweep): this wave's slots and count; every
        // wave of the tile writes its count, zero included
        const bool record = D == 3 && copy && list == LIST_INNER;
        int i, j, kk;
        const bool inside = tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk);
        const int c = inside ? i + g.n[0] * (j + g.n[1] * kk) : 0;
        const bool act = inside && g.M[c];
        if (!act && !record) continue;
        double gv[3];
        const bool cut = act ? iface<D>(g, i, j, kk, gv) > 0.0 : true;
        double gr[3];
        double gm = cut ? 0.0 : grad_phi<D>(g, cur, c, gr);
        int slot = 0;
        if (record) {
            const int lane = threadIdx.x & 63;
            const unsigned long long mk = __ballot(!cut && gm > 0.0);
            slot = __popcll(mk & ((1ull << lane) - 1ull));
            if (lane == 0) g.vl_n[4 * ti + (threadIdx.x >> 6)] = __popcll(mk);
        }
        if (cut || !(gm > 0.0)) {
            if (copy && act)
                for (int e = 0; e < D; e++) g.v[out][e][c] = g.v[in][e][c];
            continue;
        }
        double sg = phi_at(g, cur, c) < 0.0 ? -1.0 : 1.0;
        int up[3];
        double w[3], wsum = 0.0;
        for (int d = 0; d < D; d++) {
            double nd = sg * gr[d] / gm;
            up[d] = nbr(g, c, d, nd > 0.0 ? -1 : 1);
            w[d] = fabs(nd);
            wsum += w[d];
        }
        for (int e = 0; e < D; e++) {
            double acc = 0.0;
            for (int d = 0; d < D; d++) acc += w[d] * g.v[in][e][up[d]];
            g.v[out][e][c] = acc / wsum;
        }
        if (record) xl_put(g.vl_cap, g.vl_c, g.vl_up, g.vl_w, (size_t)(4 * ti + (threadIdx.x >> 6)) * VL_WAVE + slot, c,
                           up, w, wsum);
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_extv(Dev g, int list, int in, int out, const double* cur, int copy)
{
    b_extv<D>(VB::grid(), g, list, in, out, cur, copy);
}

// ---------------------------------------------------------------------------
// Temporally blocked extension (1-D and 2-D): the tile and a halo of EXT_H
// cells are staged in LDS and all Jacobi sweeps run there; a cell at depth e
// inside the halo is exact for e sweeps, so the tile itself is exact after up
// to EXT_H sweeps.  Same arithmetic as k_prims followed by k_extw / k_extv.
// ---------------------------------------------------------------------------
constexpr int EXT_H = 8;
template <int D> struct ExtRegion;
template <> struct ExtRegion<1> { static constexpr int X = 256 + 2 * EXT_H, Y = 1; };
template <> struct ExtRegion<2> { static constexpr int X = 16 + 2 * EXT_H, Y = 16 + 2 * EXT_H; };

// block sizes of the temporally blocked kernels: one thread per region cell
// (2-D), one per tile cell (1-D)
template <int D> struct ExtWG;
template <> struct ExtWG<1> { static constexpr int W = 256, V = 256; };
template <> struct ExtWG<2> { static constexpr int W = 1024, V = 1024; };

// Region position whose stencil a region position evaluates: along a
// zero-gradient direction the cells beyond the wall read the wall cell, so a
// position there repeats the wall cell's update (o: global coordinate of
// region position 0, x: global coordinate of the position).  Periodic
// directions wrap, which commutes with the stencils, so positions stay.
__device__ __forceinline__ int src_pos(const Dev& g, int d, int o, int x)
{
    if (g.bc[d] == 0) x = x < 0 ? 0 : (x >= g.n[d] ? g.n[d] - 1 : x);
    return x - o;
}

// fused primitive recovery (real band cells) + extension of one fluid's
// primitives per block (block b handles tile b/2, fluid b%2); reads
// Wb[k][in], writes the band cells of Wb[k][out]
// (at most 64 VGPRs, so that two 1024-thread blocks share a CU)
template <int D>
__device__ __forceinline__ void b_extw_tb(const VB blk, const Dev& g, int list, const double* src0, const double* src1,
                                          int in, int out, int iters, const double* cur)
{
    static_assert(D <= 2, "temporally blocked extension is for 1-D and 2-D");
    constexpr int NV = D + 2;
    constexpr int WGS = ExtWG<D>::W;
    constexpr int TX = Tile<D>::X, TY = Tile<D>::Y;
    constexpr int RX = ExtRegion<D>::X, RY = ExtRegion<D>::Y, RN = RX * RY;
    constexpr int PX = RX + 2, PY = D == 2 ? RY + 2 : 1, PN = PX * PY;   // level set with one more cell
    constexpr int CPT = (RN + WGS - 1) / WGS;
    constexpr int HY = D == 2 ? EXT_H : 0;
    __shared__ double sA[NV * RN], sB[NV * RN];
    __shared__ double sPhi[PN];
    const int* L = list_ptr(g, list);
    for (int wi = blk.b; wi < 2 * list_count(g, list); wi += blk.n) {
        int t = L[wi >> 1], k = wi & 1;
        int ox = (t % g.nt[0]) * TX, oy = D == 2 ? ((t / g.nt[0]) % g.nt[1]) * TY : 0;
        const double* src = k == 0 ? src0 : src1;
        const double* Wi = g.Wb[k][in];
        double sk = k == 0 ? 1.0 : -1.0;
        for (int r = threadIdx.x; r < PN; r += WGS) {
            int px = r % PX, py = r / PX;
            sPhi[r] = phi_at(g, cur, cidx(g, ox - EXT_H - 1 + px, D == 2 ? oy - HY - 1 + py : 0, 0));
        }
        __syncthreads();
        bool tgt[CPT];
        int up[CPT][2];
        double w[CPT][2];
#pragma unroll
        for (int m = 0; m < CPT; m++) {
            int r = threadIdx.x + m * WGS;
            tgt[m] = false;
            if (r >= RN) continue;
            int rx = r % RX, ry = r / RX;
            int c = cidx(g, ox - EXT_H + rx, oy - HY + ry, 0);
            int sx = src_pos(g, 0, ox - EXT_H, ox - EXT_H + rx), sy = D == 2 ? src_pos(g, 1, oy - HY, oy - HY + ry) : 0;
            double a = alpha_k(g, k, c);
            bool inM = g.M[c] != 0;
            if (inM && a >= g.amix) {
                double U[NV], W[NV];
                for (int q = 0; q < NV; q++) U[q] = src[(size_t)q * g.nc + c] / a;
                if (!cons2prim<D>(g.gam[k], g.pinf[k], U, W)) flag_nonphys(g, c, k);
                for (int q = 0; q < NV; q++) sA[q * RN + r] = W[q];
            } else {
                for (int q = 0; q < NV; q++) sA[q * RN + r] = Wi[(size_t)q * g.nc + c];
            }
            int pc = (sx + 1) + PX * (D == 2 ? sy + 1 : 0);
            if (!inM || !(a < g.amix) || sk * sPhi[pc] > g.extb * g.h) continue;
            double gr[2], g2 = 0.0;
            gr[0] = (sPhi[pc + 1] - sPhi[pc - 1]) / (2.0 * g.h);
            g2 += gr[0] * gr[0];
            if (D == 2) {
                gr[1] = (sPhi[pc + PX] - sPhi[pc - PX]) / (2.0 * g.h);
                g2 += gr[1] * gr[1];
            }
            double gm = sqrt(g2);
            if (!(gm > 0.0)) continue;
            bool inside = true;
            double wsum = 0.0;
            for (int d = 0; d < D; d++) {
                double nd = sk * gr[d] / gm;
                int o = nd > 0.0 ? -1 : 1;
                int qx = sx + (d == 0 ? o : 0), qy = sy + (d == 1 ? o : 0);
                inside &= qx >= 0 && qx < RX && qy >= 0 && qy < RY;
                up[m][d] = qx + RX * qy;
                w[m][d] = fabs(nd);
                wsum += w[m][d];
            }
            double iw = 1.0 / wsum;
            for (int d = 0; d < D; d++) w[m][d] *= iw;
            tgt[m] = inside;   // cells whose upwind stencil leaves the region stay frozen
        }
        __syncthreads();
        double* A = sA;
        double* B = sB;
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int m = 0; m < CPT; m++) {
                int r = threadIdx.x + m * WGS;
                if (r >= RN) continue;
                for (int q = 0; q < NV; q++) {
                    double v;
                    if (tgt[m]) {
                        v = w[m][0] * A[q * RN + up[m][0]];
                        if (D == 2) v += w[m][1] * A[q * RN + up[m][1]];
                    } else {
                        v = A[q * RN + r];
                    }
                    B[q * RN + r] = v;
                }
            }
            __syncthreads();
            double* tmp = A; A = B; B = tmp;
        }
        for (int u = threadIdx.x; u < TX * TY; u += WGS) {
            int li = u % TX, lj = u / TX;
            int i = ox + li, j = oy + lj;
            if (i < g.n[0] && j < g.n[1]) {
                int c = i + g.n[0] * j;
                if (g.M[c]) {
                    int r = (li + EXT_H) + RX * (lj + HY);
                    for (int q = 0; q < NV; q++) g.Wb[k][out][(size_t)q * g.nc + c] = A[q * RN + r];
                }
            }
        }
        __syncthreads();
    }
}
template <int D>
__global__ void __launch_bounds__(ExtWG<D>::W, 2 * ExtWG<D>::W / 256) k_extw_tb(Dev g, int list, const double* src0,
                                                                                const double* src1, int in, int out,
                                                                                int iters, const double* cur)
{
    b_extw_tb<D>(VB::grid(), g, list, src0, src1, in, out, iters, cur);
}

// Riemann problem of cut cell c with fluid states from Wb[.][wb], started
// from the cell's previous p*: st = {p*, u*, rho*_0, rho*_1}.  With the
// Laplace jump p*_0 - p*_1 = jump, fluid 1's wave curve at p - jump is that
// of the same state with (p, p_inf) shifted by (+jump, -jump) (a stiffened
// gas's wave curves see p only through p + p_inf and p - p_k), so the plain
// solver takes the shifted side and p* is fluid 0's contact pressure.
template <int D>
__device__ __forceinline__ void interface_solve(const Dev& g, int c, const double* gv, double gm, int wb, double* st,
                                                double jump = 0.0)
{
    const double p0 = g.ps[c];
    const double* W0 = g.Wb[0][wb];
    const double* W1 = g.Wb[1][wb];
    double un0 = 0.0, un1 = 0.0;
    for (int d = 0; d < D; d++) {
        un0 += W0[(size_t)(1 + d) * g.nc + c] * gv[d] / gm;
        un1 += W1[(size_t)(1 + d) * g.nc + c] * gv[d] / gm;
    }
    Side Ls = {W0[c], un0, W0[(size_t)(D + 1) * g.nc + c], g.gam[0], g.pinf[0]};
    Side Rs = {W1[c], un1, W1[(size_t)(D + 1) * g.nc + c] + jump, g.gam[1], g.pinf[1] - jump};
    riemann(Ls, Rs, p0, st);
}

// store the interface solution of the tile's own cut cell c (and book the
// correction at the slow fluid's own interface pressure); non-cut cells get
// zeros
template <int D>
__device__ __forceinline__ void interface_store(const Dev& g, int c, const double* gv, double gm, const double* st,
                                                double wcorr, int S, double jump = 0.0)
{
    if (g.pj) g.pj[c] = gm > 0.0 ? jump : 0.0;
    if (!(gm > 0.0)) {
        g.ps[c] = 0.0; g.us[c] = 0.0; g.ss[0][c] = 0.0; g.ss[1][c] = 0.0;
        return;
    }
    g.ps[c] = st[0];
    g.us[c] = st[1];
    for (int k = 0; k < 2; k++) {
        double rs = st[2 + k];
        double cs = rs > 0.0 ? csound(g.gam[k], g.pinf[k], rs, k == 0 ? st[0] : st[0] - jump) : 0.0;
        double sum = 0.0;
        for (int d = 0; d < D; d++) sum += (fabs(st[1] * gv[d] / gm) + cs) / g.h;
        g.ss[k][c] = sum;
    }
    if (wcorr != 0.0) {
        double sg = S == 0 ? 1.0 : -1.0, pS = S == 0 ? st[0] : st[0] - jump;
        for (int d = 0; d < D; d++) g.corr[(size_t)(1 + d) * g.nc + c] += wcorr * (-sg * pS * gv[d]);
        g.corr[(size_t)(D + 1) * g.nc + c] += wcorr * (-sg * pS * st[1] * gm);
    }
}

// interface interaction of the tile's own band-mask cells: every cut cell
// solves its Riemann problem once and stores p*, u*, the star-state speeds,
// the correction share, and u* n as the source of the velocity extension;
// the other band-mask cells get zeros
template <int D>
__device__ __forceinline__ void b_riemann(const VB blk, const Dev& g, int list, int wb, int vb, double wcorr, int S,
                                          const double* cur)
{
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        if (!g.M[c]) continue;   // a cut cell is a band-mask cell
        double gv[3];
        double gm = iface<D>(g, i, j, kk, gv);
        if (!(gm > 0.0)) {
            interface_store<D>(g, c, gv, gm, nullptr, 0.0, S);
            continue;
        }
        double st[4];
        const double jump = g.pj ? laplace_jump<D>(g, cur, i, j, kk) : 0.0;
        interface_solve<D>(g, c, gv, gm, wb, st, jump);
        interface_store<D>(g, c, gv, gm, st, wcorr, S, jump);
        for (int e = 0; e < D; e++) g.v[vb][e][c] = st[1] * gv[e] / gm;
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_riemann(Dev g, int list, int wb, int vb, double wcorr, int S,
                                                      const double* cur)
{
    b_riemann<D>(VB::grid(), g, list, wb, vb, wcorr, S, cur);
}

// level-set velocity extension, temporally blocked: u* n of the cut cells
// (from k_riemann, in v[in]) is extended over the tile's region in LDS
template <int D>
__device__ __forceinline__ void b_vext_tb(const VB blk, const Dev& g, int list, int in, int out, int iters,
                                          const double* cur)
{
    static_assert(D <= 2, "temporally blocked extension is for 1-D and 2-D");
    constexpr int WGS = ExtWG<D>::V;
    constexpr int TX = Tile<D>::X, TY = Tile<D>::Y;
    constexpr int RX = ExtRegion<D>::X, RY = ExtRegion<D>::Y, RN = RX * RY;
    constexpr int PX = RX + 2, PY = D == 2 ? RY + 2 : 1, PN = PX * PY;
    constexpr int CPT = (RN + WGS - 1) / WGS;
    constexpr int HY = D == 2 ? EXT_H : 0;
    __shared__ double sA[D * RN], sB[D * RN];
    __shared__ double sPhi[PN];
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int t = L[ti];
        int ox = (t % g.nt[0]) * TX, oy = D == 2 ? ((t / g.nt[0]) % g.nt[1]) * TY : 0;
        for (int r = threadIdx.x; r < PN; r += WGS) {
            int px = r % PX, py = r / PX;
            sPhi[r] = phi_at(g, cur, cidx(g, ox - EXT_H - 1 + px, D == 2 ? oy - HY - 1 + py : 0, 0));
        }
        __syncthreads();
        bool tgt[CPT];
        int up[CPT][2];
        double w[CPT][2];
#pragma unroll
        for (int m = 0; m < CPT; m++) {
            int r = threadIdx.x + m * WGS;
            tgt[m] = false;
            if (r >= RN) continue;
            int rx = r % RX, ry = r / RX;
            int gi = ox - EXT_H + rx, gj = oy - HY + ry;
            int c = cidx(g, gi, gj, 0);
            int sx = src_pos(g, 0, ox - EXT_H, gi), sy = D == 2 ? src_pos(g, 1, oy - HY, gj) : 0;
            for (int e = 0; e < D; e++) sA[e * RN + r] = g.v[in][e][c];
            if (!g.M[c]) continue;
            int ci, cj, ck;
            coords(g, c, ci, cj, ck);
            double gv[3];
            if (iface<D>(g, ci, cj, ck, gv) > 0.0) continue;   // cut cells are the sources
            int pc = (sx + 1) + PX * (D == 2 ? sy + 1 : 0);
            double gr[2], g2 = 0.0;
            gr[0] = (sPhi[pc + 1] - sPhi[pc - 1]) / (2.0 * g.h);
            g2 += gr[0] * gr[0];
            if (D == 2) {
                gr[1] = (sPhi[pc + PX] - sPhi[pc - PX]) / (2.0 * g.h);
                g2 += gr[1] * gr[1];
            }
            double gmp = sqrt(g2);
            if (!(gmp > 0.0)) continue;
            double sg = sPhi[pc] < 0.0 ? -1.0 : 1.0;
            bool inside = true;
            double wsum = 0.0;
            for (int d = 0; d < D; d++) {
                double nd = sg * gr[d] / gmp;
                int o = nd > 0.0 ? -1 : 1;
                int qx = sx + (d == 0 ? o : 0), qy = sy + (d == 1 ? o : 0);
                inside &= qx >= 0 && qx < RX && qy >= 0 && qy < RY;
                up[m][d] = qx + RX * qy;
                w[m][d] = fabs(nd);
                wsum += w[m][d];
            }
            double iw = 1.0 / wsum;
            for (int d = 0; d < D; d++) w[m][d] *= iw;
            tgt[m] = inside;
        }
        __syncthreads();
        double* A = sA;
        double* B = sB;
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int m = 0; m < CPT; m++) {
                int r = threadIdx.x + m * WGS;
                if (r >= RN) continue;
                for (int e = 0; e < D; e++) {
                    double v;
                    if (tgt[m]) {
                        v = w[m][0] * A[e * RN + up[m][0]];
                        if (D == 2) v += w[m][1] * A[e * RN + up[m][1]];
                    } else {
                        v = A[e * RN + r];
                    }
                    B[e * RN + r] = v;
                }
            }
            __syncthreads();
            double* tmp = A; A = B; B = tmp;
        }
        for (int u = threadIdx.x; u < TX * TY; u += WGS) {
            int li = u % TX, lj = u / TX;
            int i = ox + li, j = oy + lj;
            if (i < g.n[0] && j < g.n[1]) {
                int c = i + g.n[0] * j;
                if (g.M[c]) {
                    int r = (li + EXT_H) + RX * (lj + HY);
                    for (int e = 0; e < D; e++) g.v[out][e][c] = A[e * RN + r];
                }
            }
        }
        __syncthreads();
    }
}
template <int D>
__global__ void __launch_bounds__(ExtWG<D>::V, 2 * ExtWG<D>::V / 256) k_vext_tb(Dev g, int list, int in, int out,
                                                                                int iters, const double* cur)
{
    b_vext_tb<D>(VB::grid(), g, list, in, out, iters, cur);
}

// ---------------------------------------------------------------------------
// interface interaction: exact Riemann problem per cut cell; exchange term of
// fluid 0 per unit volume X/dV = (0, -p* g, -p* u* |g|); optionally books
// wcorr * X_slow into the interfacial flux correction
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void b_interact(const VB blk, const Dev& g, int list, int wb, int vb, double wcorr, int S,
                                           const double* cur)
{
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        if (!g.M[c]) continue;   // a cut cell is a band-mask cell; nothing reads these fields off the mask
        double gv[3];
        double gm = iface<D>(g, i, j, kk, gv);
        if (!(gm > 0.0)) {
            interface_store<D>(g, c, gv, gm, nullptr, 0.0, S);
            continue;
        }
        double st[4];
        const double jump = g.pj ? laplace_jump<D>(g, cur, i, j, kk) : 0.0;
        interface_solve<D>(g, c, gv, gm, wb, st, jump);
        interface_store<D>(g, c, gv, gm, st, wcorr, S, jump);
        for (int d = 0; d < D; d++) g.v[vb][d][c] = st[1] * gv[d] / gm;
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_interact(Dev g, int list, int wb, int vb, double wcorr, int S,
                                                       const double* cur)
{
    b_interact<D>(VB::grid(), g, list, wb, vb, wcorr, S, cur);
}

// corr += w * X_slow from the stored interface solution (cycle start)
template <int D>
__device__ __forceinline__ void b_corr_add(const VB blk, const Dev& g, int list, double w, int S)
{
    if (g.use_sched) w = g.sched[SCHED_W0];
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        double gv[3];
        double gm = iface<D>(g, i, j, kk, gv);
        if (!(gm > 0.0)) continue;
        double sg = S == 0 ? 1.0 : -1.0, p = (S == 1 && g.pj) ? g.ps[c] - g.pj[c] : g.ps[c];
        for (int d = 0; d < D; d++) g.corr[(size_t)(1 + d) * g.nc + c] += w * (-sg * p * gv[d]);
        g.corr[(size_t)(D + 1) * g.nc + c] += w * (-sg * p * g.us[c] * gm);
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_corr_add(Dev g, int list, double w, int S)
{
    b_corr_add<D>(VB::grid(), g, list, w, S);
}

// slow fluid += correction; the correction is reset for the next cycle
template <int D>
__device__ __forceinline__ void b_corr_apply(const VB blk, const Dev& g, int list, int S, int apply)
{
    constexpr int NV = D + 2;
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        for (int q = 1; q < NV; q++) {
            size_t e = (size_t)q * g.nc + c;
            if (apply) g.X[S][e] += g.corr[e];
            g.corr[e] = 0.0;
        }
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_corr_apply(Dev g, int list, int S, int apply)
{
    b_corr_apply<D>(VB::grid(), g, list, S, apply);
}

// ---------------------------------------------------------------------------
// CFL: max over cells holding fluid k of sum_d (|u_d| + c)/dx, with the star
// state of cut cells; also counts the cells holding the fluid
// ---------------------------------------------------------------------------
template <int D, bool BAND>
__device__ __forceinline__ void b_cfl(const VB blk, const Dev& g, int list, int k, const double* cons, int wb)
{
    constexpr int NV = D + 2;
    __shared__ double smax[SHARP_WG / 64];
    __shared__ unsigned long long scnt[SHARP_WG / 64];
    const int* L = list_ptr(g, list);
    if (blk.b >= list_count(g, list)) return;   // idle block: nothing to reduce
    double mx = 0.0;
    unsigned long long cnt = 0;
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        double a = BAND ? alpha_k(g, k, c) : 1.0;
        if (!(a > 0.0)) continue;
        cnt++;
        double W[NV];
        if (BAND && (g.M[c] || a < g.amix)) {
            for (int q = 0; q < NV; q++) W[q] = g.Wb[k][wb][(size_t)q * g.nc + c];
        } else {
            double U[NV];
            for (int q = 0; q < NV; q++) U[q] = cons[(size_t)q * g.nc + c] / a;
            if (!cons2prim<D>(g.gam[k], g.pinf[k], U, W)) flag_nonphys(g, c, k);
        }
        double cs = csound(g.gam[k], g.pinf[k], W[0], W[D + 1]), s = 0.0;
        for (int d = 0; d < D; d++) s += (fabs(W[1 + d]) + cs) / g.h;
        mx = fmax(mx, s);
        if (BAND && g.M[c]) mx = fmax(mx, g.ss[k][c]);   // star speeds live on the band-mask cells
    }
    // wavefront then block reduction (max is order independent)
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_down(mx, off, 64));
        cnt += __shfl_down(cnt, off, 64);
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { smax[wid] = mx; scnt[wid] = cnt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < SHARP_WG / 64; w++) { mx = fmax(mx, smax[w]); cnt += scnt[w]; }
        if (!(mx >= 0.0) || isinf(mx)) { flag_error(g, ERR_NONPHYS); mx = 0.0; }
        atomicMax(&g.red[k], (unsigned long long)__double_as_longlong(mx));
        atomicAdd(&g.red[2 + k], cnt);
    }
}
template <int D, bool BAND>
__global__ void __launch_bounds__(SHARP_WG) k_cfl(Dev g, int list, int k, const double* cons, int wb)
{
    b_cfl<D, BAND>(VB::grid(), g, list, k, cons, wb);
}

// Check of a call's final state: every cell of fluid k on its bulk tiles,
// and every real cell (alpha_k >= alpha_mix) of the band tiles, must hold a
// physical state.  The lists are those of the last cycle start, which cover
// every cell the cycle could move into a fluid.
template <int D>
__device__ __forceinline__ void b_verify(const VB blk, const Dev& g, int list, int k)
{
    constexpr int NV = D + 2;
    const int* L = list_ptr(g, list);
    const double* cons = g.X[k];
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        double a = list == LIST_BAND ? alpha_k(g, k, c) : 1.0;
        if (a < g.amix) continue;
        double U[NV], W[NV];
        for (int q = 0; q < NV; q++) U[q] = cons[(size_t)q * g.nc + c] / a;
        if (!cons2prim<D>(g.gam[k], g.pinf[k], U, W)) flag_nonphys(g, c, k);
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_verify(Dev g, int list, int k)
{
    b_verify<D>(VB::grid(), g, list, k);
}

__device__ __forceinline__ void b_zero_red(const VB blk, const Dev& g)
{
    if (threadIdx.x < 4) g.red[threadIdx.x] = 0ull;
}
__global__ void k_zero_red(Dev g)
{
    b_zero_red(VB::grid(), g);
}
// accumulators of a run of captured steps or cycles (reduction words 5-7):
// each fluid's active-cell count summed over its steps, and the step or
// cycle count.  `add` 0 resets them; otherwise bit k adds fluid k's count
// of the last CFL reduction (word 2 + k) to word 5 + k, bit 2 counts a step
// or cycle, and bit 3 keeps both counts (words 9, 10) as those at the start
// of the last one
__device__ __forceinline__ void b_acc(const VB blk, const Dev& g, int add)
{
    if (threadIdx.x == 0) {
        if (add == 0) {
            g.red[5] = 0ull;
            g.red[6] = 0ull;
            g.red[7] = 0ull;
            return;
        }
        if (add & 1) g.red[5] += g.red[2];
        if (add & 2) g.red[6] += g.red[3];
        if (add & 4) g.red[7] += 1ull;
        if (add & 8) {
            g.red[9] = g.red[2];
            g.red[10] = g.red[3];
        }
    }
}
__global__ void k_acc(Dev g, int add)
{
    b_acc(VB::grid(), g, add);
}

// ---------------------------------------------------------------------------
// one Shu-Osher stage of fluid k (the stage kernels below):
//   out = a*base + (1-a)*(self + dt*L),  L = sum_d (A_lo F_lo - A_hi F_hi)/dx + X/dV
// Face fluxes of a tile are computed once into LDS (the high faces of the
// tile edge are recomputed by the neighbour tile), then combined per cell.
// BAND: apertures, ghost states, exchange term, optional override `self2`
// (read instead of `in` at band-mask cells: the slow fluid's mixed state).
// ---------------------------------------------------------------------------
template <int D> struct FaceCount;
template <> struct FaceCount<1> { static constexpr int n0 = 257, n1 = 0, n2 = 0; };
template <> struct FaceCount<2> { static constexpr int n0 = 17 * 16, n1 = 16 * 17, n2 = 0; };

// state of fluid k at cell c for a stage: primitives W and conservative U
// (ghost states below alpha_mix on band tiles)
// mine: the cell is known to lie in fluid k (alpha_k = 1, not read)
template <int D, bool BAND>
__device__ __forceinline__ void load_state(const Dev& g, int k, const double* in, const double* self2, int wb,
                                           int c, double* W, double* U, bool mine = false)
{
    constexpr int NV = D + 2;
    double a = BAND ? (mine ? 1.0 : alpha_k(g, k, c)) : 1.0;
    if (BAND && a < g.amix) {
        const double* Wg = g.Wb[k][wb];
        for (int q = 0; q < NV; q++) W[q] = Wg[(size_t)q * g.nc + c];
        prim2cons<D>(g.gam[k], g.pinf[k], W, U);
        return;
    }
    const double* src = (BAND && self2 && g.M[c]) ? self2 : in;
    if (BAND) {
        for (int q = 0; q < NV; q++) U[q] = src[(size_t)q * g.nc + c] / a;
    } else {
        for (int q = 0; q < NV; q++) U[q] = src[(size_t)q * g.nc + c];
    }
    cons2prim<D>(g.gam[k], g.pinf[k], U, W);
}

// Band tiles far from the interface.  When the level set stays farther than
// 8 cells from every cell of the tile and its one-cell halo (the geometry
// kernels record that minimum), the stage's region (three cells beyond the
// tile), its faces and their vertices lie on one side of the interface:
// volume fractions and apertures are exactly 1 or 0 and no cell is cut.
// Returns 1 when that side is fluid k (the band update is the plain update:
// the fractions and apertures are not read, the interface term is zero), 2
// when it is the other fluid (every aperture is 0: no flux, the update keeps
// the stage input), 0 otherwise.
constexpr double STAGE_FAR = 8.0;
template <int D>
__device__ __forceinline__ int band_far(const Dev& g, int k, int t, int ox, int oy, int oz)
{
    if (!(g.tphimin[t] > STAGE_FAR * g.h)) return 0;
    return alpha_k(g, k, ox + g.n[0] * (oy + g.n[1] * oz)) == 1.0 ? 1 : 2;
}

// ---------------------------------------------------------------------------
// LDS-staged stage kernel (1-D and 2-D): the primitives of the tile and its
// three-cell halo are computed once per cell into LDS (SoA), every face flux
// of the tile is computed once from LDS, then each cell combines its faces.
// ---------------------------------------------------------------------------
template <int D> struct Region;
template <> struct Region<1> { static constexpr int X = 256 + 6, Y = 1; };
template <> struct Region<2> { static constexpr int X = 16 + 6, Y = 16 + 6; };

// threads per block of the LDS stage kernel (one per tile cell: blocks with
// a fifth wavefront share a SIMD between two of theirs and run slower)
template <int D> struct StageWG { static constexpr int N = SHARP_WG; };

// `tmp` (band tiles, may be null): the output of inner band tiles goes there
// instead of `out`, to be mixed into `out` out of place
template <int D, bool BAND>
__device__ __forceinline__ void b_stage_lds(const VB blk, const Dev& g, int list, int k, const double* in,
                                            const double* self2, const double* base, double* out, double a, double dt,
                                            double wflux, int wb, int cfl, double* tmp)
{
    constexpr int NT = StageWG<D>::N;
    __shared__ double sMax[NT / 64];
    double cmax = 0.0;          // CFL speed of this thread's output cells (bulk, when cfl != 0)
    unsigned long long ccnt = 0;
    static_assert(D <= 2, "LDS stage kernel is for 1-D and 2-D");
    constexpr int NV = D + 2;
    constexpr int TX = Tile<D>::X, TY = Tile<D>::Y;
    constexpr int RX = Region<D>::X, RY = Region<D>::Y, RN = RX * RY;
    constexpr int F0 = FaceCount<D>::n0, F1 = FaceCount<D>::n1;
    constexpr int FT = F0 + F1;
    __shared__ double sR[RN], sU[RN], sV[D > 1 ? RN : 1], sE[RN], sP[RN], sC[RN];
    __shared__ double sF[FT * NV];
    const int* L = list_ptr(g, list);
    const double gm = g.gam[k], pi = g.pinf[k];
    const double farea = D == 1 ? 1.0 : g.h;
    const double ih = 1.0 / g.h;
    const double eps4 = 4.0 * g.eps;
    if (g.use_sched) { dt = g.sched[SCHED_DT]; wflux = g.sched[SCHED_W0]; }
    const ListRange lr = xcd_range(blk, list_count(g, list));
    for (int ti = lr.begin; ti < lr.end; ti += lr.step) {
        int t = L[ti];
        int tx = t % g.nt[0], ty = (t / g.nt[0]) % g.nt[1];
        int ox = tx * TX, oy = ty * TY;
        const int far = BAND ? band_far<D>(g, k, t, ox, oy, 0) : 0;
        // ---- primitives of the tile and its halo (the corners are never used:
        // in 2-D the 448 other region cells are enumerated densely) ----
        constexpr int NL = D == 2 ? RN - 4 * 9 : RN;
        for (int q = threadIdx.x; q < (far == 2 ? 0 : NL); q += NT) {
            int rx, ry;
            if (D == 1) {
                rx = q;
                ry = 0;
            } else if (q < 3 * TX) {
                ry = q / TX;
                rx = 3 + q % TX;
            } else if (q < 3 * TX + TY * RX) {
                int u = q - 3 * TX;
                ry = 3 + u / RX;
                rx = u % RX;
            } else {
                int u = q - 3 * TX - TY * RX;
                ry = TY + 3 + u / TX;
                rx = 3 + u % TX;
            }
            int r = rx + RX * ry;
            int c = cidx(g, ox - 3 + rx, D == 2 ? oy - 3 + ry : 0, 0);
            double W[NV], U[NV];
            load_state<D, BAND>(g, k, in, self2, wb, c, W, U, far == 1);
            sR[r] = W[0];
            sU[r] = W[1];
            if (D == 2) sV[r] = W[2];
            sE[r] = U[NV - 1];
            sP[r] = W[NV - 1];
            sC[r] = csound(gm, pi, W[0], W[NV - 1]);
        }
        __syncthreads();
        // ---- face fluxes ----
        for (int f = threadIdx.x; f < FT; f += NT) {
            int d, li, lj;
            if (f < F0) { d = 0; li = f % (TX + 1); lj = f / (TX + 1); }
            else { int r = f - F0; d = 1; li = r % TX; lj = r / TX; }
            int i = ox + li, j = oy + lj;
            bool ok = far != 2 && (d == 0 ? (i <= g.n[0] && j < g.n[1]) : (i < g.n[0] && j <= g.n[1]));
            double* Fo = sF + (size_t)f * NV;
            double A = 1.0;
            if (ok && BAND && !far) {
                A = g.ap[d][fidx(g, i, j, 0)];
                if (k == 1) A = 1.0 - A;
                ok = A > 0.0;
            }
            if (!ok) {
#pragma unroll
                for (int q = 0; q < NV; q++) Fo[q] = 0.0;
                continue;
            }
            // stencil m = 0..5 <-> cells i-3 .. i+2 along d (region coordinates)
            int r0 = d == 0 ? (li + RX * (D == 2 ? lj + 3 : 0)) : (li + 3 + RX * lj);
            int st = d == 0 ? 1 : RX;
            double rho[6], un[6], ut[6], E[6], p[6];
            double amax = 0.0;
#pragma unroll
            for (int m = 0; m < 6; m++) {
                int r = r0 + m * st;
                rho[m] = sR[r];
                double uu = sU[r], vv = D == 2 ? sV[r] : 0.0;
                un[m] = d == 0 ? uu : vv;
                ut[m] = d == 0 ? vv : uu;
                E[m] = sE[r];
                p[m] = sP[r];
                amax = fmax(amax, fabs(un[m]) + sC[r]);
            }
 #pragma unroll
            for (int q = 0; q < NV; q++) {
                // split fluxes F +- a U of component q (the factor 1/2 and the
                // 1/6 of the candidate stencils are applied once at the end)
                double fp[6], fm[6];
#pragma unroll
                for (int m = 0; m < 6; m++) {
                    double Uq, Fq;
                    if (q == 0) { Uq = rho[m]; Fq = rho[m] * un[m]; }
                    else if (q == NV - 1) { Uq = E[m]; Fq = (E[m] + p[m]) * un[m]; }
                    else {
                        // momentum component q-1 (x for q = 1, y for q = 2)
                        bool normal = (q - 1) == d;
                        double uq = normal ? un[m] : ut[m];
                        Uq = rho[m] * uq;
                        Fq = Uq * un[m] + (normal ? p[m] : 0.0);
                    }
                    fp[m] = fma(amax, Uq, Fq);
                    fm[m] = fma(-amax, Uq, Fq);
                }
                double Fh = weno5_q(fp[0], fp[1], fp[2], fp[3], fp[4], eps4)
                          + weno5_q(fm[5], fm[4], fm[3], fm[2], fm[1], eps4);
                Fo[q] = (A * (1.0 / 12.0)) * Fh;
            }
            if (g.bc[d] == 0 && wflux != 0.0) {
                int fi = d == 0 ? i : j;
                if (fi == 0 || fi == g.n[d]) {
                    int side = fi == 0 ? 0 : 1;
                    int b = g.bface_off[d][side] + (d == 0 ? j : i);
                    double sgn = side == 0 ? 1.0 : -1.0;
                    for (int q = 0; q < NV; q++) g.bacc[k][(size_t)q * g.nbface + b] += sgn * wflux * farea * Fo[q];
                }
            }
        }
        __syncthreads();
        // ---- cell update ----
        if (threadIdx.x < TX * TY) {
            int li = threadIdx.x % TX, lj = threadIdx.x / TX;
            int i = ox + li, j = oy + lj;
            if (i < g.n[0] && j < g.n[1]) {
                int c = i + g.n[0] * j;
                double Lr[NV];
                int fxl = li + (TX + 1) * lj;
#pragma unroll
                for (int q = 0; q < NV; q++) Lr[q] = (sF[(size_t)fxl * NV + q] - sF[(size_t)(fxl + 1) * NV + q]) * ih;
                if (D == 2) {
                    int fyl = F0 + li + TX * lj;
#pragma unroll
                    for (int q = 0; q < NV; q++) Lr[q] += (sF[(size_t)fyl * NV + q] - sF[(size_t)(fyl + TX) * NV + q]) * ih;
                }
                if (BAND && !far) {
                    double gv[3];
                    double gn = iface<D>(g, i, j, 0, gv);
                    if (gn > 0.0) {
                        double sg = k == 0 ? 1.0 : -1.0, p = (k == 1 && g.pj) ? g.ps[c] - g.pj[c] : g.ps[c];
                        for (int d = 0; d < D; d++) Lr[1 + d] += -sg * p * gv[d];
                        Lr[D + 1] += -sg * p * g.us[c] * gn;
                    }
                }
                const double* sin_ = (BAND && self2 && g.M[c]) ? self2 : in;
                double* dst = (BAND && tmp && !(g.tflag[t] & 4)) ? tmp : out;
                double Uo[NV];
#pragma unroll
                for (int q = 0; q < NV; q++) {
                    size_t e = (size_t)q * g.nc + c;
                    double s = sin_[e] + dt * Lr[q];
                    Uo[q] = (a == 0.0) ? s : a * base[e] + (1.0 - a) * s;
                    dst[e] = Uo[q];
                }
                if (!BAND && cfl) {
                    double W[NV];
                    if (!cons2prim<D>(gm, pi, Uo, W)) flag_nonphys(g, c, k);
                    double cs = csound(gm, pi, W[0], W[D + 1]), sp = 0.0;
                    for (int d = 0; d < D; d++) sp += (fabs(W[1 + d]) + cs) / g.h;
                    cmax = fmax(cmax, sp);
                    ccnt++;
                }
            }
        }
        __syncthreads();
    }
    if (!BAND && cfl) {
        if (lr.begin >= lr.end) return;   // idle block: nothing to reduce
        for (int off = 32; off > 0; off >>= 1) {
            cmax = fmax(cmax, __shfl_down(cmax, off, 64));
            ccnt += __shfl_down(ccnt, off, 64);
        }
        __shared__ unsigned long long sCnt[NT / 64];
        int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        if (lane == 0) { sMax[wid] = cmax; sCnt[wid] = ccnt; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < NT / 64; w++) { cmax = fmax(cmax, sMax[w]); ccnt += sCnt[w]; }
            if (!(cmax >= 0.0) || isinf(cmax)) { flag_error(g, ERR_NONPHYS); cmax = 0.0; }
            atomicMax(&g.red[k], (unsigned long long)__double_as_longlong(cmax));
            atomicAdd(&g.red[2 + k], ccnt);
        }
    }
}
template <int D, bool BAND>
__global__ void __launch_bounds__(StageWG<D>::N) k_stage_lds(Dev g, int list, int k, const double* in,
                                                             const double* self2, const double* base, double* out,
                                                             double a, double dt, double wflux, int wb, int cfl,
                                                             double* tmp)
{
    b_stage_lds<D, BAND>(VB::grid(), g, list, k, in, self2, base, out, a, dt, wflux, wb, cfl, tmp);
}

// ---------------------------------------------------------------------------
// LDS-staged stage kernel (3-D), one direction at a time: for d = x, y, z
// the primitives of the tile and its three-cell halo along d (448 or 640
// cells) are staged in LDS, the tile's faces normal to d (288 or 320) are
// computed from LDS, and each cell adds its flux difference along d.  The
// tile's own cells are converted once and kept in registers; LDS holds one
// direction's region and faces (49 KB).  Same arithmetic as the 2-D kernel.
// ---------------------------------------------------------------------------
// 256 threads (one per tile cell), three waves per SIMD.  The block size is
// fixed: a build with 320 threads per block (one face round per direction)
// faulted the GPU in a timing experiment, with no cause found in the code.
#define SHARP_WG3 256
#define SHARP_WG3_WAVES 3
// LDS of one block of the 3-D stage: one direction's region (primitives,
// energy and sound speed of the tile and its three-cell halo along that
// direction) and the faces normal to it
struct Stage3Lds {
    static constexpr int TX = 8, TY = 8, TZ = 4;
    static constexpr int RMAX = TX * TY * (TZ + 6);   // largest directional region (z)
    static constexpr int FMAX = TX * TY * (TZ + 1);   // most faces normal to one direction (z)
    double R[RMAX], U[RMAX], V[RMAX], W[RMAX], E[RMAX], P[RMAX], C[RMAX];
    double F[FMAX * 5];
};

// Component q of the WENO5-LLF flux through the face whose stencil starts at
// region index r0 (cells -3 .. +2 along d, stride st), times A/12.  Density
// and normal velocity come in registers; the other values are read from LDS
// where the component needs them.
template <int d, int q>
__device__ __forceinline__ double face3_comp(const Stage3Lds& S, int r0, int st, const double* rho, const double* un,
                                             double amax, double eps4, double A)
{
    constexpr int NV = 5;
    const double* Sq = q == 1 ? S.U : (q == 2 ? S.V : S.W);
    double fp[6], fm[6];
#pragma unroll
    for (int m = 0; m < 6; m++) {
        const int r = r0 + m * st;
        double Uq, Fq;
        if (q == 0) { Uq = rho[m]; Fq = rho[m] * un[m]; }
        else if (q == NV - 1) { const double E = S.E[r]; Uq = E; Fq = (E + S.P[r]) * un[m]; }
        else {
            // momentum component along axis q-1
            Uq = rho[m] * Sq[r];
            Fq = Uq * un[m] + (q - 1 == d ? S.P[r] : 0.0);
        }
        fp[m] = fma(amax, Uq, Fq);
        fm[m] = fma(-amax, Uq, Fq);
    }
    double Fh = weno5_q(fp[0], fp[1], fp[2], fp[3], fp[4], eps4) + weno5_q(fm[5], fm[4], fm[3], fm[2], fm[1], eps4);
    return (A * (1.0 / 12.0)) * Fh;
}

// One direction d of the 3-D stage for the tile at (ox, oy, oz): stage the
// halo along d (the tile's own cells come from registers), compute the faces
// normal to d, and add each cell's flux difference along d to Lr.  The
// direction is a template parameter, so the region and face shapes, the
// stencil stride and the normal velocity are compile-time constants.
template <int d, bool BAND>
__device__ __forceinline__ void stage3_dir(const Dev& g, int k, const double* in, const double* self2, int wb,
                                           int far, int ox, int oy, int oz, int tid, bool own, bool inside,
                                           int li, int lj, int lk, const double* Wc, const double* Uc, double cc,
                                           double gm, double pi, double eps4, double ih, double farea, double wflux,
                                           Stage3Lds& S, double* Lr)
{
    constexpr int NV = 5, NT = SHARP_WG3;
    constexpr int TX = Stage3Lds::TX, TY = Stage3Lds::TY, TZ = Stage3Lds::TZ;
    constexpr int RX = TX + (d == 0 ? 6 : 0), RY = TY + (d == 1 ? 6 : 0), RZ = TZ + (d == 2 ? 6 : 0);
    constexpr int hx = d == 0 ? 3 : 0, hy = d == 1 ? 3 : 0, hz = d == 2 ? 3 : 0;
    // the six halo layers along d: layer l < 3 is below the tile, l >= 3 above
    constexpr int A0 = d == 0 ? TY : TX;                       // extents across d
    constexpr int A1 = d == 2 ? TY : TZ;
    constexpr int NH = 6 * A0 * A1;
    for (int q = tid; q < NH; q += NT) {
        const int a0 = q % A0, a1 = (q / A0) % A1, l = q / (A0 * A1);
        const int od = l < 3 ? l : l + (d == 0 ? TX : (d == 1 ? TY : TZ));   // position along d in the region
        const int rx = d == 0 ? od : a0, ry = d == 1 ? od : (d == 0 ? a0 : a1), rz = d == 2 ? od : a1;
        const int r = rx + RX * (ry + RY * rz);
        int c = cidx(g, ox - hx + rx, oy - hy + ry, oz - hz + rz);
        double W[NV], U[NV];
        load_state<3, BAND>(g, k, in, self2, wb, c, W, U, far == 1);
        S.R[r] = W[0];
        S.U[r] = W[1];
        S.V[r] = W[2];
        S.W[r] = W[3];
        S.E[r] = U[NV - 1];
        S.P[r] = W[NV - 1];
        S.C[r] = csound(gm, pi, W[0], W[NV - 1]);
    }
    if (own) {
        const int r = (li + hx) + RX * ((lj + hy) + RY * (lk + hz));
        S.R[r] = Wc[0];
        S.U[r] = Wc[1];
        S.V[r] = Wc[2];
        S.W[r] = Wc[3];
        S.E[r] = Uc[NV - 1];
        S.P[r] = Wc[NV - 1];
        S.C[r] = cc;
    }
    __syncthreads();
    // faces normal to d
    constexpr int FX = TX + (d == 0), FY = TY + (d == 1), FZ = TZ + (d == 2);
    constexpr int FN = FX * FY * FZ;
    constexpr int st = d == 0 ? 1 : (d == 1 ? RX : RX * RY);
    // The face's aperture (0 when it carries no flux of fluid k) and its
    // boundary side; the LLF speed of its six-cell stencil.
    auto face_at = [&](int f, int& fi, int& fj, int& fk, double& A) {
        const int fx = f % FX, fy = (f / FX) % FY, fz = f / (FX * FY);
        fi = ox + fx;
        fj = oy + fy;
        fk = oz + fz;
        bool ok = (d == 0 ? fi <= g.n[0] : fi < g.n[0]) && (d == 1 ? fj <= g.n[1] : fj < g.n[1]) &&
                  (d == 2 ? fk <= g.n[2] : fk < g.n[2]);
        A = ok ? 1.0 : 0.0;
        if (ok && BAND && !far) {
            A = g.ap[d][fidx(g, fi, fj, fk)];
            if (k == 1) A = 1.0 - A;
        }
        return fx + RX * (fy + RY * fz);      // region index of stencil cell m = 0
    };
    auto bflux = [&](int fi, int fj, int fk, int q, double Fq) {
        const int fd = d == 0 ? fi : (d == 1 ? fj : fk);
        if (g.bc[d] == 0 && wflux != 0.0 && (fd == 0 || fd == g.n[d])) {
            int side = fd == 0 ? 0 : 1;
            int o1 = d == 0 ? fj : fi, o2 = d == 2 ? fj : fk;
            int n1 = d == 0 ? g.n[1] : g.n[0];
            int b = g.bface_off[d][side] + o1 + n1 * o2;
            double sgn = side == 0 ? 1.0 : -1.0;
            g.bacc[k][(size_t)q * g.nbface + b] += sgn * wflux * farea * Fq;
        }
    };
    // stencil m = 0..5 <-> cells -3 .. +2 along d from the face: density,
    // normal velocity and the LLF speed max(|u_d| + c)
    const double* Sd = d == 0 ? S.U : (d == 1 ? S.V : S.W);
    auto stencil = [&](int r0, double* rho, double* un) {
        double amax = 0.0;
#pragma unroll
        for (int m = 0; m < 6; m++) {
            const int r = r0 + m * st;
            rho[m] = S.R[r];
            un[m] = Sd[r];
            amax = fmax(amax, fabs(un[m]) + S.C[r]);
        }
        return amax;
    };
    // One thread per face, all components, for the first NT faces
    constexpr int FULL = FN < NT ? FN : NT;
    if (tid < FULL) {
        const int f = tid;
        int fi, fj, fk;
        double A;
        const int r0 = face_at(f, fi, fj, fk, A);
        double* Fo = S.F + (size_t)f * NV;
        if (!(A > 0.0)) {
#pragma unroll
            for (int q = 0; q < NV; q++) Fo[q] = 0.0;
        } else {
            double rho[6], un[6];
            const double amax = stencil(r0, rho, un);
            Fo[0] = face3_comp<d, 0>(S, r0, st, rho, un, amax, eps4, A);
            Fo[1] = face3_comp<d, 1>(S, r0, st, rho, un, amax, eps4, A);
            Fo[2] = face3_comp<d, 2>(S, r0, st, rho, un, amax, eps4, A);
            Fo[3] = face3_comp<d, 3>(S, r0, st, rho, un, amax, eps4, A);
            Fo[4] = face3_comp<d, 4>(S, r0, st, rho, un, amax, eps4, A);
#pragma unroll
            for (int q = 0; q < NV; q++) bflux(fi, fj, fk, q, Fo[q]);
        }
    }
    // The remaining FN - NT faces (32 or 64) would leave all but one wave
    // idle for a whole face each: they are spread over the block as one
    // thread per (face, component), 64 slots per component so that each
    // wave works on one component (a uniform branch to the same code as
    // above).
    constexpr int REST = FN - FULL;
    static_assert(REST <= 64, "at most 64 remaining faces");
    for (int it = tid; REST > 0 && it < NV * 64; it += NT) {
        const int q = __builtin_amdgcn_readfirstlane(it >> 6), j = it & 63;
        if (j >= REST) continue;
        const int f = FULL + j;
        int fi, fj, fk;
        double A;
        const int r0 = face_at(f, fi, fj, fk, A);
        double* Fo = S.F + (size_t)f * NV;
        double Fq = 0.0;
        if (A > 0.0) {
            double rho[6], un[6];
            const double amax = stencil(r0, rho, un);
            switch (q) {
            case 0: Fq = face3_comp<d, 0>(S, r0, st, rho, un, amax, eps4, A); break;
            case 1: Fq = face3_comp<d, 1>(S, r0, st, rho, un, amax, eps4, A); break;
            case 2: Fq = face3_comp<d, 2>(S, r0, st, rho, un, amax, eps4, A); break;
            case 3: Fq = face3_comp<d, 3>(S, r0, st, rho, un, amax, eps4, A); break;
            default: Fq = face3_comp<d, 4>(S, r0, st, rho, un, amax, eps4, A); break;
            }
            bflux(fi, fj, fk, q, Fq);
        }
        Fo[q] = Fq;
    }
    __syncthreads();
    if (inside) {
        const int flo = li + FX * (lj + FY * lk);
        constexpr int fs = d == 0 ? 1 : (d == 1 ? FX : FX * FY);
#pragma unroll
        for (int q = 0; q < NV; q++) Lr[q] += (S.F[(size_t)flo * NV + q] - S.F[(size_t)(flo + fs) * NV + q]) * ih;
    }
    __syncthreads();
}

template <bool BAND>
__device__ __forceinline__ void b_stage_lds3(const VB blk, const Dev& g, int list, int k, const double* in,
                                             const double* self2, const double* base, double* out, double a, double dt,
                                             double wflux, int wb, int cfl, double* tmp)
{
    constexpr int D = 3, NV = 5, NT = SHARP_WG3;
    constexpr int TX = Stage3Lds::TX, TY = Stage3Lds::TY, TZ = Stage3Lds::TZ, TN = TX * TY * TZ;
    __shared__ Stage3Lds S;
    __shared__ double sMax[(NT + 63) / 64];
    __shared__ unsigned long long sCnt[(NT + 63) / 64];
    double cmax = 0.0;
    unsigned long long ccnt = 0;
    const int* L = list_ptr(g, list);
    const double gm = g.gam[k], pi = g.pinf[k];
    const double farea = g.h * g.h;
    const double ih = 1.0 / g.h;
    const double eps4 = 4.0 * g.eps;
    if (g.use_sched) { dt = g.sched[SCHED_DT]; wflux = g.sched[SCHED_W0]; }
    const int tid = threadIdx.x;
    const bool own = tid < TN;
    const int li = tid % TX, lj = (tid / TX) % TY, lk = tid / (TX * TY);
    const ListRange lr = xcd_range(blk, list_count(g, list));
    for (int ti = lr.begin; ti < lr.end; ti += lr.step) {
        int t = L[ti];
        int ox, oy, oz;
        tile_origin<D>(g, t, ox, oy, oz);
        const int i = ox + li, j = oy + lj, kk = oz + lk;
        const bool inside = own && i < g.n[0] && j < g.n[1] && kk < g.n[2];
        const int far = BAND ? band_far<D>(g, k, t, ox, oy, oz) : 0;
        // the thread's own cell, converted once
        double Wc[NV], Uc[NV], cc = 0.0;
        if (own && far != 2) {
            int c = cidx(g, i, j, kk);
            load_state<D, BAND>(g, k, in, self2, wb, c, Wc, Uc, far == 1);
            cc = csound(gm, pi, Wc[0], Wc[NV - 1]);
        }
        double Lr[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) Lr[q] = 0.0;
        if (far != 2) {
            stage3_dir<0, BAND>(g, k, in, self2, wb, far, ox, oy, oz, tid, own, inside, li, lj, lk, Wc, Uc, cc, gm, pi,
                                eps4, ih, farea, wflux, S, Lr);
            stage3_dir<1, BAND>(g, k, in, self2, wb, far, ox, oy, oz, tid, own, inside, li, lj, lk, Wc, Uc, cc, gm, pi,
                                eps4, ih, farea, wflux, S, Lr);
            stage3_dir<2, BAND>(g, k, in, self2, wb, far, ox, oy, oz, tid, own, inside, li, lj, lk, Wc, Uc, cc, gm, pi,
                                eps4, ih, farea, wflux, S, Lr);
        }
        // ---- cell update ----
        if (inside) {
            int c = i + g.n[0] * (j + g.n[1] * kk);
            if (BAND && !far) {
                double gv[3];
                double gn = iface<D>(g, i, j, kk, gv);
                if (gn > 0.0) {
                    double sg = k == 0 ? 1.0 : -1.0, pp = (k == 1 && g.pj) ? g.ps[c] - g.pj[c] : g.ps[c];
                    for (int e = 0; e < D; e++) Lr[1 + e] += -sg * pp * gv[e];
                    Lr[D + 1] += -sg * pp * g.us[c] * gn;
                }
            }
            const double* sin_ = (BAND && self2 && g.M[c]) ? self2 : in;
            double* dst = (BAND && tmp && !(g.tflag[t] & 4)) ? tmp : out;
            double Uo[NV];
#pragma unroll
            for (int q = 0; q < NV; q++) {
                size_t e = (size_t)q * g.nc + c;
                double sv = sin_[e] + dt * Lr[q];
                Uo[q] = (a == 0.0) ? sv : a * base[e] + (1.0 - a) * sv;
                dst[e] = Uo[q];
            }
            if (!BAND && cfl) {
                double W[NV];
                if (!cons2prim<D>(gm, pi, Uo, W)) flag_nonphys(g, c, k);
                double cs = csound(gm, pi, W[0], W[D + 1]), sp = 0.0;
                for (int e = 0; e < D; e++) sp += (fabs(W[1 + e]) + cs) / g.h;
                cmax = fmax(cmax, sp);
                ccnt++;
            }
        }
    }
    if (!BAND && cfl) {
        if (lr.begin >= lr.end) return;   // idle block: nothing to reduce
        for (int off = 32; off > 0; off >>= 1) {
            cmax = fmax(cmax, __shfl_down(cmax, off, 64));
            ccnt += __shfl_down(ccnt, off, 64);
        }
        int lane = tid & 63, wid = tid >> 6;
        if (lane == 0) { sMax[wid] = cmax; sCnt[wid] = ccnt; }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < (NT + 63) / 64; w++) { cmax = fmax(cmax, sMax[w]); ccnt += sCnt[w]; }
            if (!(cmax >= 0.0) || isinf(cmax)) { flag_error(g, ERR_NONPHYS); cmax = 0.0; }
            atomicMax(&g.red[k], (unsigned long long)__double_as_longlong(cmax));
            atomicAdd(&g.red[2 + k], ccnt);
        }
    }
}
template <bool BAND>
__global__ void __launch_bounds__(SHARP_WG3, SHARP_WG3_WAVES) k_stage_lds3(Dev g, int list, int k, const double* in,
                                                                           const double* self2, const double* base,
                                                                           double* out, double a, double dt,
                                                                           double wflux, int wb, int cfl, double* tmp)
{
    b_stage_lds3<BAND>(VB::grid(), g, list, k, in, self2, base, out, a, dt, wflux, wb, cfl, tmp);
}

// ---------------------------------------------------------------------------
// level set: one Shu-Osher stage of Eq. (LS:linearadvection), WENO5 upwind
// derivatives, band cells only
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void b_ls(const VB blk, const Dev& g, int list, double a, double dt, const double* in,
                                     double* out, int vb)
{
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        if (!g.M[c]) continue;
        double rhs = 0.0;
        for (int d = 0; d < D; d++) {
            double vd = g.v[vb][d][c];
            if (vd == 0.0) continue;
            double p[7];
            for (int m = 0; m < 7; m++) p[m] = phi_at(g, in, cidx(g, i + (d == 0) * (m - 3), j + (d == 1) * (m - 3), kk + (d == 2) * (m - 3)));
            double D1[6];
            for (int m = 0; m < 6; m++) D1[m] = (p[m + 1] - p[m]) / g.h;
            double der = vd > 0.0 ? weno5(D1[0], D1[1], D1[2], D1[3], D1[4], g.eps)
                                  : weno5(D1[5], D1[4], D1[3], D1[2], D1[1], g.eps);
            rhs -= vd * der;
        }
        double s = in[c] + dt * rhs;
        out[c] = (a == 0.0) ? s : a * g.phiP[c] + (1.0 - a) * s;
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_ls(Dev g, int list, double a, double dt, const double* in, double* out,
                                                 int vb)
{
    b_ls<D>(VB::grid(), g, list, a, dt, in, out, vb);
}

// ---------------------------------------------------------------------------
// reinitialisation: Godunov sweeps of phi_tau + S(phi0)(|grad phi| - 1) = 0,
// cells near a sign change of phi0 are kept
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void b_nearif(const VB blk, const Dev& g, int list, const double* phi0)
{
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        int neg = 0, pos = 0;
        int rz = D > 2 ? 1 : 0, ry = D > 1 ? 1 : 0;
        for (int dz = -rz; dz <= rz; dz++)
            for (int dy = -ry; dy <= ry; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    double v = phi_at(g, phi0, cidx(g, i + dx, j + dy, kk + dz));
                    if (v < 0.0) neg = 1; else pos = 1;
                }
        g.nearif[c] = (uint8_t)(neg && pos);
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_nearif(Dev g, int list, const double* phi0)
{
    b_nearif<D>(VB::grid(), g, list, phi0);
}

template <int D>
__device__ __forceinline__ void b_reinit(const VB blk, const Dev& g, int list, const double* phi0, const double* in,
                                         double* out)
{
    const int* L = list_ptr(g, list);
    const double h = g.h, dtau = 0.5 * g.h;
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        if (!g.M[c]) continue;
        double pc = in[c];
        bool frz = false;
        int rz = D > 2 ? 1 : 0, ry = D > 1 ? 1 : 0;
        for (int dz = -rz; dz <= rz; dz++)
            for (int dy = -ry; dy <= ry; dy++)
                for (int dx = -1; dx <= 1; dx++) frz |= g.nearif[cidx(g, i + dx, j + dy, kk + dz)] != 0;
        if (frz) { out[c] = pc; continue; }
        double p0 = phi0[c];
        double S = p0 / sqrt(p0 * p0 + h * h), g2 = 0.0;
        for (int d = 0; d < D; d++) {
            double am = (pc - phi_at(g, in, nbr(g, c, d, -1))) / h;
            double bp = (phi_at(g, in, nbr(g, c, d, 1)) - pc) / h;
            double x, y;
            if (S > 0.0) { x = am > 0.0 ? am : 0.0; y = bp < 0.0 ? bp : 0.0; }
            else { x = am < 0.0 ? am : 0.0; y = bp > 0.0 ? bp : 0.0; }
            g2 += (x * x > y * y) ? x * x : y * y;
        }
        out[c] = pc - dtau * S * (sqrt(g2) - 1.0);
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_reinit(Dev g, int list, const double* phi0, const double* in,
                                                     double* out)
{
    b_reinit<D>(VB::grid(), g, list, phi0, in, out);
}

// copy a scalar field on the band-mask cells (reinitialisation disabled)
template <int D>
__device__ __forceinline__ void b_copy_masked(const VB blk, const Dev& g, int list, const double* src, double* dst)
{
    const int* L = list_ptr(g, list);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int i, j, kk;
        if (!tile_cell<D>(g, L[ti], threadIdx.x, i, j, kk)) continue;
        int c = i + g.n[0] * (j + g.n[1] * kk);
        if (g.M[c]) dst[c] = src[c];
    }
}
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_copy_masked(Dev g, int list, const double* src, double* dst)
{
    b_copy_masked<D>(VB::grid(), g, list, src, dst);
}

// the level set a stage sees, over every cell (a tape entry or a stage
// record): the working buffer on the band-mask cells, the base elsewhere
__global__ void __launch_bounds__(256) k_phi_merge(Dev g, const double* cur, double* out)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x)
        out[c] = g.M[c] ? cur[c] : g.phiP[c];
}

// ---------------------------------------------------------------------------
// The level-set chain of one stage for one tile in one kernel (1-D and 2-D),
// temporally blocked: extension of the interface velocity from the cut cells'
// u* n (k_vext_tb), one Shu-Osher stage of Eq. (LS:linearadvection) (k_ls),
// on the last stage of a step K reinitialisation sweeps (k_nearif, k_reinit),
// and the geometry of the resulting level set (k_geom_lds).  Each step runs
// on a region that shrinks by the reach of the next one, so the tile's values
// are those of the separate kernels:
//   geometry          tile + 1
//   reinit sweep m    tile + K - m + 1, sign-change flags tile + K + 1
//   level-set stage   tile + HL  (HL = K + 2 on the last stage, else 1)
//   velocity          tile + HL + EXT_H (exact at tile + HL after EXT_H sweeps)
//   input level set   tile + HL + EXT_H + 1
// Writes v[vout] and, on the band-mask cells of the tile, the stage output
// (K < 0: not the last stage) or the reinitialised level set to `po`; the
// geometry goes to alpha_out / ap_out (the second buffer set).  The
// reinitialised level set is not written to phiP here: other blocks still
// read phiP in their halos (base of the Shu-Osher stage).

// ---------------------------------------------------------------------------
template <int D, int HL>
__device__ __forceinline__ void b_lsgeo_tb(const VB blk, const Dev& g, int list, int vin, int vout, int iters,
                                           const double* phin, double a, double dt, double* po, int K,
                                           double* alpha_out, double* ap_out0, double* ap_out1, double* tpm_out)
{
    static_assert(D <= 2, "temporally blocked level-set chain is for 1-D and 2-D");
    constexpr int WGS = ExtWG<D>::V;
    constexpr int TX = Tile<D>::X, TY = Tile<D>::Y;
    constexpr int LX = TX + 2 * HL, LY = D == 2 ? TY + 2 * HL : 1, LN = LX * LY;
    constexpr int VH = HL + EXT_H;
    constexpr int VX = TX + 2 * VH, VY = D == 2 ? TY + 2 * VH : 1, VN = VX * VY;
    constexpr int PX = VX + 2, PY = D == 2 ? VY + 2 : 1, PN = PX * PY;
    constexpr int CPT = (VN + WGS - 1) / WGS;
    constexpr int GX = TX + 1, GY = D == 2 ? TY + 1 : 1;
    constexpr bool REUSE = 2 * LN <= D * VN;   // reinitialisation buffers fit in the free velocity buffer
    __shared__ double sQR[REUSE ? 1 : 2 * LN];
    __shared__ double sPhi[PN];
    __shared__ double sA[D * VN], sB[D * VN];
    __shared__ double sL[LN];
    __shared__ uint8_t sM[LN], sN[LN];
    __shared__ double sV[GX * GY];
    __shared__ double sMn[WGS / 64];
    const int* L = list_ptr(g, list);
    const bool last = K >= 0;
    if (g.use_sched) dt = g.sched[SCHED_DT];
    tpm_carry(blk, WGS, g, list, g.tphimin, tpm_out);
    for (int ti = blk.b; ti < list_count(g, list); ti += blk.n) {
        int t = L[ti];
        int ox = (t % g.nt[0]) * TX, oy = D == 2 ? ((t / g.nt[0]) % g.nt[1]) * TY : 0;
        const int vox = ox - VH, voy = D == 2 ? oy - VH : 0;     // velocity region origin
        const int lox = ox - HL, loy = D == 2 ? oy - HL : 0;     // level-set region origin
        // ---- input level set ----
        for (int r = threadIdx.x; r < PN; r += WGS) {
            int px = r % PX, py = r / PX;
            sPhi[r] = phi_at(g, phin, cidx(g, vox - 1 + px, D == 2 ? voy - 1 + py : 0, 0));
        }
        __syncthreads();
        // ---- velocity extension: sources (cut cells), targets, upwind weights ----
        bool tgt[CPT];
        int up[CPT][2];
        double w[CPT][2];
#pragma unroll
        for (int m = 0; m < CPT; m++) {
            int r = threadIdx.x + m * WGS;
            tgt[m] = false;
            if (r >= VN) continue;
            int rx = r % VX, ry = r / VX;
            int gi = vox + rx, gj = voy + ry;
            int c = cidx(g, gi, gj, 0);
            int sx = src_pos(g, 0, vox, gi), sy = D == 2 ? src_pos(g, 1, voy, gj) : 0;
            for (int e = 0; e < D; e++) sA[e * VN + r] = g.v[vin][e][c];
            if (!g.M[c]) continue;
            int ci, cj, ck;
            coords(g, c, ci, cj, ck);
            double gv[3];
            if (iface<D>(g, ci, cj, ck, gv) > 0.0) continue;
            int pc = (sx + 1) + PX * (D == 2 ? sy + 1 : 0);
            double gr[2], g2 = 0.0;
            gr[0] = (sPhi[pc + 1] - sPhi[pc - 1]) / (2.0 * g.h);
            g2 += gr[0] * gr[0];
            if (D == 2) {
                gr[1] = (sPhi[pc + PX] - sPhi[pc - PX]) / (2.0 * g.h);
                g2 += gr[1] * gr[1];
            }
            double gmp = sqrt(g2);
            if (!(gmp > 0.0)) continue;
            double sg = sPhi[pc] < 0.0 ? -1.0 : 1.0;
            bool inside = true;
            double wsum = 0.0;
            for (int d = 0; d < D; d++) {
                double nd = sg * gr[d] / gmp;
                int o = nd > 0.0 ? -1 : 1;
                int qx = sx + (d == 0 ? o : 0), qy = sy + (d == 1 ? o : 0);
                inside &= qx >= 0 && qx < VX && qy >= 0 && qy < VY;
                up[m][d] = qx + VX * qy;
                w[m][d] = fabs(nd);
                wsum += w[m][d];
            }
            double iw = 1.0 / wsum;
            for (int d = 0; d < D; d++) w[m][d] *= iw;
            tgt[m] = inside;
        }
        __syncthreads();
        double* A = sA;
        double* B = sB;
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int m = 0; m < CPT; m++) {
                int r = threadIdx.x + m * WGS;
                if (r >= VN) continue;
                for (int e = 0; e < D; e++) {
                    double v;
                    if (tgt[m]) {
                        v = w[m][0] * A[e * VN + up[m][0]];
                        if (D == 2) v += w[m][1] * A[e * VN + up[m][1]];
                    } else {
                        v = A[e * VN + r];
                    }
                    B[e * VN + r] = v;
                }
            }
            __syncthreads();
            double* tmp = A; A = B; B = tmp;
        }
        // ---- level-set stage on tile + HL (WENO5 upwind derivatives) ----
        for (int r = threadIdx.x; r < LN; r += WGS) {
            int lx = r % LX, ly = r / LX;
            int gi = lox + lx, gj = loy + ly;
            int c = cidx(g, gi, gj, 0);
            int sx = src_pos(g, 0, lox, gi), sy = D == 2 ? src_pos(g, 1, loy, gj) : 0;
            int vs = (sx + EXT_H) + VX * (D == 2 ? sy + EXT_H : 0);
            int ps = (sx + EXT_H + 1) + PX * (D == 2 ? sy + EXT_H + 1 : 0);
            bool inM = g.M[c] != 0;
            sM[r] = inM;
            double phi0 = sPhi[ps];
            if (inM) {
                double rhs = 0.0;
                for (int d = 0; d < D; d++) {
                    double vd = A[d * VN + vs];
                    if (vd == 0.0) continue;
                    int st = d == 0 ? 1 : PX;
                    double p[7];
                    for (int q = 0; q < 7; q++) p[q] = sPhi[ps + (q - 3) * st];
                    double D1[6];
                    for (int q = 0; q < 6; q++) D1[q] = (p[q + 1] - p[q]) / g.h;
                    double der = vd > 0.0 ? weno5(D1[0], D1[1], D1[2], D1[3], D1[4], g.eps)
                                          : weno5(D1[5], D1[4], D1[3], D1[2], D1[1], g.eps);
                    rhs -= vd * der;
                }
                double s1 = phi0 + dt * rhs;
                phi0 = (a == 0.0) ? s1 : a * g.phiP[c] + (1.0 - a) * s1;
            }
            sL[r] = phi0;
            bool own = lx >= HL && lx < HL + TX && (D == 1 || (ly >= HL && ly < HL + TY)) && gi < g.n[0] &&
                       (D == 1 || gj < g.n[1]);
            if (own && inM) {
                for (int e = 0; e < D; e++) g.v[vout][e][c] = A[e * VN + vs];
                if (!last) po[c] = phi0;
            }
        }
        __syncthreads();
        // ---- reinitialisation on the last stage ----
        const double* fin = sL;
        if (last && K > 0) {
            double* Q = REUSE ? ((A == sA) ? sB : sA) : sQR;
            double* R = Q + LN;
            const double h = g.h, dtau = 0.5 * g.h;
            // sign changes of the stage output around tile + K + 1
            for (int r = threadIdx.x; r < LN; r += WGS) {
                int lx = r % LX, ly = r / LX;
                int ex = lx < HL ? HL - lx : (lx >= HL + TX ? lx - (HL + TX - 1) : 0);
                int ey = D == 2 ? (ly < HL ? HL - ly : (ly >= HL + TY ? ly - (HL + TY - 1) : 0)) : 0;
                sN[r] = 0;
                if (ex > K + 1 || ey > K + 1) continue;
                int sx = src_pos(g, 0, lox, lox + lx), sy = D == 2 ? src_pos(g, 1, loy, loy + ly) : 0;
                int neg = 0, pos = 0;
                for (int dy = -(D == 2); dy <= (D == 2); dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        double v = sL[(sx + dx) + LX * (sy + dy)];
                        if (v < 0.0) neg = 1; else pos = 1;
                    }
                sN[r] = (uint8_t)(neg && pos);
            }
            __syncthreads();
            const double* in = sL;
            for (int m = 1; m <= K; m++) {
                double* out = (m % 2 == 1) ? Q : R;
                int reach = K - m + 1;
                for (int r = threadIdx.x; r < LN; r += WGS) {
                    int lx = r % LX, ly = r / LX;
                    int ex = lx < HL ? HL - lx : (lx >= HL + TX ? lx - (HL + TX - 1) : 0);
                    int ey = D == 2 ? (ly < HL ? HL - ly : (ly >= HL + TY ? ly - (HL + TY - 1) : 0)) : 0;
                    if (ex > reach || ey > reach) continue;
                    int sx = src_pos(g, 0, lox, lox + lx), sy = D == 2 ? src_pos(g, 1, loy, loy + ly) : 0;
                    int rs = sx + LX * sy;
                    double pc = in[rs];
                    if (!sM[rs]) { out[r] = pc; continue; }
                    bool frz = false;
                    for (int dy = -(D == 2); dy <= (D == 2); dy++)
                        for (int dx = -1; dx <= 1; dx++) frz |= sN[rs + dx + LX * dy] != 0;
                    if (frz) { out[r] = pc; continue; }
                    double p0 = sL[rs];
                    double S = p0 / sqrt(p0 * p0 + h * h), g2 = 0.0;
                    for (int d = 0; d < D; d++) {
                        int st = d == 0 ? 1 : LX;
                        double am = (pc - in[rs - st]) / h;
                        double bp = (in[rs + st] - pc) / h;
                        double x, y;
                        if (S > 0.0) { x = am > 0.0 ? am : 0.0; y = bp < 0.0 ? bp : 0.0; }
                        else { x = am < 0.0 ? am : 0.0; y = bp > 0.0 ? bp : 0.0; }
                        g2 += (x * x > y * y) ? x * x : y * y;
                    }
                    out[r] = pc - dtau * S * (sqrt(g2) - 1.0);
                }
                __syncthreads();
                in = out;
            }
            fin = in;
        }
        if (last) {
            for (int u = threadIdx.x; u < TX * TY; u += WGS) {
                int li = u % TX, lj = u / TX;
                int i = ox + li, j = oy + lj;
                int r = (li + HL) + LX * (D == 2 ? lj + HL : 0);
                if (i < g.n[0] && (D == 1 || j < g.n[1]) && sM[r]) po[i + g.n[0] * j] = fin[r];
            }
        }
        // ---- geometry of the new level set (tile cells, padded high faces) ----
        for (int r = threadIdx.x; r < GX * GY; r += WGS) {
            int vx = r % GX, vy = r / GX;
            double sum = 0.0;
#pragma unroll
            for (int b = 0; b < (1 << D); b++) {
                int cx = HL - 1 + vx + (b & 1);
                int cy = D == 2 ? HL - 1 + vy + ((b >> 1) & 1) : 0;
                sum += fin[cx + LX * cy];
            }
            sV[r] = sum / (double)(1 << D);
        }
        // min |phi| over the tile and its one-cell halo (the mixing region)
        {
            constexpr int MX = TX + 2, MN = MX * (D == 2 ? TY + 2 : 1);
            double pmin = INFINITY;
            for (int r = threadIdx.x; r < MN; r += WGS)
                pmin = fmin(pmin, fabs(fin[(HL - 1 + r % MX) + LX * (D == 2 ? HL - 1 + r / MX : 0)]));
            for (int off = 32; off > 0; off >>= 1) pmin = fmin(pmin, __shfl_down(pmin, off, 64));
            if ((threadIdx.x & 63) == 0) sMn[threadIdx.x >> 6] = pmin;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double pmin = sMn[0];
            for (int w = 1; w < WGS / 64; w++) pmin = fmin(pmin, sMn[w]);
            tpm_out[t] = pmin;
        }
        for (int u = threadIdx.x; u < TX * TY; u += WGS) {
            int li = u % TX, lj = u / TX;
            int i = ox + li, j = oy + lj;
            if (i >= g.n[0] || (D == 2 && j >= g.n[1])) continue;
            int c = i + g.n[0] * j;
            auto V = [&](int x, int y) { return sV[(li + x) + GX * (D == 2 ? lj + y : 0)]; };
            double* apo[2] = {ap_out0, ap_out1};
            int ii[2] = {i, j};
#pragma unroll
            for (int d = 0; d < D; d++) {
                double alo, ahi;
                if (D == 1) {
                    alo = V(0, 0) < 0.0 ? 1.0 : 0.0;
                    ahi = V(1, 0) < 0.0 ? 1.0 : 0.0;
                } else if (d == 0) {
                    alo = edge_frac(V(0, 0), V(0, 1));
                    ahi = edge_frac(V(1, 0), V(1, 1));
                } else {
                    alo = edge_frac(V(0, 0), V(1, 0));
                    ahi = edge_frac(V(0, 1), V(1, 1));
                }
                apo[d][fidx(g, i, j, 0)] = alo;
                if (ii[d] == g.n[d] - 1) apo[d][fidx(g, i + (d == 0), j + (d == 1), 0)] = ahi;
            }
            double al;
            if (D == 1) {
                al = edge_frac(V(0, 0), V(1, 0));
            } else {
                double v4[4] = {V(0, 0), V(1, 0), V(1, 1), V(0, 1)};
                al = clip_area(v4);
            }
            alpha_out[c] = al;
        }
        __syncthreads();
    }
}
template <int D, int HL>
__global__ void __launch_bounds__(ExtWG<D>::V) k_lsgeo_tb(Dev g, int list, int vin, int vout, int iters,
                                                          const double* phin, double a, double dt, double* po, int K,
                                                          double* alpha_out, double* ap_out0, double* ap_out1,
                                                          double* tpm_out)
{
    b_lsgeo_tb<D, HL>(VB::grid(), g, list, vin, vout, iters, phin, a, dt, po, K, alpha_out, ap_out0, ap_out1,
                      tpm_out);
}

// ---------------------------------------------------------------------------
// initial state: cell contents alpha_k U_k of the given primitives; the
// given primitives also start every ghost state
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(SHARP_WG) k_init(Dev g, const double* prim)
{
    constexpr int NV = D + 2;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        for (int k = 0; k < 2; k++) {
            double W[NV], U[NV];
            for (int q = 0; q < NV; q++) W[q] = prim[((size_t)k * NV + q) * g.nc + c];
            prim2cons<D>(g.gam[k], g.pinf[k], W, U);
            double a = alpha_k(g, k, c);
            for (int q = 0; q < NV; q++) {
                size_t e = (size_t)q * g.nc + c;
                g.X[k][e] = a * U[q];
                g.Wb[k][0][e] = W[q];
                g.Wb[k][1][e] = W[q];
            }
        }
    }
}

// ===========================================================================
// Fused launches over the simulations of a batch.  One grid runs a kernel
// body for every simulation whose next launch it is; record r holds that
// simulation's block count, its device view (an index into `devs`) and the
// launch's other arguments, and owns blocks [pre[r], pre[r] + nblk) of the
// grid.  Shares of 8k blocks start at a multiple of 8 (the XCD mapping of
// xcd_range); the blocks in between exit at once.
// ===========================================================================
template <typename... P> struct Pack;
template <> struct Pack<> {};
template <typename H, typename... T> struct Pack<H, T...> {
    H h;
    Pack<T...> t;
};
template <typename... P> struct PackOf;
template <> struct PackOf<> {
    static Pack<> make() { return {}; }
};
template <typename H, typename... T> struct PackOf<H, T...> {
    template <typename A0, typename... A>
    static Pack<H, T...> make(A0&& a0, A&&... a)
    {
        Pack<H, T...> p;
        p.h = H(a0);
        p.t = PackOf<T...>::make(std::forward<A>(a)...);
        return p;
    }
};
template <typename... P> struct FusedRec {
    int dev;
    int nblk;
    Pack<P...> a;
};

template <auto F, typename... Done>
__device__ __forceinline__ void unpack(const VB blk, const Dev& g, const Pack<>&, Done... d)
{
    F(blk, g, d...);
}
template <auto F, typename H, typename... T, typename... Done>
__device__ __forceinline__ void unpack(const VB blk, const Dev& g, const Pack<H, T...>& p, Done... d)
{
    unpack<F>(blk, g, p.t, d..., p.h);
}

// record of block b: the last r with pre[r] <= b (pre ascending, pre[0] = 0),
// by two ballots over a wave: first over every chunk-th record, then within
// the chunk (at most 64 * 64 records)
__device__ __forceinline__ int fused_rec(const int* __restrict__ pre, int nrec, int b)
{
    const int lane = threadIdx.x & 63;
    const int chunk = (nrec + 63) >> 6;
    const int i = lane * chunk;
    unsigned long long m = __ballot(i < nrec && pre[i] <= b);
    const int base = (63 - __clzll((long long)m)) * chunk;
    const int j = base + lane;
    m = __ballot(lane < chunk && j < nrec && pre[j] <= b);
    return __builtin_amdgcn_readfirstlane(base + 63 - __clzll((long long)m));
}

template <auto F, typename... P>
__device__ __forceinline__ void fused_body(const Dev* __restrict__ devs, const FusedRec<P...>* __restrict__ recs,
                                           const int* __restrict__ pre, int nrec)
{
    const int r = fused_rec(pre, nrec, (int)blockIdx.x);
    const FusedRec<P...>& R = recs[r];
    const int b = (int)blockIdx.x - pre[r];
    if (b >= R.nblk) return;
    unpack<F>(VB{b, R.nblk}, devs[R.dev], R.a);
}
// the bounds of the kernel the body comes from: maximum block size only, or
// block size and minimum waves per SIMD
template <auto F, int WG, typename... P>
__global__ void __launch_bounds__(WG) k_fused(const Dev* __restrict__ devs, const FusedRec<P...>* __restrict__ recs,
                                              const int* __restrict__ pre, int nrec)
{
    fused_body<F, P...>(devs, recs, pre, nrec);
}
template <auto F, int WG, int WAVES, typename... P>
__global__ void __launch_bounds__(WG, WAVES) k_fused_w(const Dev* __restrict__ devs,
                                                       const FusedRec<P...>* __restrict__ recs,
                                                       const int* __restrict__ pre, int nrec)
{
    fused_body<F, P...>(devs, recs, pre, nrec);
}

// readback copy of the reduction block into a batch slot
__device__ __forceinline__ void b_red_copy(const VB blk, const Dev& g, unsigned long long* dst)
{
    for (int w = threadIdx.x; w < RED_WORDS; w += blockDim.x) dst[w] = g.red[w];
}

// ===========================================================================
// Engine: the host-side schedule of kernels for one dimension D.  It mirrors
// the method step by step: the original single-dt step and the accelerated
// cycle of Sec. 3.1 (generalised from RK2 to any Shu-Osher table).
// ===========================================================================
static const double RK3_A[3] = {0.0, 0.75, 1.0 / 3.0};
static const double RK3_C[3] = {0.0, 1.0, 0.5};
static const double RK3_B[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
static const double RK2_A[2] = {0.0, 0.5};
static const double RK2_C[2] = {0.0, 1.0};
static const double RK2_B[2] = {0.5, 0.5};

// truncation of the step ratio n (Sec. 3.1): if the fractional part of
// n = dt_slow/dt_fast is below the threshold, dt_slow is cut to floor(n) dt_fast
static void plan_cycle(double dt_slow, double dt_fast, double remaining, double thr, double* dts, int* single)
{
    double n = dt_slow / dt_fast;
    double fl = floor(n);
    double d = (n - fl < thr) ? fl * dt_fast : dt_slow;
    if (d > remaining) d = remaining;
    *dts = d;
    *single = !(d > dt_fast * (1.0 + 1e-12));
}

// next fast sub-step: stops exactly at t1 (and, for RK3, at t1/2).  Shared
// by the host and the device planner; no contraction, so both take the
// decisions with the same operations.
__host__ __device__ static double next_substep(double tau, double t1, double dt_fast, int rk, int half_done, int* hh,
                                               int* fin)
{
#pragma clang fp contract(off)
    *hh = 0;
    *fin = 0;
    double half = 0.5 * t1;
    if (rk == 3 && !half_done && tau < half) {
        if (tau + dt_fast * (1.0 + 1e-9) >= half) { *hh = 1; return half - tau; }
        return dt_fast;
    }
    if (tau + dt_fast * (1.0 + 1e-9) >= t1) { *fin = 1; return t1 - tau; }
    return dt_fast;
}

// Device planner of a fast sub-step, run right after its CFL reduction: the
// fast fluid's dt from the reduced speed, the sub-step length (truncated at
// t1/2 and t1), and the values the sub-step's first stage needs (dl, b_1 dl,
// and the slow fluid's interpolation weight for the second stage).  The host
// enqueues that first stage before it has read the plan back.
__device__ __forceinline__ void b_plan(const VB blk, const Dev& g, int F, double tau, double t1, int rk, int half_done,
                                       double cfl, double b0, double c1)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0) return;
    double m = __longlong_as_double((long long)g.red[F]);
    unsigned long long cnt = g.red[2 + F];
    double dtf = (cnt > 0 && m > 0.0) ? cfl / m : INFINITY;
    int hh = 0, fin = 0;
    double dl = NAN, th1 = NAN;
    if (isfinite(dtf) && dtf > 0.0) {
        dl = next_substep(tau, t1, dtf, rk, half_done, &hh, &fin);
        th1 = (fin && c1 == 1.0) ? 1.0 : (tau + c1 * dl) / t1;
    }
    double* sc = g.sched;
    sc[SCHED_DT] = dl;
    sc[SCHED_W0] = b0 * dl;
    sc[SCHED_TH1] = th1;
    sc[SCHED_HH] = hh;
    sc[SCHED_FIN] = fin;
    sc[SCHED_DTF] = dtf;
    sc[SCHED_CNT] = (double)cnt;
}
__global__ void k_plan(Dev g, int F, double tau, double t1, int rk, int half_done, double cfl, double b0, double c1)
{
    b_plan(VB::grid(), g, F, tau, t1, rk, half_done, cfl, b0, c1);
}

template <int D>
struct Engine {
    static constexpr int NV = D + 2;
    Sim& s;
    Dev& g;
    explicit Engine(Sim& sim) : s(sim), g(sim.g) {}

    // grid of a tile-list kernel: one block per listed tile (capped); the
    // kernels loop over the device-side count, so any grid size is correct
    // (a captured step is replayed while the lists change: its grids are
    // sized for the next power of two of the count, the graph's key)
    dim3 grid(int list, int per_tile = 1, int cap = 0) const
    {
        long long c = (long long)(s.capturing ? pow2_at_least(s.lcount[list]) : s.lcount[list]) * per_tile;
        if (cap <= 0) cap = s.max_blocks;
        if (s.o.grid_cap > 0 && cap > s.o.grid_cap) cap = s.o.grid_cap;
        if (c < 1) c = 1;
        if (c > cap) c = cap;
        return dim3((unsigned)c);
    }
    static int pow2_at_least(int n)
    {
        int p = 1;
        while (p < n && p < (1 << 30)) p <<= 1;
        return p;
    }
    dim3 wg() const { return dim3(SHARP_WG); }

    // Launch of kernel body F: the kernel `direct` on stream st or, while a
    // batch records this simulation, a record of the fused kernel with the
    // same body and bounds (WAVES: the minimum waves per SIMD of `direct`,
    // 0 when it states none)
    template <auto F, int WG, int WAVES = 0, typename... P, typename... A>
    void go(void (*direct)(Dev, P...), dim3 gr, dim3 bl, hipStream_t st, const Dev& dv, A... a)
    {
        if (s.rec) {
            record<F, WG, WAVES, P...>((int)gr.x, (int)bl.x, dv, a...);
            return;
        }
        hipLaunchKernelGGL(direct, gr, bl, 0, st, dv, P(a)...);
    }
    template <auto F, int WG, int WAVES, typename... P, typename... A>
    void record(int nblk, int block, const Dev& dv, A... a)
    {
        FusedRec<P...> r;
        r.dev = s.rec->dev_index(dv);
        r.nblk = nblk;
        r.a = PackOf<P...>::make(a...);
        const void* fn;
        if constexpr (WAVES > 0)
            fn = reinterpret_cast<const void*>(&k_fused_w<F, WG, WAVES, P...>);
        else
            fn = reinterpret_cast<const void*>(&k_fused<F, WG, P...>);
        s.rec->add(fn, block, nblk, &r, sizeof r);
    }
    // Readback of the reduction block into s.h_red: rb_begin enqueues the
    // copy (with an event when the host waits later), rb_wait waits for it.
    // Under a batch the copy goes to the simulation's slot and the wait
    // yields to the batch driver, which fills s.h_red.
    sim_status rb_begin(int words, bool event)
    {
        if (s.rec) {
            record<b_red_copy, 64, 0, unsigned long long*>(1, 64, g, s.rec->slot);
            s.rec->rb_pending = true;
            return SIM_OK;
        }
        ls_join();   // the flags of the level-set chain's kernels
        SHARP_HIP(hipMemcpyAsync(s.h_red, g.red, words * sizeof(unsigned long long), hipMemcpyDeviceToHost, s.stream));
        if (event) SHARP_HIP(hipEventRecord(s.ev_rb, s.stream));
        return SIM_OK;
    }
    sim_status rb_wait(bool event)
    {
        if (s.rec) {
            s.rec->yield(s.rec->yield_arg);
            return s.rec->status;
        }
        if (event) SHARP_HIP(hipEventSynchronize(s.ev_rb));
        else SHARP_HIP(hipStreamSynchronize(s.stream));
        return SIM_OK;
    }

    // ---- tiles and masks ----
    void mask(int list, int ring) { go<b_mask<D>, SHARP_WG>(k_mask<D>, grid(list), wg(), s.stream, g, list, ring); }
    void tiles()
    {
        int b = (g.ntiles + 255) / 256;
        go<b_tiles1<D>, 256>(k_tiles1<D>, b, 256, s.stream, g);
        go<b_tiles2<D>, 256>(k_tiles2<D>, b, 256, s.stream, g);
        go<b_compact, 1024>(k_compact, 1, 1024, s.stream, g);
    }
    // geometry of the level set `cur` into the second buffer set, which then
    // becomes current (kernels launched before keep reading the old one)
    void geom(const double* cur, int list = LIST_BAND)
    {
        Dev gn = g;
        gn.alpha = s.alpha_alt;
        for (int d = 0; d < 3; d++) gn.ap[d] = s.ap_alt[d];
        gn.tphimin = s.tphimin_alt;
        go<b_geom_lds<D>, SHARP_WG>(k_geom_lds<D>, grid(list), wg(), s.stream, gn, list, cur,
                                    static_cast<const double*>(g.tphimin));
        std::swap(g.alpha, s.alpha_alt);
        for (int d = 0; d < 3; d++) std::swap(g.ap[d], s.ap_alt[d]);
        std::swap(g.tphimin, s.tphimin_alt);
    }
    template <int HL>
    void launch_lsgeo(const double* phin, double a, double dt, double* po, int K)
    {
        if constexpr (D <= 2)
            go<b_lsgeo_tb<D, HL>, ExtWG<D>::V>(
                k_lsgeo_tb<D, HL>, grid(LIST_INNER), ExtWG<D>::V, s.stream, g, LIST_INNER, s.vcur, 1 - s.vcur,
                s.o.ext_iters, phin, a, dt, po, K, s.alpha_alt, s.ap_alt[0], s.ap_alt[1], s.tphimin_alt);
    }
    // level-set stage q (Shu-Osher coefficient a, step dt) from phin; the
    // last stage of a step reinitialises.  Returns the new level set.  With
    // `commit`, the fused path leaves the reinitialised values in phiB[2],
    // returns that buffer (read through phi_at it is the new level set) and
    // sets *commit: the caller copies it to phiP on the band-mask cells.
    const double* ls_chain(int q, bool last, double a, double dt, const double* phin,
                           const double** commit = nullptr)
    {
        if (commit) *commit = nullptr;
        if constexpr (D <= 2) {
            if (fused_ls()) {
                int K = last ? s.o.reinit_iters : -1;
                double* po = last ? g.phiB[2] : phi_stage_out(q);
                switch (K >= 1 ? K + 2 : 1) {
                case 1: launch_lsgeo<1>(phin, a, dt, po, K); break;
                case 3: launch_lsgeo<3>(phin, a, dt, po, K); break;
                default: launch_lsgeo<4>(phin, a, dt, po, K); break;
                }
                s.vcur ^= 1;
                std::swap(g.alpha, s.alpha_alt);
                for (int d = 0; d < 3; d++) std::swap(g.ap[d], s.ap_alt[d]);
                std::swap(g.tphimin, s.tphimin_alt);
                if (!last) return po;
                if (commit) { *commit = po; return po; }
                go<b_copy_masked<D>, SHARP_WG>(k_copy_masked<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, po, g.phiP);
                return g.phiP;
            }
        }
        double* po = phi_stage_out(q);
        const double* cur = po;
        if (replaying()) {
            // the recorded level set of this stage (every cell: the band
            // values the stage had and the base values elsewhere)
            double* dst = last ? g.phiP : po;
            if (last && s.stream != s.ls_stream) snap_guard(s.stream);
            (void)hipMemcpyAsync(dst, s.ls_src[s.ls_pos++], sizeof(double) * g.nc, hipMemcpyDeviceToDevice, s.stream);
            cur = dst;
        } else {
            ls(a, dt, phin, po);
            if (last) { reinit(po); cur = g.phiP; }
        }
        geom(cur);
        return cur;
    }

    // ---- band physics ----
    void prims(const double* src0, const double* src1)
    {
        go<b_prims<D>, SHARP_WG>(k_prims<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, src0, src1, s.wcur);
    }
    void extw(const double* cur)
    {
        if constexpr (D == 3) {
            // the first sweep records the targets, the others walk the list
            if (s.o.ext_iters < 1) return;
            go<b_extw<D>, SHARP_WG>(k_extw<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, s.wcur, 1 - s.wcur, cur, 1);
            s.wcur ^= 1;
            for (int it = 1; it < s.o.ext_iters; it++) {
                go<b_extw_list, SHARP_WG>(k_extw_list, grid(LIST_INNER), wg(), s.stream, g, s.wcur, 1 - s.wcur);
                s.wcur ^= 1;
            }
            return;
        }
        for (int it = 0; it < s.o.ext_iters; it++) {
            go<b_extw<D>, SHARP_WG>(k_extw<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, s.wcur, 1 - s.wcur, cur,
                                     it == 0);
            s.wcur ^= 1;
        }
    }
    void interact(double wcorr, int S, const double* cur)
    {
        go<b_interact<D>, SHARP_WG>(k_interact<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, s.wcur, s.vcur,
                                    wcorr, S, cur);
    }
    void extv(const double* cur)
    {
        if constexpr (D == 3) {
            if (s.o.ext_iters < 1) return;
            go<b_extv<D>, SHARP_WG>(k_extv<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, s.vcur, 1 - s.vcur, cur, 1);
            s.vcur ^= 1;
            for (int it = 1; it < s.o.ext_iters; it++) {
                go<b_extv_list, SHARP_WG>(k_extv_list, grid(LIST_INNER), wg(), s.stream, g, s.vcur, 1 - s.vcur);
                s.vcur ^= 1;
            }
            return;
        }
        for (int it = 0; it < s.o.ext_iters; it++) {
            go<b_extv<D>, SHARP_WG>(k_extv<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, s.vcur, 1 - s.vcur, cur,
                                     it == 0);
            s.vcur ^= 1;
        }
    }
    // primitives of both fluids on the band (real cells from src, ghost cells
    // by extension), then the interaction and the level-set velocity
    void band_state(const double* src0, const double* src1, const double* cur)
    {
        if constexpr (D <= 2) {
            if (s.o.ext_iters <= EXT_H) {
                go<b_extw_tb<D>, ExtWG<D>::W, 2 * ExtWG<D>::W / 256>(k_extw_tb<D>, grid(LIST_INNER, 2), ExtWG<D>::W,
                                                                       s.stream, g, LIST_INNER, src0, src1, s.wcur,
                                                                       1 - s.wcur, s.o.ext_iters, cur);
                s.wcur ^= 1;
                return;
            }
        }
        prims(src0, src1);
        extw(cur);
    }
    void velocity(const double* cur) { extv(cur); }
    // the velocity extension runs inside the fused level-set kernel
    bool fused_ls() const { return D <= 2 && s.o.ext_iters <= EXT_H && s.o.reinit_iters <= 2 && !replaying(); }
    // the stages take recorded level sets (frozen geometry)
    bool replaying() const { return !s.ls_src.empty(); }
    // interface interaction: ghost states, Riemann problems, and (unless a
    // fused level-set stage follows and extends it) the level-set velocity
    void interaction(const double* src0, const double* src1, const double* cur, double wcorr, int S,
                     bool ls_follows = true)
    {
        // a velocity extension left to a level-set chain that never came
        // runs before the Riemann problems overwrite its input
        if (s.vel_deferred) {
            s.vel_deferred = false;
            velocity(s.vel_cur);
        }
        band_state(src0, src1, cur);
        if constexpr (D <= 2) {
            if (s.o.ext_iters <= EXT_H) {
                go<b_riemann<D>, SHARP_WG>(k_riemann<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, s.wcur, s.vcur,
                                           wcorr, S, cur);
                if (ls_follows && fused_ls()) return;
                go<b_vext_tb<D>, ExtWG<D>::V, 2 * ExtWG<D>::V / 256>(k_vext_tb<D>, grid(LIST_INNER), ExtWG<D>::V,
                                                                       s.stream, g, LIST_INNER, s.vcur, 1 - s.vcur,
                                                                       s.o.ext_iters, cur);
                s.vcur ^= 1;
                return;
            }
        }
        interact(wcorr, S, cur);
        if (ls_follows && ls_overlap()) {
            // the level-set chain that follows extends the velocity, beside
            // the band stage
            s.vel_deferred = true;
            s.vel_cur = cur;
            return;
        }
        velocity(cur);
    }
    // ---- the level-set chain beside the band stage ----
    // A stage's level-set chain (velocity extension, advection,
    // reinitialisation, geometry) needs only the interaction's velocity and
    // writes only the level set, the velocity buffers and the second
    // geometry buffer set, none of which the band stage, the correction or
    // the bulk stage read.  So it runs on its own stream from the end of the
    // interaction (ls_fork, recorded before the stage launches) and the
    // mixing, which reads its results, waits for it (ls_join).  The stage
    // launches are issued before the chain, whose geometry buffer swap they
    // must not see.  Only a chain of several kernels (3-D, or any run
    // outside the fused 1-D/2-D level-set kernel) is moved: beside one fused
    // kernel the cross-stream events cost more than the overlap saves
    // (measured: 3-D droplet 64^3-256^3 1.5-4.5% faster per cycle, 1-D tube
    // 10% slower, 2-D 1024^2 unchanged).
    // The stream is created on first use: a process's streams share a few
    // hardware queues, and an unused one costs the runs that never overlap.
    bool ls_overlap() const
    {
        return s.side[0] && !s.rec && !s.run_serial && !s.capturing && !fused_ls();
    }
    bool ls_forked = false;
    void ls_fork()
    {
        if (!ls_overlap()) return;
        if (!s.ls_stream) {
            if (hipStreamCreateWithFlags(&s.ls_stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.ev_ls_go, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s.ev_ls_done, hipEventDisableTiming) != hipSuccess) {
                // no stream for the chain: it runs in line, as before
                (void)hipGetLastError();
                if (s.ls_stream) (void)hipStreamDestroy(s.ls_stream);
                if (s.ev_ls_go) (void)hipEventDestroy(s.ev_ls_go);
                if (s.ev_ls_done) (void)hipEventDestroy(s.ev_ls_done);
                s.ls_stream = nullptr;
                s.ev_ls_go = s.ev_ls_done = nullptr;
                return;
            }
        }
        (void)hipEventRecord(s.ev_ls_go, s.stream);
        ls_forked = true;
    }
    const double* ls_stage(int q, bool last, double a, double dt, const double* phin, const double** commit)
    {
        if (!ls_forked) {
            if (s.vel_deferred) {
                s.vel_deferred = false;
                velocity(s.vel_cur);
            }
            return ls_chain(q, last, a, dt, phin, commit);
        }
        ls_forked = false;
        (void)hipStreamWaitEvent(s.ls_stream, s.ev_ls_go, 0);
        // the last stage writes the base level set: after the cycle-start
        // copy of it (the main stream's own wait may come after the fork)
        if (last && s.snap_pending && !s.capturing) (void)hipStreamWaitEvent(s.ls_stream, s.ev_snap, 0);
        hipStream_t main = s.stream;
        s.stream = s.ls_stream;
        if (s.vel_deferred) {
            s.vel_deferred = false;
            velocity(s.vel_cur);
        }
        const double* cur = ls_chain(q, last, a, dt, phin, commit);
        s.stream = main;
        (void)hipEventRecord(s.ev_ls_done, s.ls_stream);
        s.ls_pending = true;
        return cur;
    }
    void ls_join()
    {
        if (!s.ls_pending) return;
        (void)hipStreamWaitEvent(s.stream, s.ev_ls_done, 0);
        s.ls_pending = false;
    }
    void corr_add(double w, int S)
    {
        go<b_corr_add<D>, SHARP_WG>(k_corr_add<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, w, S);
    }
    void mix(int k, double* cons, const double* cur)
    {
        go<b_mixdelta_lds<D>, SHARP_WG>(k_mixdelta_lds<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, k, cons,
                                        cur);
        go<b_mixapply<D>, SHARP_WG>(k_mixapply<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, cons);
    }
    // the band stage writes the inner tiles' output to Tm and one launch
    // mixes it into the stage buffer, optionally together with a second
    // mixed copy (the other fluid, or the slow fluid's interpolated state
    // for the next stage) and the level-set commit
    void mix_fused(const MixPart& A, const MixPart* B, const double* cur, const double* commit)
    {
        go<b_mix_parts<D>, SHARP_WG>(k_mix_parts<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, A, B ? *B : A,
                                     B ? 2 : 1, cur, commit,
                                                                commit ? g.phiP : nullptr);
    }
    MixPart tm_part(int k, double* out) const
    {
        MixPart P = {k, 1.0, g.Tm[k], 0.0, nullptr, out, 1, 0};
        return P;
    }
    void axpby(double a1, const double* s1, double a2, const double* s2, double* dst, int ncomp)
    {
        go<b_axpby<D>, SHARP_WG>(k_axpby<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, a1, s1, a2, s2, dst,
                                  ncomp);
    }

    // ---- stages ----
    // A bulk tile lies at least one tile away from every band-mask cell, so
    // its stencil (three cells) reads only bulk and ring-tile cells, which no
    // band kernel writes except the band stage.  The bulk stage of fluid k
    // therefore waits only for the previous band stage of k, and the band
    // stage only for the previous bulk stage of k (it reads that output in
    // its halo); everything in between (extension, interaction, level set,
    // geometry, mixing) overlaps with the bulk stage on its side stream.
    void stage(int k, const double* in, const double* self2, const double* base, double* out, double a, double dt,
               double wflux, int cfl = 0, double* tmp = nullptr)
    {
        int bl = k == 0 ? LIST_BULK0 : LIST_BULK1;
        const bool ov = s.side[k] != nullptr && !s.rec && !s.run_serial;
        hipStream_t bs = ov ? s.side[k] : s.stream;
        // the band stage is enqueued first: on the critical path, it takes the
        // CUs before the bulk stage fills them
        hipEvent_t prev_band = nullptr;
        if (ov) {
            if (s.bulk_pending[k]) (void)hipStreamWaitEvent(s.stream, s.ev_bulk[k], 0);
            prev_band = s.band_rec[k] ? s.ev_band[k] : nullptr;
        }
        if (out == g.X[k]) snap_guard(s.stream);
        launch_stage<true>(s.stream, LIST_BAND, k, in, self2, base, out, a, dt, wflux, 0, tmp);
        if (ov) {
            if (g.use_sched) {
                // a planned stage: the bulk kernel reads its step from the plan,
                // so it waits for everything enqueued so far (the planner)
                (void)hipEventRecord(s.ev_band[k], s.stream);
                (void)hipStreamWaitEvent(bs, s.ev_band[k], 0);
            } else if (prev_band) {
                // the bulk stage reads ring-tile cells of `in`, written by the
                // previous band stage
                (void)hipStreamWaitEvent(bs, prev_band, 0);
            }
        }
        if (cfl) go<b_zero_red, 64>(k_zero_red, 1, 64, bs, g);
        size_t ev = 0;
        if (s.prof) {
            if (s.ev_used + 2 > s.ev_pool.size()) profile_flush();
            ev = s.ev_used;
            s.ev_used += 2;
        }
        if (out == g.X[k]) snap_guard(bs);
        launch_stage<false>(bs, bl, k, in, nullptr, base, out, a, dt, wflux, cfl, nullptr,
                            s.prof ? s.ev_pool[ev] : nullptr, s.prof ? s.ev_pool[ev + 1] : nullptr);
        if (s.prof) {
            // cells this launch advances by one stage; the first stage of a
            // step (a == 0) reads no base state
            s.prof_cells.push_back(a == 0.0 ? -s.bulk_cells[k] : s.bulk_cells[k]);
        }
        if (ov) {
            (void)hipEventRecord(s.ev_bulk[k], bs);
            s.bulk_pending[k] = true;
            if (!g.use_sched) (void)hipEventRecord(s.ev_band[k], s.stream);
            s.band_rec[k] = true;
        }
        fused_cfl = cfl;
    }
    // order the outstanding bulk stages before what follows on the stream
    void join()
    {
        ls_join();
        for (int k = 0; k < 2; k++)
            if (s.bulk_pending[k]) {
                (void)hipStreamWaitEvent(s.stream, s.ev_bulk[k], 0);
                s.bulk_pending[k] = false;
            }
    }
    bool fused_cfl = false;    // the last bulk stage already reduced the fast fluid's CFL speed
    template <bool BAND>
    // e0, e1 (optional): events stamped by the dispatch itself at the start
    // and end of the kernel's execution
    void launch_stage(hipStream_t st, int list, int k, const double* in, const double* self2, const double* base,
                      double* out, double a, double dt, double wflux, int cfl, double* tmp,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
    {
        dim3 gr = grid(list, 1, BAND ? 0 : s.bulk_blocks);
        if (s.rec) {
            if constexpr (D <= 2)
                record<b_stage_lds<D, BAND>, StageWG<D>::N, 0, int, int, const double*, const double*, const double*,
                       double*, double, double, double, int, int, double*>((int)gr.x, StageWG<D>::N, g, list, k, in,
                                                                            self2, base, out, a, dt, wflux, s.wcur,
                                                                            cfl, tmp);
            else
                record<b_stage_lds3<BAND>, SHARP_WG3, SHARP_WG3_WAVES, int, int, const double*, const double*,
                       const double*, double*, double, double, double, int, int, double*>(
                    (int)gr.x, SHARP_WG3, g, list, k, in, self2, base, out, a, dt, wflux, s.wcur, cfl, tmp);
            return;
        }
        if (!e0 && !e1) {
            if constexpr (D <= 2)
                k_stage_lds<D, BAND><<<gr, dim3(StageWG<D>::N), 0, st>>>(g, list, k, in, self2, base, out, a, dt, wflux,
                                                                        s.wcur, cfl, tmp);
            else
                k_stage_lds3<BAND><<<gr, dim3(SHARP_WG3), 0, st>>>(g, list, k, in, self2, base, out, a, dt, wflux, s.wcur,
                                                                  cfl, tmp);
            return;
        }
        if constexpr (D <= 2)
            hipExtLaunchKernelGGL(k_stage_lds<D, BAND>, gr, dim3(StageWG<D>::N), 0, st, e0, e1, 0, g, list, k, in,
                                  self2, base, out, a, dt, wflux, s.wcur, cfl, tmp);
        else
            hipExtLaunchKernelGGL(k_stage_lds3<BAND>, gr, dim3(SHARP_WG3), 0, st, e0, e1, 0, g, list, k, in, self2,
                                  base, out, a, dt, wflux, s.wcur, cfl, tmp);
    }
    void profile_flush()
    {
        (void)hipStreamSynchronize(s.stream);
        for (int k = 0; k < 2; k++)
            if (s.side[k]) (void)hipStreamSynchronize(s.side[k]);
        for (size_t e = 0; e + 1 < s.ev_used; e += 2) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, s.ev_pool[e], s.ev_pool[e + 1]);
            s.prof_ms += ms;
            s.prof_launches++;
            long long c = s.prof_cells[e / 2];
            s.prof_cell_stages += c < 0 ? -c : c;
            if (c < 0) s.prof_first_stages += -c;
        }
        s.ev_used = 0;
        s.prof_cells.clear();
    }

    // level-set stage buffers: stage outputs alternate B0, B1; reinitialisation
    // iterates through the free buffers and ends in the base buffer P
    double* phi_stage_out(int st) { return g.phiB[st % 2]; }
    void reinit(double* phi0)
    {
        int K = s.o.reinit_iters;
        if (K <= 0) {
            go<b_copy_masked<D>, SHARP_WG>(k_copy_masked<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, phi0,
                                           g.phiP);
            return;
        }
        go<b_nearif<D>, SHARP_WG>(k_nearif<D>, grid(LIST_BAND), wg(), s.stream, g, LIST_BAND, phi0);
        double* other = (phi0 == g.phiB[0]) ? g.phiB[1] : g.phiB[0];
        const double* in = phi0;
        for (int m = 1; m <= K; m++) {
            double* out = (m == K) ? g.phiP : ((m % 2 == 1) ? g.phiB[2] : other);
            go<b_reinit<D>, SHARP_WG>(k_reinit<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, phi0, in, out);
            in = out;
        }
    }
    void ls(double a, double dt, const double* in, double* out)
    {
        go<b_ls<D>, SHARP_WG>(k_ls<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, a, dt, in, out, s.vcur);
    }

    // ---- rollback snapshot ----
    // Taken at a cycle start once the readback of that start has found the
    // state physical: the boundary ledger in stream order (every stage adds
    // to it), the contents and the level set on the snapshot stream, beside
    // the cycle's first stages (which write stage buffers only).  Every
    // kernel that writes X or phiP waits for the copies first (snap_guard).
    // Under the serial schedule the copies run on the stream.
    sim_status snap_begin(const sim_stats* st)
    {
        s.snap_valid = false;
        s.snap_pending = false;
        if (!s.snapPhi || s.rec || s.capturing) return SIM_OK;
        const size_t nv = (size_t)NV * g.nc, nb = (size_t)NV * (g.nbface > 0 ? g.nbface : 1);
        for (int k = 0; k < 2; k++)
            SHARP_HIP(hipMemcpyAsync(s.snapBacc[k], g.bacc[k], nb * sizeof(double), hipMemcpyDeviceToDevice, s.stream));
        const bool own = !s.run_serial && !s.o.serial;
        hipStream_t cs = s.stream;
        if (own) {
            if (!s.snap_stream) SHARP_HIP(hipStreamCreateWithFlags(&s.snap_stream, hipStreamNonBlocking));
            SHARP_HIP(hipEventRecord(s.ev_cs, s.stream));
            SHARP_HIP(hipStreamWaitEvent(s.snap_stream, s.ev_cs, 0));
            cs = s.snap_stream;
        }
        for (int k = 0; k < 2; k++)
            SHARP_HIP(hipMemcpyAsync(s.snapX[k], g.X[k], nv * sizeof(double), hipMemcpyDeviceToDevice, cs));
        SHARP_HIP(hipMemcpyAsync(s.snapPhi, g.phiP, (size_t)g.nc * sizeof(double), hipMemcpyDeviceToDevice, cs));
        if (own) {
            SHARP_HIP(hipEventRecord(s.ev_snap, cs));
            s.snap_pending = true;
            for (bool& w : s.snap_waited) w = false;
        }
        s.snap_t = s.t;
        s.snap_stats = *st;
        s.snap_valid = true;
        return SIM_OK;
    }
    // order the next writer of X or phiP on stream st after the snapshot
    void snap_guard(hipStream_t st)
    {
        if (!s.snap_pending || s.capturing) return;
        const int i = (s.side[0] && st == s.side[0]) ? 1 : ((s.side[1] && st == s.side[1]) ? 2 : 0);
        if (s.snap_waited[i]) return;
        (void)hipStreamWaitEvent(st, s.ev_snap, 0);
        s.snap_waited[i] = true;
    }
    // back to the snapshot: contents, level set, boundary ledger, time and
    // the call's statistics; the geometry, band and tile lists are rebuilt
    // from the level set as sim_set_state builds them
    sim_status rollback(sim_stats* st)
    {
        join();
        s.vel_deferred = false;
        if (s.ls_stream) SHARP_HIP(hipStreamSynchronize(s.ls_stream));
        for (int k = 0; k < 2; k++)
            if (s.side[k]) SHARP_HIP(hipStreamSynchronize(s.side[k]));
        if (s.snap_stream) SHARP_HIP(hipStreamSynchronize(s.snap_stream));
        SHARP_HIP(hipStreamSynchronize(s.stream));
        s.snap_pending = false;
        const size_t nb = (size_t)NV * (g.nbface > 0 ? g.nbface : 1);
        for (int k = 0; k < 2; k++)
            SHARP_HIP(hipMemcpyAsync(g.bacc[k], s.snapBacc[k], nb * sizeof(double), hipMemcpyDeviceToDevice, s.stream));
        sim_status rc = restore_state(s.snapX[0], s.snapX[1], s.snapPhi);
        if (rc != SIM_OK) return rc;
        s.t = s.snap_t;
        *st = s.snap_stats;
        s.rollbacks++;
        if (s.o.tape && s.tape_fluid >= 0) {
            s.tape_fluid = -1;
            s.tape_why = "a step turned non-physical and the state was rolled back";
        }
        return SIM_OK;
    }
    // contents and level set from device copies; the geometry, band and
    // tile lists rebuilt from the level set as sim_set_state builds them
    sim_status restore_state(const double* X0, const double* X1, const double* phi)
    {
        const size_t nv = (size_t)NV * g.nc;
        SHARP_HIP(hipMemcpyAsync(g.X[0], X0, nv * sizeof(double), hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(hipMemcpyAsync(g.X[1], X1, nv * sizeof(double), hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(hipMemcpyAsync(g.phiP, phi, (size_t)g.nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream));
        s.lcount[LIST_ALL] = g.ntiles;
        geom(g.phiP, LIST_ALL);
        geom(g.phiP, LIST_ALL);
        mask(LIST_ALL, 0);
        tiles();
        SHARP_HIP(reset_flags());
        SHARP_HIP(hipMemcpyAsync(s.h_red, g.red, RED_WORDS * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 s.stream));
        SHARP_HIP(hipStreamSynchronize(s.stream));
        take_counts();
        return SIM_OK;
    }
    // one single-dt step of length dt from the current state (the stage
    // level sets from s.ls_src), its stages recorded to *rec; `prepared`:
    // the step-start interaction's results (primitives, interface solution)
    // are already in place, restored with the state
    sim_status replay_step(double dt, StageRec* rec, bool prepared)
    {
        double d[2];
        long long cnt[2];
        s.stage_rec = rec;
        sim_status rc = prepared ? SIM_OK : prepare(true, d, cnt);
        if (rc == SIM_OK) {
            step_single(dt);
            join();
        }
        s.stage_rec = nullptr;
        return rc;
    }
    // ---- single operations of the adjoint's composed forward ----
    sim_status op_prepare()
    {
        double d[2];
        long long cnt[2];
        return prepare(true, d, cnt);
    }
    void op_corr_apply(int S)
    {
        go<b_corr_apply<D>, SHARP_WG>(k_corr_apply<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, S, 1);
    }
    void op_axpby_all(double a1, const double* x, double a2, const double* y, double* dst)
    {
        go<b_axpby<D>, SHARP_WG>(k_axpby<D>, grid(LIST_ALL), wg(), s.stream, g, LIST_ALL, a1, x, a2, y, dst, NV);
    }
    // reductions and error flags to zero, no non-physical cell recorded
    hipError_t reset_flags()
    {
        hipError_t e = hipMemsetAsync(g.red, 0, 8 * sizeof(unsigned long long), s.stream);
        if (e == hipSuccess) e = hipMemsetAsync(g.red + RED_CELL, 0xff, sizeof(unsigned long long), s.stream);
        return e;
    }

    // ---- CFL ----
    void cfl_launch(int k, const double* cons)
    {
        int bl = k == 0 ? LIST_BULK0 : LIST_BULK1;
        go<b_cfl<D, false>, SHARP_WG>(k_cfl<D, false>, grid(bl), wg(), s.stream, g, bl, k, cons, s.wcur);
        go<b_cfl<D, true>, SHARP_WG>(k_cfl<D, true>, grid(LIST_BAND), wg(), s.stream, g, LIST_BAND, k, cons, s.wcur);
    }
    // read back the reductions; fills dt and active-cell counts of the fluids in `which`
    // list counts and error flags of a completed readback
    sim_status check_flags()
    {
        take_counts();
        unsigned long long err = s.h_red[4];
        if (err & ERR_BAND_OVERFLOW) { set_error("the interface band left its tile set within a cycle"); return SIM_EDEVICE; }
        if (err & ERR_NONPHYS) { nonphys_error(); return SIM_ENONPHYS; }
        return SIM_OK;
    }
    // message of a non-physical state, naming the cell the kernels recorded
    void nonphys_error()
    {
        const unsigned long long code = s.h_red[RED_CELL];
        if (code == ~0ull) {
            set_error("non-physical state (rho <= 0, p + p_inf <= 0 or NaN)");
            return;
        }
        const int c = (int)(code >> 1), k = (int)(code & 1);
        const int i = c % g.n[0], j = (c / g.n[0]) % g.n[1], kk = c / (g.n[0] * g.n[1]);
        set_error("non-physical state (rho <= 0, p + p_inf <= 0 or NaN) of fluid %d in cell %d (i %d, j %d, k %d)", k,
                  c, i, j, kk);
    }
    sim_status readback(int which, double* dt, long long* cnt)
    {
        sim_status rc = rb_begin(RED_WORDS, false);
        if (rc == SIM_OK) rc = rb_wait(false);
        if (rc == SIM_OK) rc = check_flags();
        if (rc != SIM_OK) return rc;
        for (int k = 0; k < 2; k++) {
            if (!(which & (1 << k))) continue;
            double m = __longlong_as_double_host(s.h_red[k]);
            cnt[k] = (long long)s.h_red[2 + k];
            dt[k] = (cnt[k] > 0 && m > 0.0) ? s.o.cfl / m : INFINITY;
        }
        return SIM_OK;
    }
    // The CFL steps of a (sub)step start (fluid 0 before fluid 1): the
    // prescribed ones when the simulation replays a schedule; every step
    // taken goes to the schedule log
    sim_status take_cfl(int which, double* dt)
    {
        for (int k = 0; k < 2; k++) {
            if (!(which & (1 << k))) continue;
            if (!s.dt_replay.empty()) {
                if (s.replay_pos >= s.dt_replay.size()) {
                    set_error("dt_replay exhausted after %zu steps", s.replay_pos);
                    return SIM_EINVAL;
                }
                dt[k] = s.dt_replay[s.replay_pos++];
            }
            s.dt_log.push_back(dt[k]);
        }
        return SIM_OK;
    }
    void take_counts()
    {
        const int* cc = reinterpret_cast<const int*>(s.h_red + RED_COUNTS);
        for (int l = 0; l < 4; l++) s.lcount[l] = cc[l];
        s.lcount[LIST_INNER] = cc[LIST_INNER];
        s.lcount[LIST_ALL] = g.ntiles;
        s.bulk_cells[0] = cc[8 + 2];
        s.bulk_cells[1] = cc[8 + 3];
    }
    static double __longlong_as_double_host(unsigned long long b)
    {
        double d;
        std::memcpy(&d, &b, sizeof d);
        return d;
    }

    // ---- (sub)step start: band mask, primitives, extension, interaction, CFL ----
    sim_status prepare(bool cycle_start, double* dt, long long* cnt)
    {
        if (cycle_start) {
            mask(LIST_CAND, 0);
            tiles();
        }
        interaction(g.X[0], g.X[1], g.phiP, 0.0, 0);
        go<b_zero_red, 64>(k_zero_red, 1, 64, s.stream, g);
        cfl_launch(0, g.X[0]);
        cfl_launch(1, g.X[1]);
        return readback(3, dt, cnt);
    }

    // ---- the original method: one dt for both fluids and the level set ----
    int fill_blocks() const
    {
        int b = (g.nc + 255) / 256;
        return b > 65535 ? 65535 : b;
    }
    // the stage record of a replayed step: what the stage's interaction saw
    void rec_in(const double* const* in, const double* phin)
    {
        StageRec& r = *s.stage_rec;
        double* b = r.base + (size_t)r.next * r.stride;
        const size_t nv = (size_t)NV * g.nc, nc = (size_t)g.nc;
        for (int k = 0; k < 2; k++) {
            (void)hipMemcpyAsync(b + r.in[k], in[k], nv * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
            (void)hipMemcpyAsync(b + r.W[k], g.Wb[k][s.wcur], nv * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
        }
        (void)hipMemcpyAsync(b + r.ps, g.ps, nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
        (void)hipMemcpyAsync(b + r.us, g.us, nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
        (void)hipMemcpyAsync(b + r.al, g.alpha, nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
        for (int d = 0; d < D; d++)
            (void)hipMemcpyAsync(b + r.ap + (size_t)d * g.nfc, g.ap[d], (size_t)g.nfc * sizeof(double),
                                 hipMemcpyDeviceToDevice, s.stream);
        k_phi_merge<<<fill_blocks(), 256, 0, s.stream>>>(g, phin, b + r.phi);
        (void)hipMemcpyAsync(b + r.M, g.M, nc, hipMemcpyDeviceToDevice, s.stream);
    }
    // ... and the geometry its mixing used
    void rec_out(const double* cur)
    {
        StageRec& r = *s.stage_rec;
        double* b = r.base + (size_t)r.next * r.stride;
        (void)hipMemcpyAsync(b + r.aln, g.alpha, (size_t)g.nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
        k_phi_merge<<<fill_blocks(), 256, 0, s.stream>>>(g, cur, b + r.phin);
        r.next++;
    }
    void step_single(double dt)
    {
        int ns = s.o.rk;
        const double* A = ns == 3 ? RK3_A : RK2_A;
        const double* B = ns == 3 ? RK3_B : RK2_B;
        const double* in[2] = {g.X[0], g.X[1]};
        const double* phin = g.phiP;
        for (int st = 0; st < ns; st++) {
            if (st > 0) interaction(in[0], in[1], phin, 0.0, 0);
            if (s.stage_rec) rec_in(in, phin);
            ls_fork();
            double* out[2];
            for (int k = 0; k < 2; k++) {
                out[k] = (st == ns - 1) ? g.X[k] : (st == 0 ? g.Y[k] : g.Z[k]);
                stage(k, in[k], nullptr, g.X[k], out[k], A[st], dt, B[st] * dt, 0, g.Tm[k]);
            }
            const double* commit = nullptr;
            const double* cur = ls_stage(st, st == ns - 1, A[st], dt, phin, &commit);
            ls_join();
            if (s.stage_rec) rec_out(cur);
            else if (s.tape_fluid == 2 && !s.tape_ls.empty())
                k_phi_merge<<<fill_blocks(), 256, 0, s.stream>>>(g, cur, s.tape_ls.back() + (size_t)st * g.nc);
            MixPart m1 = tm_part(1, out[1]);
            mix_fused(tm_part(0, out[0]), &m1, cur, commit);
            if (commit) cur = g.phiP;
            in[0] = out[0];
            in[1] = out[1];
            phin = cur;
        }
        join();
        s.t += dt;
    }

    // ---- captured single-dt steps and prescribed accelerated cycles (o.graph) ----
    // A step of the fixed length dt_fixed (its start: band tiles,
    // interaction, CFL reductions; then the stages) issues the same launches
    // whenever the host state they are made from is the same: the device
    // view (its geometry buffers alternate), the Jacobi buffer parities and
    // the grid sizes.  Such a step is captured once into a HIP graph and
    // replayed; the kernels read every count from the device, so a replay
    // gives the results of the launches it recorded.  The capture issues
    // every kernel on the one stream (a graph with the bulk stages on side
    // streams and the events between them ran slower than the launches it
    // replaces).  A run of whole steps is enqueued without waiting for any of
    // them: the active-cell counts are summed on the device and read back,
    // with the error flags, once at the end of the run.  Under graph = 1
    // only grids of at most SIM_GRAPH_MAX_CELLS cells (accelerated cycles:
    // SIM_GRAPH_MAX_CELLS_CYCLE) are captured: above
    // that the side-stream overlap of the bulk stages, which the graph gives
    // up, is worth more than the launch latency it saves.
    bool graph_run_ok(bool cycles = false) const
    {
        const long long cap = cycles ? SIM_GRAPH_MAX_CELLS_CYCLE : SIM_GRAPH_MAX_CELLS;
        const bool size_ok = s.o.graph == 2 || (s.o.graph == 1 && (long long)g.nc <= cap);
        return size_ok && (cycles ? fixed_multi() : s.o.dt_fixed > 0.0) && !s.rec && !s.prof && !s.o.tape &&
               !replaying() && (!s.o.autotune || s.tune_cur >= Sim::NTUNE);
    }
    // accelerated cycles with prescribed steps of both fluids
    bool fixed_multi() const { return s.o.dt_fixed_fluid[0] > 0.0 && s.o.dt_fixed_fluid[1] > 0.0; }
    static void put(std::vector<unsigned char>& v, const void* p, size_t n)
    {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        v.insert(v.end(), b, b + n);
    }
    // the host state a step changes
    std::vector<unsigned char> step_state() const
    {
        std::vector<unsigned char> v;
        put(v, &g, sizeof g);
        put(v, &s.wcur, sizeof s.wcur);
        put(v, &s.vcur, sizeof s.vcur);
        put(v, &s.alpha_alt, sizeof s.alpha_alt);
        put(v, s.ap_alt, sizeof s.ap_alt);
        return v;
    }
    void set_step_state(const std::vector<unsigned char>& v)
    {
        size_t o = 0;
        auto get = [&](void* p, size_t n) {
            std::memcpy(p, v.data() + o, n);
            o += n;
        };
        get(&g, sizeof g);
        get(&s.wcur, sizeof s.wcur);
        get(&s.vcur, sizeof s.vcur);
        get(&s.alpha_alt, sizeof s.alpha_alt);
        get(s.ap_alt, sizeof s.ap_alt);
    }
    // ... and, with what else sizes or orders the launches, the graph's key
    std::vector<unsigned char> launch_key(double d) const
    {
        std::vector<unsigned char> v = step_state();
        put(v, &s.bulk_blocks, sizeof s.bulk_blocks);
        put(v, &s.max_blocks, sizeof s.max_blocks);
        for (int l = 0; l < NLISTS; l++) {
            int c = pow2_at_least(s.lcount[l]);
            put(v, &c, sizeof c);
        }
        put(v, &d, sizeof d);
        return v;
    }
    // the launches of one whole step, as the uncaptured path issues them
    void graph_step_body(double d)
    {
        mask(LIST_CAND, 0);
        tiles();
        interaction(g.X[0], g.X[1], g.phiP, 0.0, 0);
        go<b_zero_red, 64>(k_zero_red, 1, 64, s.stream, g);
        cfl_launch(0, g.X[0]);
        cfl_launch(1, g.X[1]);
        go<b_acc, 64>(k_acc, 1, 64, s.stream, g, 15);
        step_single(d);
    }
    // ... and of one whole accelerated cycle with the prescribed steps: the
    // same start, then the cycle, whose fast sub-steps add the fast fluid's
    // counts on the device instead of reading them back; cs gets the
    // cycle's step counts
    void graph_cycle_body(sim_stats* cs)
    {
        mask(LIST_CAND, 0);
        tiles();
        interaction(g.X[0], g.X[1], g.phiP, 0.0, 0);
        go<b_zero_red, 64>(k_zero_red, 1, 64, s.stream, g);
        cfl_launch(0, g.X[0]);
        cfl_launch(1, g.X[1]);
        go<b_acc, 64>(k_acc, 1, 64, s.stream, g, 15);
        const long long cnt[2] = {0, 0};
        (void)cycle(s.o.dt_fixed_fluid, cnt, INFINITY, cs);
    }
    // capture of the launches `body` issues (one whole step or cycle) into
    // a graph under `key`; the graph keeps the host state after it, the
    // time it advances and the steps each fluid takes in it
    template <typename Body>
    sim_status capture(std::vector<unsigned char>&& key, Body body, const char* what)
    {
        if (!s.cap_stream) SHARP_HIP(hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking));
        if (s.graphs.size() >= Sim::MAX_GRAPHS) {
            (void)hipGraphExecDestroy(s.graphs.front().exec);
            s.graphs.erase(s.graphs.begin());
        }
        // what the uncaptured path put on the side streams was joined into
        // the stream before the graphs that follow it
        if (s.vel_deferred) {
            s.vel_deferred = false;
            velocity(s.vel_cur);
        }
        join();
        for (int k = 0; k < 2; k++) s.band_rec[k] = false;
        const std::vector<unsigned char> before = step_state();
        hipStream_t user = s.stream;
        const double t0 = s.t;
        const bool serial = s.run_serial;
        SHARP_HIP(hipStreamBeginCapture(s.cap_stream, hipStreamCaptureModeThreadLocal));
        s.stream = s.cap_stream;
        s.capturing = true;
        s.run_serial = true;
        sim_stats cs;
        std::memset(&cs, 0, sizeof cs);
        cycle_adv = 0.0;
        body(&cs);
        hipGraph_t graph = nullptr;
        hipError_t e = hipSuccess;
        hipError_t e2 = hipStreamEndCapture(s.cap_stream, &graph);
        s.stream = user;
        s.capturing = false;
        s.run_serial = serial;
        s.t = t0;
        for (int k = 0; k < 2; k++) {
            s.band_rec[k] = false;
            s.bulk_pending[k] = false;
        }
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess && e2 == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            set_step_state(before);
            set_error("capture of %s failed: %s", what, hipGetErrorString(e != hipSuccess ? e : e2));
            return SIM_EDEVICE;
        }
        Sim::StepGraph sg;
        sg.key = std::move(key);
        sg.after = step_state();
        sg.exec = exec;
        sg.adv = cycle_adv;
        sg.steps[0] = cs.steps[0];
        sg.steps[1] = cs.steps[1];
        sg.last_n = cs.last_n;
        set_step_state(before);
        s.graphs.push_back(std::move(sg));
        s.graph_captures++;
        return SIM_OK;
    }
    // K whole steps of length dt_fixed from graphs, then one readback
    sim_status graph_steps(long long K, double t_end, sim_stats* st)
    {
        const double d = s.o.dt_fixed;
        join();
        snap_guard(s.stream);
        go<b_acc, 64>(k_acc, 1, 64, s.stream, g, 0);
        for (long long i = 0; i < K; i++) {
            std::vector<unsigned char> key = launch_key(d);
            int found = -1;
            for (size_t j = 0; j < s.graphs.size(); j++)
                if (s.graphs[j].key == key) found = (int)j;
            if (found < 0) {
                sim_status rc = capture(std::move(key), [&](sim_stats*) { graph_step_body(d); }, "a single-dt step");
                if (rc != SIM_OK) return rc;
                found = (int)s.graphs.size() - 1;
            }
            SHARP_HIP(hipGraphLaunch(s.graphs[found].exec, s.stream));
            set_step_state(s.graphs[found].after);
            s.t += d;
            if (t_end - s.t <= 1e-14 * t_end) s.t = t_end;
            s.graph_replays++;
        }
        sim_status rc = rb_begin(RED_WORDS, false);
        if (rc == SIM_OK) rc = rb_wait(false);
        if (rc == SIM_OK) rc = check_flags();
        if (rc != SIM_OK) return rc;
        if ((long long)s.h_red[7] != K) {
            set_error("captured steps: %lld of %lld ran", (long long)s.h_red[7], K);
            return SIM_EDEVICE;
        }
        for (int k = 0; k < 2; k++) {
            double m = __longlong_as_double_host(s.h_red[k]);
            long long cnt = (long long)s.h_red[2 + k];
            st->last_dt[k] = (cnt > 0 && m > 0.0) ? s.o.cfl / m : INFINITY;
            st->steps[k] += K;
            st->cell_updates[k] += (long long)s.h_red[5 + k];
            st->active_cells[k] = cnt;
        }
        st->cycles += K;
        st->last_n = 1.0;
        if (!(fmin(st->last_dt[0], st->last_dt[1]) > 0.0)) {
            set_error("invalid time step");
            return SIM_ENONPHYS;
        }
        return SIM_OK;
    }

    // K whole accelerated cycles with the prescribed steps, from graphs, then
    // one readback (the cycle of Sec. 3.1 with its sub-step plan fixed by
    // the prescribed steps: the launches of every cycle are the same)
    sim_status graph_cycles(long long K, sim_stats* st)
    {
        const double* dt = s.o.dt_fixed_fluid;
        const char tag = 'C';
        join();
        snap_guard(s.stream);
        go<b_acc, 64>(k_acc, 1, 64, s.stream, g, 0);
        int last = -1;
        for (long long i = 0; i < K; i++) {
            std::vector<unsigned char> key = launch_key(dt[0]);
            put(key, &dt[1], sizeof dt[1]);
            put(key, &tag, 1);
            int found = -1;
            for (size_t j = 0; j < s.graphs.size(); j++)
                if (s.graphs[j].key == key) found = (int)j;
            if (found < 0) {
                sim_status rc = capture(std::move(key), [&](sim_stats* cs) { graph_cycle_body(cs); },
                                        "an accelerated cycle");
                if (rc != SIM_OK) return rc;
                found = (int)s.graphs.size() - 1;
            }
            const Sim::StepGraph& G = s.graphs[found];
            SHARP_HIP(hipGraphLaunch(G.exec, s.stream));
            set_step_state(G.after);
            s.t += G.adv;
            for (int k = 0; k < 2; k++) st->steps[k] += G.steps[k];
            st->last_n = G.last_n;
            last = found;
            s.graph_replays++;
        }
        sim_status rc = rb_begin(RED_WORDS, false);
        if (rc == SIM_OK) rc = rb_wait(false);
        if (rc == SIM_OK) rc = check_flags();
        if (rc != SIM_OK) return rc;
        if ((long long)s.h_red[7] != K) {
            set_error("captured cycles: %lld of %lld ran", (long long)s.h_red[7], K);
            return SIM_EDEVICE;
        }
        (void)last;
        for (int k = 0; k < 2; k++) {
            st->last_dt[k] = dt[k];
            st->cell_updates[k] += (long long)s.h_red[5 + k];
            st->active_cells[k] = (long long)s.h_red[9 + k];
        }
        st->cycles += K;
        return SIM_OK;
    }

    // slow fluid's intermediate state, Eq. (interpolation), mixed with the
    // current geometry unless it is the (already mixed) previous state
    MixPart interp_part(int S, double theta) const
    {
        MixPart P = {S, 1.0 - theta, g.X[S], theta, g.Y[S], g.T2, theta != 0.0, 0};
        return P;
    }
    void interp_slow(int S, double theta, const double* cur)
    {
        go<b_mixinterp_lds<D>, SHARP_WG>(k_mixinterp_lds<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER,
                                          interp_part(S, theta), cur);
    }
    // copy of src mixed with the current geometry
    void mixed_copy(int S, const double* src, const double* cur)
    {
        MixPart P = {S, 1.0, src, 0.0, nullptr, g.T2, 1, 0};
        go<b_mixinterp_lds<D>, SHARP_WG>(k_mixinterp_lds<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, P, cur);
    }

    // ---- the accelerated cycle (Sec. 3.1) ----
    double cycle_adv = 0.0;    // the time the last cycle advanced
    sim_status cycle(const double* dt, const long long* cnt, double t_end, sim_stats* st)
    {
        int ns = s.o.rk;
        const double* A = ns == 3 ? RK3_A : RK2_A;
        const double* C = ns == 3 ? RK3_C : RK2_C;
        const double* B = ns == 3 ? RK3_B : RK2_B;
        int S = dt[0] >= dt[1] ? 0 : 1, F = 1 - S;
        double dtS, rem = t_end - s.t;
        int single;
        if (!std::isfinite(dt[F])) { S = F; F = 1 - S; }
        if (!std::isfinite(dt[S]) || !std::isfinite(dt[F])) {
            double d = dt[0] < dt[1] ? dt[0] : dt[1];
            if (d > rem) d = rem;
            single = 1;
            dtS = d;
        } else {
            plan_cycle(dt[S], dt[F], rem, s.o.n_thr, &dtS, &single);
            if (single && s.o.force_cycle && dtS >= dt[F] * (1.0 - 1e-12)) single = 0;
        }
        const bool taped = s.o.tape && s.tape_fluid == 2 && !s.stage_rec;
        if (single) {
            if (taped) {
                sim_status rc = tape_step(s, dtS);
                if (rc != SIM_OK) return rc;
            }
            cycle_adv = dtS;
            step_single(dtS);
            st->cycles++;
            for (int k = 0; k < 2; k++) { st->steps[k]++; st->cell_updates[k] += cnt[k]; }
            st->last_n = 1.0;
            return SIM_OK;
        }
        const bool corr = !s.o.no_correction;
        double t1 = dtS;
        st->last_n = t1 / dt[F];
        if (taped) {
            sim_status rc = tape_cycle(s, S, t1);
            if (rc != SIM_OK) return rc;
        }
        // (1) slow fluid's first stage with dt_S on the cycle-start interaction
        stage(S, g.X[S], nullptr, g.X[S], g.Y[S], A[0], t1, B[0] * t1);
        double tau = 0.0, dtF = dt[F];
        int first = 1, half_done = 0;
        long long cntF = cnt[F];
        // One stage q of a fast sub-step of length dl.  With `planned` (the
        // first stage of a sub-step planned on the device), dl, b_1 dl and the
        // next interpolation weight are read by the kernels from the device
        // plan (Dev::use_sched) and the host arguments are placeholders.
        auto fast_stage = [&](int q, const double*& in, const double*& phin, double dl, int fin, bool planned) {
            bool shared = false;
            if (q > 0) {
                // the slow fluid's interpolated state for this stage was
                // built by the previous stage's mixing launch
                shared = fin && C[q] == 1.0;
                double w = !corr ? 0.0 : (shared ? -B[q] * t1 + B[q] * dl : B[q] * dl);
                interaction(S == 0 ? g.T2 : in, S == 0 ? in : g.T2, phin, w, S);
            }
            ls_fork();
            if (shared) {
                // shared with the slow fluid's second stage, Eq. (firstcorrection)
                stage(S, g.Y[S], g.T2, g.X[S], ns == 2 ? g.X[S] : g.Z[S], A[q], t1, B[q] * t1);
            }
            double* out = (q == ns - 1) ? g.X[F] : (q == 0 ? g.Y[F] : g.Z[F]);
            stage(F, in, nullptr, g.X[F], out, A[q], dl, B[q] * dl, (q == ns - 1 && !fin) ? 1 : 0, g.Tm[F]);
            // Eq. (secondcorrection); booked after the stage launch (the stage does not
            // read the correction) so that the GPU gets work soon after the readback
            if (q == 0 && !first && corr) corr_add(B[0] * dl, S);
            const double* commit = nullptr;
            const double* cur = ls_stage(q, q == ns - 1, A[q], dl, phin, &commit);
            ls_join();
            if (taped)
                k_phi_merge<<<fill_blocks(), 256, 0, s.stream>>>(g, cur, s.tape_ls.back() + (size_t)q * g.nc);
            if (q + 1 < ns) {
                // the slow fluid's state for the next stage, Eq. (interpolation)
                double theta1 = (fin && C[q + 1] == 1.0) ? 1.0 : (tau + C[q + 1] * dl) / t1;
                MixPart ms = interp_part(S, theta1);
                ms.sched_theta = planned ? 1 : 0;
                mix_fused(tm_part(F, out), &ms, cur, commit);
            } else {
                mix_fused(tm_part(F, out), nullptr, cur, commit);
            }
            if (commit) cur = g.phiP;
            in = out;
            phin = cur;
        };
        // sub-steps after the first are planned on the device when every
        // kernel of a stage can take its step from there
        const bool fixed = fixed_multi();
        const bool plan_dev = fused_ls() && s.dt_replay.empty() && !fixed;
        for (;;) {
            int hh = 0, fin = 0, q0 = 0;
            double dl = 0.0;
            const double* in = g.X[F];
            const double* phin = g.phiP;
            if (taped) {
                sim_status rc = tape_sub(s);
                if (rc != SIM_OK) return rc;
            }
            if (!first) {
                mask(LIST_BAND, 1);
                interp_slow(S, tau / t1, g.phiP);
                interaction(S == 0 ? g.T2 : g.X[F], S == 0 ? g.X[F] : g.T2, g.phiP, 0.0, S);
                join();
                if (fused_cfl) {
                    // bulk tiles were reduced by the previous sub-step's last stage
                    go<b_cfl<D, true>, SHARP_WG>(k_cfl<D, true>, grid(LIST_BAND), wg(), s.stream, g, LIST_BAND, F, g.X[F],
                                                  s.wcur);
                } else {
                    go<b_zero_red, 64>(k_zero_red, 1, 64, s.stream, g);
                    cfl_launch(F, g.X[F]);
                }
                fused_cfl = false;
                if (fixed) {
                    // prescribed steps: the reduction counts the fast fluid's
                    // cells (summed on the device while captured)
                    if (s.capturing) {
                        go<b_acc, 64>(k_acc, 1, 64, s.stream, g, 1 << F);
                    } else {
                        double d2[2];
                        long long c2[2];
                        sim_status rc = readback(1 << F, d2, c2);
                        if (rc != SIM_OK) return rc;
                        cntF = c2[F];
                    }
                    dtF = dt[F];
                } else if (plan_dev) {
                    // plan on the device, read the plan back, and enqueue the
                    // first stage before waiting for it
                    go<b_plan, 64>(k_plan, 1, 64, s.stream, g, F, tau, t1, ns, half_done, s.o.cfl, B[0], C[1]);
                    sim_status rc = rb_begin(RED_WORDS, true);
                    if (rc != SIM_OK) return rc;
                    g.use_sched = 1;
                    fast_stage(0, in, phin, 0.0, 0, true);
                    g.use_sched = 0;
                    rc = rb_wait(true);
                    if (rc == SIM_OK) rc = check_flags();
                    if (rc != SIM_OK) return rc;
                    const double* sc = reinterpret_cast<const double*>(s.h_red + RED_SCHED);
                    dtF = sc[SCHED_DTF];
                    s.dt_log.push_back(dtF);
                    cntF = (long long)sc[SCHED_CNT];
                    dl = sc[SCHED_DT];
                    hh = sc[SCHED_HH] != 0.0;
                    fin = sc[SCHED_FIN] != 0.0;
                    q0 = 1;
                } else {
                    double d2[2];
                    long long c2[2];
                    sim_status rc = readback(1 << F, d2, c2);
                    if (rc == SIM_OK) rc = take_cfl(1 << F, d2);
                    if (rc != SIM_OK) return rc;
                    dtF = d2[F];
                    cntF = c2[F];
                }
                if (!std::isfinite(dtF) || !(dtF > 0.0)) {
                    set_error("invalid fast-fluid time step");
                    return SIM_ENONPHYS;
                }
            }
            if (q0 == 0) {
                dl = next_substep(tau, t1, dtF, ns, half_done, &hh, &fin);
                if (first && corr) corr_add(-B[0] * t1 + B[0] * dl, S);
            }
            if (taped) s.tape_units.back().sub.back() = {dl, hh, fin};
            for (int q = q0; q < ns; q++) fast_stage(q, in, phin, dl, fin, false);
            st->steps[F]++;
            st->cell_updates[F] += cntF;
            tau = hh ? 0.5 * t1 : (fin ? t1 : tau + dl);
            if (hh) {
                half_done = 1;
                axpby(1.0, g.X[F], 0.0, nullptr, g.Fh, NV);
                axpby(1.0, g.phiP, 0.0, nullptr, g.phiH, 1);
            }
            first = 0;
            if (fin) break;
        }
        if (ns == 3) {
            // slow fluid's third stage at t1/2 against the snapshots
            geom(g.phiH);
            mixed_copy(S, g.Z[S], g.phiH);
            interaction(S == 0 ? g.T2 : g.Fh, S == 0 ? g.Fh : g.T2, g.phiH, corr ? -B[2] * t1 : 0.0, S, false);
            stage(S, g.Z[S], g.T2, g.X[S], g.X[S], A[2], t1, B[2] * t1);
            geom(g.phiP);
        }
        // interfacial flux correction of the slow fluid, then mixing
        go<b_corr_apply<D>, SHARP_WG>(k_corr_apply<D>, grid(LIST_INNER), wg(), s.stream, g, LIST_INNER, S,
                                      corr ? 1 : 0);
        mix(S, g.X[S], g.phiP);
        join();
        s.t += t1;
        cycle_adv = t1;
        st->cycles++;
        st->steps[S]++;
        st->cell_updates[S] += cnt[S];
        return SIM_OK;
    }

    sim_status advance(double t_end, int mode, long long max_cycles, sim_stats* st)
    {
        long long done = 0;
        sim_status rc = SIM_OK;
        if (mode != SIM_SINGLE_DT && replaying()) {
            set_error("ls_replay covers single-dt steps only");
            return SIM_EINVAL;
        }
        // a state found non-physical at this call's first cycle start is
        // left as the call found it
        s.snap_valid = false;
        s.snap_pending = false;
        while (s.t < t_end && (max_cycles <= 0 || done < max_cycles)) {
            if (mode == SIM_SINGLE_DT && graph_run_ok()) {
                // the whole steps of length dt_fixed before t_end, from graphs
                long long K = 0;
                double t = s.t;
                while ((max_cycles <= 0 || done + K < max_cycles) && t < t_end && !(s.o.dt_fixed > t_end - t)) {
                    t += s.o.dt_fixed;
                    if (t_end - t <= 1e-14 * t_end) t = t_end;
                    K++;
                }
                if (K > 0) {
                    // the run reports its flags once, at its end: the
                    // snapshot is that of the run's start
                    rc = snap_begin(st);
                    if (rc == SIM_OK) rc = graph_steps(K, t_end, st);
                    if (rc != SIM_OK) break;
                    done += K;
                    continue;
                }
            }
            if (mode == SIM_MULTI_DT && graph_run_ok(true)) {
                // the whole cycles before t_end, from graphs
                const double* f = s.o.dt_fixed_fluid;
                const int S = f[0] >= f[1] ? 0 : 1;
                double t1;
                int single;
                plan_cycle(f[S], f[1 - S], INFINITY, s.o.n_thr, &t1, &single);
                long long K = 0;
                double t = s.t;
                while ((max_cycles <= 0 || done + K < max_cycles) && t < t_end && !(t1 > t_end - t)) {
                    t += t1;
                    if (t_end - t <= 1e-14 * t_end) t = t_end;
                    K++;
                }
                if (K > 0) {
                    rc = snap_begin(st);
                    if (rc == SIM_OK) rc = graph_cycles(K, st);
                    if (rc != SIM_OK) break;
                    if (t_end - s.t <= 1e-14 * t_end) s.t = t_end;
                    done += K;
                    continue;
                }
            }
            double dt[2];
            long long cnt[2];
            rc = prepare(true, dt, cnt);
            if (rc != SIM_OK) break;
            // CFL steps (not for single-dt steps of the fixed length); the
            // prescribed steps of accelerated cycles
            if (mode == SIM_MULTI_DT && fixed_multi()) {
                dt[0] = s.o.dt_fixed_fluid[0];
                dt[1] = s.o.dt_fixed_fluid[1];
            } else if (!(mode == SIM_SINGLE_DT && s.o.dt_fixed > 0.0)) {
                rc = take_cfl(3, dt);
            }
            if (rc != SIM_OK) break;
            rc = snap_begin(st);
            if (rc != SIM_OK) break;
            if (s.o.autotune && !s.rec) tune_step(st);
            st->last_dt[0] = dt[0];
            st->last_dt[1] = dt[1];
            st->active_cells[0] = cnt[0];
            st->active_cells[1] = cnt[1];
            if (!(fmin(dt[0], dt[1]) > 0.0)) { set_error("invalid time step"); rc = SIM_ENONPHYS; break; }
            if (mode == SIM_SINGLE_DT) {
                double d = s.o.dt_fixed > 0.0 ? s.o.dt_fixed : (dt[0] < dt[1] ? dt[0] : dt[1]);
                if (d > t_end - s.t) d = t_end - s.t;
                if (replaying() && s.ls_pos + (size_t)s.o.rk > s.ls_src.size()) {
                    set_error("ls_replay exhausted after %zu stages", s.ls_pos);
                    rc = SIM_EINVAL;
                    break;
                }
                if (s.o.tape) {
                    rc = tape_step(s, d);
                    if (rc != SIM_OK) break;
                }
                step_single(d);
                st->cycles++;
                for (int k = 0; k < 2; k++) { st->steps[k]++; st->cell_updates[k] += cnt[k]; }
                st->last_n = 1.0;
            } else {
                if (s.o.tape && s.tape_fluid >= 0 && s.tape_fluid != 2) {
                    s.tape_fluid = -1;
                    s.tape_why = "a run in which one fluid fills the grid took accelerated (multi-dt) cycles";
                }
                rc = cycle(dt, cnt, t_end, st);
                if (rc != SIM_OK) break;
            }
            if (t_end - s.t <= 1e-14 * t_end) s.t = t_end;
            done++;
        }
        join();
        s.tune_open = false;    // time between calls is not a cycle
        if (rc == SIM_OK && done > 0) {
            // the call's final state: a cycle whose last stages produced a
            // non-physical state is found here, not at the next call's start
            for (int k = 0; k < 2; k++) {
                const int bl = k == 0 ? LIST_BULK0 : LIST_BULK1;
                go<b_verify<D>, SHARP_WG>(k_verify<D>, grid(bl), wg(), s.stream, g, bl, k);
                go<b_verify<D>, SHARP_WG>(k_verify<D>, grid(LIST_BAND), wg(), s.stream, g, LIST_BAND, k);
            }
        }
        if (rc == SIM_OK) {
            // late non-physical flags (stages after the last readback, and
            // the check of the final state)
            rc = rb_begin(RED_CELL + 1, false);
            if (rc == SIM_OK) rc = rb_wait(false);
            if (rc == SIM_OK && (s.h_red[4] & ERR_NONPHYS)) { nonphys_error(); rc = SIM_ENONPHYS; }
        }
        if (s.prof) profile_flush();
        if (rc == SIM_ENONPHYS && s.snap_valid) {
            std::string why = sim_last_error();
            sim_status r2 = rollback(st);
            if (r2 != SIM_OK) return r2;
            set_error("%s, in the cycle or step starting at t = %.17g (after %lld completed ones in this call); "
                      "the state is rolled back to that start",
                      why.c_str(), s.t, (long long)st->cycles);
        }
        st->t = s.t;
        return rc;
    }

    // Autotuner of the bulk-stage grid bound: called at each cycle start,
    // after the readback that ends the previous cycle's work.  One warm-up
    // cycle, then one cycle per candidate, timed by the host clock per
    // cell-update; then the fastest candidate stays.  The bound only changes
    // how tiles are spread over blocks, never a result.
    static double now_s()
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    }
    void tune_step(const sim_stats* st)
    {
        static const int cand[Sim::NTUNE] = {1024, 2048, 4096, 8192, 2048};
        static const bool cser[Sim::NTUNE] = {false, false, false, false, true};
        if (s.tune_cur >= Sim::NTUNE) return;
        const long long cells = st->cell_updates[0] + st->cell_updates[1];
        if (s.tune_open) {
            if (s.tune_cur >= 0 && cells > s.tune_cells0)
                s.tune_cost[s.tune_cur] = (now_s() - s.tune_t0) / (double)(cells - s.tune_cells0);
            s.tune_cur++;
        } else if (s.tune_cur == -2) {
            s.tune_cur = -1;
        }
        if (s.tune_cur >= Sim::NTUNE) {
            int best = 0;
            for (int i = 1; i < Sim::NTUNE; i++)
                if (s.tune_cost[i] < s.tune_cost[best]) best = i;
            s.bulk_blocks = cand[best];
            s.run_serial = cser[best];
            return;
        }
        s.bulk_blocks = cand[s.tune_cur < 0 ? 1 : s.tune_cur];
        s.run_serial = s.tune_cur < 0 ? false : cser[s.tune_cur];
        s.tune_t0 = now_s();
        s.tune_cells0 = cells;
        s.tune_open = true;
    }

    sim_status set_state(const double* phi, const double* prim)
    {
        s.lcount[LIST_ALL] = g.ntiles;
        SHARP_HIP(hipMemcpyAsync(g.phiP, phi, sizeof(double) * g.nc, hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(hipMemsetAsync(g.M, 0, g.nc, s.stream));
        geom(g.phiP, LIST_ALL);
        geom(g.phiP, LIST_ALL);   // both geometry buffers start from the initial level set
        int b = (g.nc + 255) / 256;
        if (b > 65535) b = 65535;
        k_init<D><<<b, 256, 0, s.stream>>>(g, prim);
        // band of the initial level set over every tile
        mask(LIST_ALL, 0);
        tiles();
        for (int k = 0; k < 2; k++)
            SHARP_HIP(hipMemsetAsync(g.bacc[k], 0, sizeof(double) * NV * (size_t)(g.nbface > 0 ? g.nbface : 1), s.stream));
        SHARP_HIP(reset_flags());
        SHARP_HIP(hipMemcpyAsync(s.h_red, g.red, RED_WORDS * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 s.stream));
        SHARP_HIP(hipStreamSynchronize(s.stream));
        SHARP_HIP(hipGetLastError());
        take_counts();
        s.snap_valid = false;
        s.snap_pending = false;
        s.t = 0.0;
        s.wcur = 0;
        s.vcur = 0;
        s.has_state = true;
        s.ls_src.clear();
        s.ls_pos = 0;
        for (size_t i = 0; i < s.n_ls_rep; i++) s.ls_src.push_back(s.ls_rep + i * (size_t)g.nc);
        if (s.o.tape) return tape_begin(s, prim);
        return SIM_OK;
    }

    sim_status bflux(double out[2][5])
    {
        std::vector<double> h((size_t)NV * (g.nbface > 0 ? g.nbface : 1));
        for (int k = 0; k < 2; k++) {
            SHARP_HIP(hipMemcpy(h.data(), g.bacc[k], sizeof(double) * h.size(), hipMemcpyDeviceToHost));
            for (int q = 0; q < 5; q++) out[k][q] = 0.0;
            for (int q = 0; q < NV; q++) {
                double sum = 0.0;
                for (int b = 0; b < g.nbface; b++) sum += h[(size_t)q * g.nbface + b];
                out[k][q] = sum;
            }
        }
        return SIM_OK;
    }
};

sim_status engine_set_state(Sim& s, const double* phi, const double* prim)
{
    switch (s.g.D) {
    case 1: return Engine<1>(s).set_state(phi, prim);
    case 2: return Engine<2>(s).set_state(phi, prim);
    default: return Engine<3>(s).set_state(phi, prim);
    }
}

sim_status engine_advance(Sim& s, double t_end, int mode, long long max_cycles, sim_stats* st)
{
    sim_status rc;
    switch (s.g.D) {
    case 1: rc = Engine<1>(s).advance(t_end, mode, max_cycles, st); break;
    case 2: rc = Engine<2>(s).advance(t_end, mode, max_cycles, st); break;
    default: rc = Engine<3>(s).advance(t_end, mode, max_cycles, st); break;
    }
    hipError_t e = hipGetLastError();
    if (rc == SIM_OK && e != hipSuccess) {
        set_error("kernel launch failed: %s", hipGetErrorString(e));
        return SIM_EDEVICE;
    }
    return rc;
}

void engine_bulk_stage(Sim& s, int k, const double* in, const double* base, double* out, double a, double dt)
{
    const int list = k == 0 ? LIST_BULK0 : LIST_BULK1;
    switch (s.g.D) {
    case 1: Engine<1>(s).launch_stage<false>(s.stream, list, k, in, nullptr, base, out, a, dt, 0.0, 0, nullptr); break;
    case 2: Engine<2>(s).launch_stage<false>(s.stream, list, k, in, nullptr, base, out, a, dt, 0.0, 0, nullptr); break;
    default: Engine<3>(s).launch_stage<false>(s.stream, list, k, in, nullptr, base, out, a, dt, 0.0, 0, nullptr); break;
    }
}

sim_status engine_restore(Sim& s, const double* X0, const double* X1, const double* phi)
{
    switch (s.g.D) {
    case 1: return Engine<1>(s).restore_state(X0, X1, phi);
    case 2: return Engine<2>(s).restore_state(X0, X1, phi);
    default: return Engine<3>(s).restore_state(X0, X1, phi);
    }
}

sim_status engine_replay_step(Sim& s, double dt, StageRec* rec, bool prepared)
{
    switch (s.g.D) {
    case 1: return Engine<1>(s).replay_step(dt, rec, prepared);
    case 2: return Engine<2>(s).replay_step(dt, rec, prepared);
    default: return Engine<3>(s).replay_step(dt, rec, prepared);
    }
}

#define SHARP_ENGINE(call)                 \
    switch (s.g.D) {                       \
    case 1: { Engine<1> e(s); call; } break; \
    case 2: { Engine<2> e(s); call; } break; \
    default: { Engine<3> e(s); call; } break; \
    }
sim_status engine_op_prepare(Sim& s)
{
    sim_status rc = SIM_OK;
    SHARP_ENGINE(rc = e.op_prepare());
    return rc;
}
void engine_op_interaction(Sim& s, const double* in0, const double* in1, const double* cur)
{
    SHARP_ENGINE(e.interaction(in0, in1, cur, 0.0, 0, false));
}
void engine_op_stage(Sim& s, int k, const double* in, const double* base, double* out, double a, double dt)
{
    SHARP_ENGINE(e.stage(k, in, nullptr, base, out, a, dt, 0.0, 0, nullptr); e.join());
}
const double* engine_op_ls(Sim& s, int q, bool last, double a, double dt, const double* phin)
{
    const double* cur = nullptr;
    SHARP_ENGINE(cur = e.ls_chain(q, last, a, dt, phin, nullptr));
    return cur;
}
void engine_op_mix(Sim& s, int k, double* buf, const double* cur)
{
    SHARP_ENGINE(e.mix(k, buf, cur));
}
void engine_op_mask(Sim& s)
{
    SHARP_ENGINE(e.mask(LIST_BAND, 1));
}
void engine_op_geom(Sim& s, const double* phi)
{
    SHARP_ENGINE(e.geom(phi));
}
void engine_op_corr_add(Sim& s, double w, int S)
{
    SHARP_ENGINE(e.corr_add(w, S));
}
void engine_op_corr_apply(Sim& s, int S)
{
    SHARP_ENGINE(e.op_corr_apply(S));
}
void engine_op_axpby(Sim& s, double a1, const double* x, double a2, const double* y, double* dst)
{
    SHARP_ENGINE(e.op_axpby_all(a1, x, a2, y, dst));
}
#undef SHARP_ENGINE

sim_status engine_bflux(Sim& s, double out[2][5])
{
    switch (s.g.D) {
    case 1: return Engine<1>(s).bflux(out);
    case 2: return Engine<2>(s).bflux(out);
    default: return Engine<3>(s).bflux(out);
    }
}

}  // namespace sharp
