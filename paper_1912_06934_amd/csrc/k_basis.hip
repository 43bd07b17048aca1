// Basis construction kernels: filter + Jacobi operator, initial basis and the
// restricted smoothing iteration of enhanced MsRSB (Sec. 2.1, Sec. 3.1,
// Alg. 1).
//
// Layouts.  P is stored row-major ELL: the pw slots of fine row i at
// i*pw .. i*pw+pw-1 (pw = 4 or 8, rows padded with zero values and column -1),
// so one thread reads a whole row with 16-byte loads and a wavefront reads
// 64 consecutive rows as one contiguous block.  J is stored slot-major
// ([jw][n], entry o of row i at o*n + i); its neighbour is either i + off[o]
// (the operator's rows use a few fixed column offsets, DIA) or an explicit
// column.
#include "internal.h"

#include <type_traits>

namespace msrsb {
namespace {

inline int grid_for(int64_t m) { return static_cast<int>((m + kBlock - 1) / kBlock); }

__device__ inline double wave_max(double v)
{
    // NaN-propagating max over the 64 lanes of a wavefront
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double o = __shfl_xor(v, off, 64);
        v = (o > v || o != o) ? o : v;
    }
    return v;
}

__device__ inline double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

// The work-group's max of the row deltas goes to part[blockIdx.x]; a
// one-block kernel reduces the partials (no contended atomics).
__device__ inline void eit_block(double emax, double *__restrict__ part)
{
    __shared__ double sh[kBlock / 64];
    emax = wave_max(emax);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = emax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0];
        for (int w = 1; w < kBlock / 64; ++w) m = nan_max(m, sh[w]);
        part[blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(1024) void k_eit_final(int nb, const double *__restrict__ part,
                                                    double *__restrict__ out)
{
    __shared__ double sh[16];
    double m = 0.0;
    for (int b = threadIdx.x; b < nb; b += 1024) m = nan_max(m, part[b]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int w = 1; w < 16; ++w) r = nan_max(r, sh[w]);
        out[0] = r;
    }
}

// Filter (eq. negoffdiag) and zero-row-sum diagonal (eq. Dhat_zero_rowsum):
// per row, Dhat_ii = -sum_{j != i, same component} G_ij with
// G_ij = min(A_ij, 0) when filtering; then J = I - omega Dhat^{-1} Ghat, i.e.
// J_ii = 1 - omega, J_ij = -omega G_ij / Dhat_ii.  A row with Dhat_ii == 0 is
// frozen (J_i = e_i).  J's entries are A's same-component entries; they are
// written to their ELL slot (the DIA offset slot, or the running position),
// and absent slots are zero.
//
// sym (a symmetric stencil A, so Ghat is symmetric): J is kept factored,
// J_ij = s_i Ghat_ij with s_i = -omega / Dhat_ii (0 for a frozen row), and
// only s (in the diagonal slot) and the upper diagonals of Ghat are stored;
// the smoothing step reads Ghat_{i,i-o} = Ghat_{i-o,i} from the neighbour's
// row and J_ii = 1 - omega (1 where s_i = 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_filter_jacobi(
    int n, int bs, int filter, double omega, const int *__restrict__ rp,
    const int *__restrict__ ci, const double *__restrict__ a, int jw, DiaOffsets joff,
    int use_dia, int sym, T *__restrict__ jv)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int e0 = rp[i], e1 = rp[i + 1];
    const int ic = i % bs;
    double d = 0.0;
    for (int e = e0; e < e1; ++e) {
        const int j = ci[e];
        if (j == i || j % bs != ic) continue;
        double g = a[e];
        if (filter && g > 0.0) g = 0.0;
        d -= g;
    }
    for (int o = 0; o < jw; ++o) jv[static_cast<int64_t>(o) * n + i] = T(0);
    int pos = 0;
    for (int e = e0; e < e1; ++e) {
        const int j = ci[e];
        if (j % bs != ic) continue;
        double v;
        if (sym) {
            if (j < i) continue;
            if (j == i) {
                v = d == 0.0 ? 0.0 : -omega / d;
            } else {
                v = a[e];
                if (filter && v > 0.0) v = 0.0;
            }
        } else if (d == 0.0) {
            v = (j == i) ? 1.0 : 0.0;
        } else if (j == i) {
            v = 1.0 - omega;
        } else {
            double g = a[e];
            if (filter && g > 0.0) g = 0.0;
            v = -omega * g / d;
        }
        int slot = pos++;
        if (use_dia) {
            const int dlt = j - i;
            for (int o = 0; o < joff.n; ++o)
                if (joff.off[o] == dlt) slot = o;
        }
        jv[static_cast<int64_t>(slot) * n + i] = static_cast<T>(v);
    }
}

// Initial basis (Sec. 2.1): characteristic function of the coarse block.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_basis(int64_t m, int pw,
                                                       const int *__restrict__ pcol,
                                                       const int *__restrict__ part,
                                                       T *__restrict__ p)
{
    // one ELL entry per thread (coalesced stores)
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= m) return;
    p[e] = (pcol[e] == part[e / pw]) ? T(1) : T(0);
}

// One restricted smoothing iteration (eq. smoother, Alg. 1), slot-map form.
//
// For output slot s of row i (coarse column c_is) the restricted product is
//   T_is = sum over J entries o of row i (ascending column) of
//          J_io * P[k_o, slot of c_is in row k_o]
// where the slot comes from a precomputed 4-bit map (0xF: c_is is not in row
// k_o's pattern, the product is absent).  Products P_kj with j outside row
// i's pattern never enter, which is the support restriction.  The row is then
// rescaled by its FP64 sum so that P stays a partition of unity, and
// |T - P_old| on interior rows feeds e_it.
//
// Each neighbour row of P is read whole with 16-byte loads and the needed
// slot is selected in registers.
// A row is moved as 16-byte vectors whose lanes are unpacked into (or packed
// from) a register array; the array itself is never addressed as memory.
template <typename T, int PW>
__device__ inline void load_row(const T *__restrict__ p, int64_t row, T (&v)[PW])
{
    constexpr int L = 16 / sizeof(T);
    static_assert(PW % L == 0, "rows are read in 16-byte pieces");
    typedef T vec __attribute__((ext_vector_type(L)));
    const vec *src = reinterpret_cast<const vec *>(p + row * PW);
#pragma unroll
    for (int q = 0; q < PW / L; ++q) {
        const vec x = src[q];
#pragma unroll
        for (int j = 0; j < L; ++j) v[q * L + j] = x[j];
    }
}

template <typename T, int PW, bool NT = false>
__device__ inline void store_row(T *__restrict__ p, int64_t row, const T (&v)[PW])
{
    constexpr int L = 16 / sizeof(T);
    typedef T vec __attribute__((ext_vector_type(L)));
    vec *dst = reinterpret_cast<vec *>(p + row * PW);
#pragma unroll
    for (int q = 0; q < PW / L; ++q) {
        vec x;
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = v[q * L + j];
        if constexpr (NT)
            __builtin_nontemporal_store(x, dst + q);
        else
            dst[q] = x;
    }
}


// v[src] for src < PW by a select tree on the bits of src
template <typename T, int PW>
__device__ inline T pick(const T (&v)[PW], uint32_t src)
{
    static_assert(PW == 4 || PW == 8, "slot maps cover 4 or 8 slots");
    const bool b0 = src & 1u, b1 = src & 2u;
    const T a0 = b0 ? v[1] : v[0], a1 = b0 ? v[3] : v[2];
    const T lo = b1 ? a1 : a0;
    if constexpr (PW == 4) {
        return lo;
    } else {
        const T a2 = b0 ? v[5] : v[4], a3 = b0 ? v[7] : v[6];
        const T hi = b1 ? a3 : a2;
        return (src & 4u) ? hi : lo;
    }
}

// Map of J entry e: a one-byte index into the LDS table, a two-byte index
// into the global table, or the map itself.
template <typename IDX>
__device__ __forceinline__ uint32_t map_of(const IDX *__restrict__ jmap, int64_t e,
                                           const uint32_t *stab, const uint32_t *__restrict__ tab)
{
    if constexpr (sizeof(IDX) == 1)
        return stab[jmap[e]];
    else if constexpr (sizeof(IDX) == 2)
        return tab[jmap[e]];
    else
        return static_cast<uint32_t>(jmap[e]);
}

// acc += w * (row v permuted by map m); absent slots (nibble 0xF) add zero
template <typename T, int PW>
__device__ __forceinline__ void accumulate(T (&acc)[PW], uint32_t m, T w, const T (&v)[PW])
{
#pragma unroll
    for (int s = 0; s < PW; ++s) {
        const uint32_t src = (m >> (4 * s)) & 0xFu;
        acc[s] += ((src & 8u) ? T(0) : w) * pick<T, PW>(v, src);
    }
}

// The same when the map is diagonal (every slot reads its own slot or
// nothing), as for neighbours with the same support pattern: no selects.
template <typename T, int PW>
__device__ __forceinline__ void accumulate_diag(T (&acc)[PW], uint32_t m, T w, const T (&v)[PW])
{
#pragma unroll
    for (int s = 0; s < PW; ++s) acc[s] += (((m >> (4 * s)) & 8u) ? T(0) : w) * v[s];
}

// The same through LDS: the neighbour row is written slot-major into this
// thread's column of sb ([PW + 1][kBlock], row PW zero) and read back at the
// mapped slots (an absent slot reads the zero row), so the permutation costs
// one address and one LDS read per slot instead of a select tree.  Each
// thread touches only its own column: no barrier is needed.
template <typename T, int PW>
__device__ __forceinline__ void accumulate_lds(T (&acc)[PW], uint32_t m, T w, const T (&v)[PW],
                                               T *sb)
{
#pragma unroll
    for (int t = 0; t < PW; ++t) sb[t * kBlock] = v[t];
#pragma unroll
    for (int s = 0; s < PW; ++s) {
        const uint32_t src = (m >> (4 * s)) & 0xFu;
        acc[s] += w * sb[min(src, static_cast<uint32_t>(PW)) * kBlock];
    }
}

__host__ __device__ inline bool map_is_diag(uint32_t m)
{
    for (int s = 0; s < 8; ++s) {
        const uint32_t src = (m >> (4 * s)) & 0xFu;
        if (src != static_cast<uint32_t>(s) && src != 0xFu) return false;
    }
    return true;
}

// t / d for 0 <= t < 2^31 from the FP64 product with 1 / d, which is off
// by at most one
__device__ __forceinline__ int div_by(int t, int d, double rd)
{
    int q = static_cast<int>(static_cast<double>(t) * rd);
    const int r = t - q * d;
    q += r < 0 ? -1 : (r >= d ? 1 : 0);
    return q;
}

// The split form's table entries of row row0 + threadIdx.x and of its six
// 7-point neighbours' axis positions (rows run x fastest; the row must lie in
// the grid): a[0..2] x, y, z; a[3..5] x-1, y-1, z-1; a[6..8] x+1, y+1, z+1,
// 0 for a position outside the grid.  All nine are loaded at once (indices
// clamped, no branches) and used only by split_index7, so that other loads
// can be issued while they are in flight.
__device__ __forceinline__ void split_load7(const SplitRows &g, int row0, int (&a)[9])
{
    const int nx = g.nx, ny = g.ny;
    const int line0 = div_by(row0, nx, g.rnx);
    const int z0 = div_by(line0, ny, g.rny);
    const int t = row0 - line0 * nx + static_cast<int>(threadIdx.x);
    const int q = div_by(t, nx, g.rnx);
    const int x = t - q * nx;
    const int yy = line0 - z0 * ny + q;
    const int q2 = div_by(yy, ny, g.rny);
    const int y = yy - q2 * ny, z = z0 + q2;
    const int *tx = g.tab, *ty = g.tab + nx, *tz = g.tab + nx + ny;
    a[0] = tx[x];
    a[1] = ty[y];
    a[2] = tz[z];
    a[3] = tx[max(x - 1, 0)];
    a[4] = ty[max(y - 1, 0)];
    a[5] = tz[max(z - 1, 0)];
    a[6] = tx[min(x + 1, nx - 1)];
    a[7] = ty[min(y + 1, ny - 1)];
    a[8] = tz[min(z + 1, g.nz - 1)];
    a[3] = x > 0 ? a[3] : 0;
    a[4] = y > 0 ? a[4] : 0;
    a[5] = z > 0 ? a[5] : 0;
    a[6] = x + 1 < nx ? a[6] : 0;
    a[7] = y + 1 < ny ? a[7] : 0;
    a[8] = z + 1 < g.nz ? a[8] : 0;
}

// Second-half indices (h) of the row and its neighbours in the order of the
// ascending 7-point offsets (-z, -y, -x, 0, +x, +y, +z), and whether each has
// 8 entries (f)
__device__ __forceinline__ void split_index7(const int (&a)[9], int (&h)[7], bool (&f)[7])
{
    constexpr int M = 0x7FFFFFFF;
    const int ax = a[0], ay = a[1], az = a[2];
    const int bx = ax & M, by = ay & M, bz = az & M;
    h[0] = bx + by + (a[5] & M);
    f[0] = (ax & ay & a[5]) < 0;
    h[1] = bx + (a[4] & M) + bz;
    f[1] = (ax & a[4] & az) < 0;
    h[2] = (a[3] & M) + by + bz;
    f[2] = (a[3] & ay & az) < 0;
    h[3] = bx + by + bz;
    f[3] = (ax & ay & az) < 0;
    h[4] = (a[6] & M) + by + bz;
    f[4] = (a[6] & ay & az) < 0;
    h[5] = bx + (a[7] & M) + bz;
    f[5] = (ax & a[7] & az) < 0;
    h[6] = bx + by + (a[8] & M);
    f[6] = (ax & ay & a[8]) < 0;
}

// JW > 0: J has exactly JW slots per row, known at compile time, and the
// neighbours are taken in chunks whose map indices, weights and rows are all
// loaded before any is used (one wavefront keeps a whole chunk in flight).
// JW == 0: any slot count, one neighbour at a time.
// SYM (JW > 0, stencil J stored factored by k_filter_jacobi's sym form):
// J_io = s_i Ghat_up[JW-1-o][i+off_o] below the diagonal, s_i Ghat_up[o][i]
// above it, and 1 - omega (1 for a frozen row) on it.
// SPLIT (PW 8, the 7-point J): P in and out in the split form (SplitRows):
// the first halves of all rows, then the second halves of the 8-entry rows.
template <typename T, typename IDX, int PW, int JW, bool SYM = false, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) void k_smooth_map(
    int n, int jw, DiaOffsets joff, const int *__restrict__ jcol, const T *__restrict__ jv,
    const IDX *__restrict__ jmap, const uint32_t *__restrict__ tab, int ntab,
    const T *__restrict__ pin, T *__restrict__ pout, const uint8_t *__restrict__ interior,
    double *__restrict__ eit_part, double omega, GridOrder go, SplitRows sg)
{
    static_assert(!SPLIT || (PW == 8 && JW == 7), "the split form covers 8-slot rows, 7-point J");
    // a one-byte map index selects from a table of at most 256 maps kept in
    // LDS; the sign bit of sdiag marks diagonal maps
    __shared__ uint32_t stab[256];
    __shared__ uint8_t sdiag[256];
    // per-thread columns for the permutation of neighbour rows (JW > 0)
    __shared__ T sperm[JW > 0 ? (PW + 1) * kBlock : 1];
    T *sb = sperm + (JW > 0 ? threadIdx.x : 0);
    if constexpr (JW > 0) sb[PW * kBlock] = T(0);
    const int row0 = grid_row0(go);
    const int i = row0 + static_cast<int>(threadIdx.x);
    // chunk: up to 9 FP32 rows or 7 FP64 rows in registers at once
    constexpr int CMAX = sizeof(T) == 8 ? 7 : 9;
    constexpr int MID = JW / 2;
    // When one chunk holds every neighbour, all of the row's global loads
    // (map indices, weights, neighbour rows) are issued before the map table
    // is staged, so the two memory round trips overlap.  The rows are read
    // before the maps are known: an absent neighbour reads any row inside the
    // matrix (its contribution is zero), one past the ends reads row i.
    constexpr bool kOne = JW > 0 && JW <= CMAX;
    constexpr int N1 = kOne ? JW : 1;
    int t1[N1];
    T w1[N1], v1[N1][PW];
    // split form: this row's second-half index and whether it has one
    int h_own = 0;
    bool f_own = false;
    if constexpr (kOne) {
        if (i < n) {
            // the neighbour rows first, then the map indices and J values
            // (all loads in flight before any arithmetic waits on one)
            int k[JW];
            if (jcol) {
#pragma unroll
                for (int o = 0; o < JW; ++o) k[o] = jcol[static_cast<int64_t>(o) * n + i];
            } else {
#pragma unroll
                for (int o = 0; o < JW; ++o) k[o] = i + joff.off[o];
            }
            // split form: the table entries, then the first halves by row;
            // the second halves follow the J loads (below)
            int sa[SPLIT ? 9 : 1];
            if constexpr (SPLIT) {
                split_load7(sg, row0, sa);
#pragma unroll
                for (int o = 0; o < JW; ++o) {
                    const int kk = (k[o] >= 0 && k[o] < n) ? k[o] : i;
                    T a4[4];
                    load_row<T, 4>(pin, kk, a4);
#pragma unroll
                    for (int s = 0; s < 4; ++s) v1[o][s] = a4[s];
                }
            } else {
#pragma unroll
                for (int o = 0; o < JW; ++o) {
                    const int kk = (k[o] >= 0 && k[o] < n) ? k[o] : i;
                    load_row<T, PW>(pin, kk, v1[o]);
                }
            }
            // J values as stored (the weights are formed after the table)
            T jraw[JW];
#pragma unroll
            for (int o = 0; o < JW; ++o) {
                const int64_t e = static_cast<int64_t>(o) * n + i;
                t1[o] = jmap[e];
                if constexpr (SYM) {
                    // the lower coefficients mirror the neighbour's upper
                    // ones; an absent neighbour's mirrored slot is zero by
                    // pattern symmetry, one beyond the ends reads row i
                    const int kn = i + joff.off[o];
                    const bool in = kn >= 0 && kn < n;
                    if (o < MID)
                        jraw[o] = jv[static_cast<int64_t>(JW - 1 - o) * n + (in ? kn : i)];
                    else
                        jraw[o] = jv[e];
                } else {
                    jraw[o] = jv[e];
                }
            }
#pragma unroll
            for (int o = 0; o < JW; ++o) w1[o] = jraw[o];
            if constexpr (SPLIT) {
                // second halves where the row has 8 entries (the other rows'
                // slots 4-7 are zero and not stored): a buffer load whose
                // offset lies past the end returns zeros without a memory
                // access, so no lane branches.  The indices are formed only
                // here (the scheduler may not hoist them above the loads
                // issued so far, which would wait for the table entries
                // before issuing those).
                __builtin_amdgcn_sched_barrier(0);
                int hs[7];
                bool fs[7];
                split_index7(sa, hs, fs);
                const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<T *>(pin + static_cast<int64_t>(n) * 4), 0,
                    static_cast<int>(sg.n8 * 4 * static_cast<int64_t>(sizeof(T))), 0x00020000);
                constexpr int L = 16 / sizeof(T);
                typedef T vec __attribute__((ext_vector_type(L)));
#pragma unroll
                for (int o = 0; o < JW; ++o) {
                    const uint32_t off =
                        fs[o] ? static_cast<uint32_t>(hs[o]) * (4 * sizeof(T)) : 0x80000000u;
#pragma unroll
                    for (int q = 0; q < 4 / L; ++q) {
                        const vec x = __builtin_bit_cast(
                            vec, __builtin_amdgcn_raw_buffer_load_b128(rh, off + 16 * q, 0, 0));
#pragma unroll
                        for (int l = 0; l < L; ++l) v1[o][4 + q * L + l] = x[l];
                    }
                }
                h_own = hs[MID];
                f_own = fs[MID];
            }
        }
    }
    if constexpr (sizeof(IDX) == 1) {
        for (int t = threadIdx.x; t < ntab; t += kBlock) {
            const uint32_t m = tab[t];
            stab[t] = m;
            sdiag[t] = map_is_diag(m) ? 1 : 0;
        }
        __syncthreads();
    }
    double emax = 0.0;
    // FP64 rows leave through LDS (below); out stays zero past n
    constexpr bool kStream = JW > 0 && sizeof(T) == 8;
    T out[PW];
#pragma unroll
    for (int s = 0; s < PW; ++s) out[s] = T(0);
    if (i < n) {
        T acc[PW];
#pragma unroll
        for (int s = 0; s < PW; ++s) acc[s] = T(0);
        if constexpr (kOne) {
            static_assert(sizeof(IDX) == 1, "fixed slot counts use the LDS map table");
            if constexpr (SYM) {
                // J = s_i Ghat: w1 holds the raw upper coefficients (the
                // neighbour's for the lower slots) and s_i in the middle
                const T si = w1[MID];
#pragma unroll
                for (int o = 0; o < JW; ++o) {
                    const int kn = i + joff.off[o];
                    const bool in = kn >= 0 && kn < n;
                    if (o < MID)
                        w1[o] = in ? si * w1[o] : T(0);
                    else if (o > MID)
                        w1[o] = si * w1[o];
                }
                w1[MID] = si == T(0) ? T(1) : static_cast<T>(1.0 - omega);
            }
            // a neighbour whose map is diagonal on every lane of the
            // wavefront (same support pattern) skips the slot selects
#pragma unroll
            for (int o = 0; o < JW; ++o) {
                const uint32_t m = stab[t1[o]];
                if (__all(sdiag[t1[o]] != 0))
                    accumulate_diag<T, PW>(acc, m, w1[o], v1[o]);
                else
                    accumulate_lds<T, PW>(acc, m, w1[o], v1[o], sb);
            }
        } else if constexpr (JW > 0) {
            static_assert(sizeof(IDX) == 1, "fixed slot counts use the LDS map table");
            T si = T(0), jd = T(0);
            if constexpr (SYM) {
                si = jv[static_cast<int64_t>(MID) * n + i];
                jd = si == T(0) ? T(1) : static_cast<T>(1.0 - omega);
            }
            constexpr int CH = JW <= CMAX ? JW : CMAX;
#pragma nounroll
            for (int o0 = 0; o0 < JW; o0 += CH) {
                uint32_t m[CH];
                T w[CH];
                int k[CH];
                bool dg[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    if (o0 + u >= JW) continue;
                    const int o = o0 + u;
                    const int64_t e = static_cast<int64_t>(o) * n + i;
                    const int t = jmap[e];
                    m[u] = stab[t];
                    dg[u] = sdiag[t] != 0;
                    if constexpr (SYM) {
                        // an absent neighbour's mirrored slot is zero by
                        // pattern symmetry; one beyond the ends reads row i
                        const int kn = i + joff.off[o];
                        const bool in = kn >= 0 && kn < n;
                        if (o < MID) {
                            const T g = jv[static_cast<int64_t>(JW - 1 - o) * n + (in ? kn : i)];
                            w[u] = in ? si * g : T(0);
                        } else if (o == MID)
                            w[u] = jd;
                        else
                            w[u] = si * jv[e];
                    } else {
                        w[u] = jv[e];
                    }
                }
                if (jcol) {
#pragma unroll
                    for (int u = 0; u < CH; ++u)
                        if (o0 + u < JW) k[u] = jcol[static_cast<int64_t>(o0 + u) * n + i];
                } else {
#pragma unroll
                    for (int u = 0; u < CH; ++u)
                        if (o0 + u < JW) k[u] = i + joff.off[o0 + u];
                }
                // an absent entry may point outside the matrix: read row i
#pragma unroll
                for (int u = 0; u < CH; ++u)
                    if (o0 + u < JW && m[u] == 0xFFFFFFFFu) k[u] = i;
                T v[CH][PW];
#pragma unroll
                for (int u = 0; u < CH; ++u)
                    if (o0 + u < JW) load_row<T, PW>(pin, k[u], v[u]);
                // a neighbour whose map is diagonal on every lane of the
                // wavefront (same support pattern) skips the slot selects
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    if (o0 + u >= JW) continue;
                    if (__all(dg[u]))
                        accumulate_diag<T, PW>(acc, m[u], w[u], v[u]);
                    else
                        accumulate_lds<T, PW>(acc, m[u], w[u], v[u], sb);
                }
            }
        } else {
            for (int o = 0; o < jw; ++o) {
                const int64_t e = static_cast<int64_t>(o) * n + i;
                const uint32_t m = map_of(jmap, e, stab, tab);
                if (m == 0xFFFFFFFFu) continue;
                const T w = jv[e];
                const int k = jcol ? jcol[e] : i + joff.off[o];
                T v[PW];
                load_row<T, PW>(pin, k, v);
                accumulate<T, PW>(acc, m, w, v);
            }
        }
        double rs = 0.0;
#pragma unroll
        for (int s = 0; s < PW; ++s) rs += static_cast<double>(acc[s]);
        T old[PW];
        if constexpr (SPLIT) {
            // the row itself is the middle neighbour
#pragma unroll
            for (int s = 0; s < PW; ++s) old[s] = v1[MID][s];
        } else {
            load_row<T, PW>(pin, i, old);
        }
        const bool inner = eit_part != nullptr && interior[i] != 0;
        const double rinv = 1.0 / rs;
#pragma unroll
        for (int s = 0; s < PW; ++s) {
            if (inner) {
                const double dlt = fabs(static_cast<double>(acc[s]) - static_cast<double>(old[s]));
                emax = (dlt > emax || dlt != dlt) ? dlt : emax;
            }
            out[s] = static_cast<T>(static_cast<double>(acc[s]) * rinv);
        }
        if constexpr (!kStream) {
            if constexpr (SPLIT) {
                T lo4[4], hi4[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    lo4[s] = out[s];
                    hi4[s] = out[4 + s];
                }
                store_row<T, 4>(pout, i, lo4);
                if (f_own) store_row<T, 4>(pout + static_cast<int64_t>(n) * 4, h_own, hi4);
            } else {
                store_row<T, PW>(pout, i, out);
            }
        }
    }
    if constexpr (kStream) {
        // FP64 rows are written as streaming stores: they are not read again
        // in this iteration, and keeping them out of the L2 leaves room for
        // the neighbour rows one grid plane apart (FP32 rows fit either way,
        // and measure faster with plain stores).  A streaming store reaches
        // memory as written, so the wavefront's 64 rows (consecutive) are
        // first transposed through the threads' LDS columns, which the
        // accumulation no longer needs: each store instruction then covers
        // 1 KB of whole cache lines instead of 16 bytes of each of 64 rows.
        constexpr int L = 16 / sizeof(T);
        typedef T vec __attribute__((ext_vector_type(L)));
        const int lane = threadIdx.x & 63, wbase = threadIdx.x & ~63;
        const int64_t wrow0 = static_cast<int64_t>(i) - lane;  // the wavefront's first row
        if constexpr (SPLIT) {
            // first halves: 64 consecutive rows of 4 slots
            constexpr int CH = 4 / L;
#pragma unroll
            for (int t = 0; t < 4; ++t) sb[t * kBlock] = out[t];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int piece = q * 64 + lane, r = piece / CH, c = piece % CH;
                vec x;
#pragma unroll
                for (int l = 0; l < L; ++l) x[l] = sperm[(c * L + l) * kBlock + wbase + r];
                if (wrow0 + r < n)
                    __builtin_nontemporal_store(x, reinterpret_cast<vec *>(pout + (wrow0 + r) * 4) + c);
            }
            // second halves of the wavefront's 8-entry rows: consecutive in
            // the second part, packed into the first columns before storing
            const bool mine = i < n && f_own;
            const uint64_t bal = __ballot(mine);
            if (bal != 0) {
                const int p = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                    static_cast<uint32_t>(bal >> 32),
                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bal), 0u)));
                const int cnt = __popcll(bal), first = __ffsll(static_cast<long long>(bal)) - 1;
                const int64_t h0 = __builtin_amdgcn_readlane(h_own - p, first);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (mine)
#pragma unroll
                    for (int t = 0; t < 4; ++t) sperm[t * kBlock + wbase + p] = out[4 + t];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                T *phi = pout + static_cast<int64_t>(n) * 4;
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const int piece = q * 64 + lane, r = piece / CH, c = piece % CH;
                    if (r < cnt) {
                        vec x;
#pragma unroll
                        for (int l = 0; l < L; ++l) x[l] = sperm[(c * L + l) * kBlock + wbase + r];
                        __builtin_nontemporal_store(x, reinterpret_cast<vec *>(phi + (h0 + r) * 4) + c);
                    }
                }
            }
        } else {
            constexpr int CH = PW / L;
#pragma unroll
            for (int t = 0; t < PW; ++t) sb[t * kBlock] = out[t];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int piece = q * 64 + lane, r = piece / CH, c = piece % CH;
                vec x;
#pragma unroll
                for (int l = 0; l < L; ++l) x[l] = sperm[(c * L + l) * kBlock + wbase + r];
                if (wrow0 + r < n)
                    __builtin_nontemporal_store(x, reinterpret_cast<vec *>(pout + (wrow0 + r) * PW) + c);
            }
        }
    }
    if (eit_part != nullptr) eit_block(emax, eit_part);
}

// Fallback for rows wider than the slot maps allow: row i's pattern (W
// slots) in registers, every entry of every neighbour row compared against it.
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_smooth_cmp(
    int n, int pw, int jw, DiaOffsets joff, const int *__restrict__ jcol,
    const T *__restrict__ jv, const int *__restrict__ pcol, const T *__restrict__ pin,
    T *__restrict__ pout, const uint8_t *__restrict__ interior,
    double *__restrict__ eit_part)
{
    const int i = xcd_row();
    double emax = 0.0;
    if (i < n) {
        int col[W];
        T acc[W];
#pragma unroll
        for (int s = 0; s < W; ++s) {
            col[s] = (s < pw) ? pcol[static_cast<int64_t>(i) * pw + s] : -1;
            acc[s] = T(0);
        }
        for (int o = 0; o < jw; ++o) {
            const int64_t e = static_cast<int64_t>(o) * n + i;
            const int k = jcol ? jcol[e] : i + joff.off[o];
            if (k < 0 || k >= n) continue;
            const T w = jv[e];
            if (w == T(0)) continue;
            for (int q = 0; q < pw; ++q) {
                const int c = pcol[static_cast<int64_t>(k) * pw + q];
                if (c < 0) break;
                const T wv = w * pin[static_cast<int64_t>(k) * pw + q];
#pragma unroll
                for (int s = 0; s < W; ++s) acc[s] += (col[s] == c) ? wv : T(0);
            }
        }
        double rs = 0.0;
#pragma unroll
        for (int s = 0; s < W; ++s) rs += static_cast<double>(acc[s]);
        const double rinv = 1.0 / rs;
        const bool inner = eit_part != nullptr && interior[i] != 0;
#pragma unroll
        for (int s = 0; s < W; ++s) {
            if (s < pw) {
                const int64_t e = static_cast<int64_t>(i) * pw + s;
                if (inner) {
                    const double dlt =
                        fabs(static_cast<double>(acc[s]) - static_cast<double>(pin[e]));
                    emax = (dlt > emax || dlt != dlt) ? dlt : emax;
                }
                pout[e] = static_cast<T>(static_cast<double>(acc[s]) * rinv);
            }
        }
    }
    if (eit_part != nullptr) eit_block(emax, eit_part);
}

// Partial statistics of P: max |row sum - 1|, min and max entry (padding
// slots hold zeros and are skipped through the column array).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_basis_stats(int n, int pw, const int *__restrict__ pcol,
                                                        const T *__restrict__ p,
                                                        double *__restrict__ partials)
{
    __shared__ double sh[3][kBlock];
    double err = 0.0, lo = 1e300, hi = -1e300;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double s = 0.0;
        for (int q = 0; q < pw; ++q) {
            const int64_t e = static_cast<int64_t>(i) * pw + q;
            if (pcol[e] < 0) continue;
            const double v = static_cast<double>(p[e]);
            s += v;
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
        const double d = fabs(s - 1.0);
        err = (d > err || d != d) ? d : err;
    }
    sh[0][threadIdx.x] = err;
    sh[1][threadIdx.x] = lo;
    sh[2][threadIdx.x] = hi;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            const double o = sh[0][threadIdx.x + st];
            sh[0][threadIdx.x] = (o > sh[0][threadIdx.x] || o != o) ? o : sh[0][threadIdx.x];
            sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + st]);
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = sh[0][0];
        partials[3 * blockIdx.x + 1] = sh[1][0];
        partials[3 * blockIdx.x + 2] = sh[2][0];
    }
}

// The same for 4- or 8-wide rows, one ELL entry per thread (coalesced): a
// row is PW consecutive lanes, its sum formed by a butterfly over them.
template <typename T, int PW>
__global__ __launch_bounds__(kBlock) void k_basis_stats_e(int64_t m, const int *__restrict__ pcol,
                                                          const T *__restrict__ p,
                                                          double *__restrict__ partials)
{
    __shared__ double sh[3][kBlock];
    double err = 0.0, lo = 1e300, hi = -1e300;
    // the stride is a multiple of PW, so a lane keeps its slot
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kBlock) {
        const bool real = pcol[e] >= 0;
        const double v = real ? static_cast<double>(p[e]) : 0.0;
        if (real) {
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
        double s = v;
#pragma unroll
        for (int off = 1; off < PW; off <<= 1) s += __shfl_xor(s, off, 64);
        if ((threadIdx.x & (PW - 1)) == 0) {
            const double d = fabs(s - 1.0);
            err = (d > err || d != d) ? d : err;
        }
    }
    sh[0][threadIdx.x] = err;
    sh[1][threadIdx.x] = lo;
    sh[2][threadIdx.x] = hi;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            const double o = sh[0][threadIdx.x + st];
            sh[0][threadIdx.x] = (o > sh[0][threadIdx.x] || o != o) ? o : sh[0][threadIdx.x];
            sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + st]);
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = sh[0][0];
        partials[3 * blockIdx.x + 1] = sh[1][0];
        partials[3 * blockIdx.x + 2] = sh[2][0];
    }
}

__global__ __launch_bounds__(kBlock) void k_basis_stats_final(int nb,
                                                              const double *__restrict__ partials,
                                                              double *__restrict__ out)
{
    __shared__ double sh[3][kBlock];
    double err = 0.0, lo = 1e300, hi = -1e300;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        const double o = partials[3 * b];
        err = (o > err || o != o) ? o : err;
        lo = fmin(lo, partials[3 * b + 1]);
        hi = fmax(hi, partials[3 * b + 2]);
    }
    sh[0][threadIdx.x] = err;
    sh[1][threadIdx.x] = lo;
    sh[2][threadIdx.x] = hi;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            const double o = sh[0][threadIdx.x + st];
            sh[0][threadIdx.x] = (o > sh[0][threadIdx.x] || o != o) ? o : sh[0][threadIdx.x];
            sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + st]);
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0][0];
        out[1] = sh[1][0];
        out[2] = sh[2][0];
    }
}

template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_convert(int64_t m, const S *__restrict__ s,
                                                    D *__restrict__ d)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t < m) d[t] = static_cast<D>(s[t]);
}

// ELL <-> CSR for P (values in double on the CSR side)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ell_to_csr(int n, int pw, const int *__restrict__ prp,
                                                       const T *__restrict__ pe,
                                                       double *__restrict__ pc)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int e0 = prp[i], np = prp[i + 1] - e0;
    for (int s = 0; s < np; ++s) pc[e0 + s] = static_cast<double>(pe[static_cast<int64_t>(i) * pw + s]);
}

__global__ __launch_bounds__(kBlock) void k_csr_to_ell(int n, int pw, const int *__restrict__ prp,
                                                       const double *__restrict__ pc,
                                                       double *__restrict__ pe)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int e0 = prp[i], np = prp[i + 1] - e0;
    for (int s = 0; s < pw; ++s)
        pe[static_cast<int64_t>(i) * pw + s] = s < np ? pc[e0 + s] : 0.0;
}

// Slot maps (see k_smooth_map): one thread per fine row.
__global__ __launch_bounds__(kBlock) void k_build_maps(int n, int pw, int jw, DiaOffsets joff,
                                                       const int *__restrict__ jcol,
                                                       const int *__restrict__ jrp,
                                                       const int *__restrict__ jci,
                                                       const int *__restrict__ pcol,
                                                       uint32_t *__restrict__ maps)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int o = 0; o < jw; ++o) {
        const int64_t e = static_cast<int64_t>(o) * n + i;
        const int k = jcol ? jcol[e] : i + joff.off[o];
        bool present = false;
        if (k >= 0 && k < n)
            for (int q = jrp[i]; q < jrp[i + 1]; ++q)
                if (jci[q] == k) present = true;
        uint32_t m = 0xFFFFFFFFu;
        if (present) {
            for (int s = 0; s < pw && s < kMapWidth; ++s) {
                const int c = pcol[static_cast<int64_t>(i) * pw + s];
                uint32_t src = 0xFu;
                if (c >= 0)
                    for (int q = 0; q < pw; ++q)
                        if (pcol[static_cast<int64_t>(k) * pw + q] == c) src = static_cast<uint32_t>(q);
                m = (m & ~(0xFu << (4 * s))) | (src << (4 * s));
            }
        }
        maps[e] = m;
    }
}

inline int grid_n(int n) { return grid_for(n); }

template <typename T, typename IDX, int PW, int JW>
void smooth_map_launch(hipStream_t s, const SmoothArgs &a, const T *jv, const T *pin, T *pout)
{
    if constexpr (JW > 0) {
        if (a.sym) {
            if constexpr (PW == 8 && JW == 7 && sizeof(IDX) == 1) {
                if (a.split.tab) {
                    k_smooth_map<T, IDX, 8, 7, true, true><<<grid_n(a.n), kBlock, 0, s>>>(
                        a.n, a.jw, a.joff, a.jcol, jv, static_cast<const IDX *>(a.jmap_idx),
                        a.jmap_tab, a.jmap_ntab, pin, pout, a.interior, a.eit_part, a.omega, a.go,
                        a.split);
                    return;
                }
            }
            k_smooth_map<T, IDX, PW, JW, true><<<grid_n(a.n), kBlock, 0, s>>>(
                a.n, a.jw, a.joff, a.jcol, jv, static_cast<const IDX *>(a.jmap_idx), a.jmap_tab,
                a.jmap_ntab, pin, pout, a.interior, a.eit_part, a.omega, a.go, SplitRows{});
            return;
        }
    }
    k_smooth_map<T, IDX, PW, JW><<<grid_n(a.n), kBlock, 0, s>>>(
        a.n, a.jw, a.joff, a.jcol, jv, static_cast<const IDX *>(a.jmap_idx), a.jmap_tab,
        a.jmap_ntab, pin, pout, a.interior, a.eit_part, a.omega, a.go, SplitRows{});
}

template <typename T, typename IDX, int PW>
void smooth_map_pw(hipStream_t s, const SmoothArgs &a, const T *jv, const T *pin, T *pout)
{
    if constexpr (sizeof(IDX) == 1) {
        // the slot counts of 1D, 2D and 3D stencils and of the 27-point
        // same-component pattern of trilinear elements
        switch (a.jw) {
        case 3: smooth_map_launch<T, IDX, PW, 3>(s, a, jv, pin, pout); return;
        case 5: smooth_map_launch<T, IDX, PW, 5>(s, a, jv, pin, pout); return;
        case 7: smooth_map_launch<T, IDX, PW, 7>(s, a, jv, pin, pout); return;
        case 9: smooth_map_launch<T, IDX, PW, 9>(s, a, jv, pin, pout); return;
        case 27: smooth_map_launch<T, IDX, PW, 27>(s, a, jv, pin, pout); return;
        default: break;
        }
    }
    smooth_map_launch<T, IDX, PW, 0>(s, a, jv, pin, pout);
}

template <typename T, typename IDX>
void smooth_map_t(hipStream_t s, const SmoothArgs &a, const T *jv, const T *pin, T *pout)
{
    if (a.pw <= 4)
        smooth_map_pw<T, IDX, 4>(s, a, jv, pin, pout);
    else
        smooth_map_pw<T, IDX, 8>(s, a, jv, pin, pout);
}

template <typename T>
void smooth_t(hipStream_t s, const SmoothArgs &a, const T *jv, const T *pin, T *pout)
{
    switch (a.jmap_kind) {
    case 1: smooth_map_t<T, uint8_t>(s, a, jv, pin, pout); return;
    case 2: smooth_map_t<T, uint16_t>(s, a, jv, pin, pout); return;
    case 3: smooth_map_t<T, uint32_t>(s, a, jv, pin, pout); return;
    default: break;
    }
    if (a.pw <= 8)
        k_smooth_cmp<T, 8><<<grid_n(a.n), kBlock, 0, s>>>(a.n, a.pw, a.jw, a.joff, a.jcol, jv,
                                                          a.pcol, pin, pout, a.interior, a.eit_part);
    else if (a.pw <= 16)
        k_smooth_cmp<T, 16><<<grid_n(a.n), kBlock, 0, s>>>(a.n, a.pw, a.jw, a.joff, a.jcol, jv,
                                                           a.pcol, pin, pout, a.interior, a.eit_part);
    else
        k_smooth_cmp<T, 32><<<grid_n(a.n), kBlock, 0, s>>>(a.n, a.pw, a.jw, a.joff, a.jcol, jv,
                                                           a.pcol, pin, pout, a.interior, a.eit_part);
}

// Row i's second-half index and whether it has 8 entries (see SplitRows)
__device__ inline bool split_row(const SplitRows &g, int i, int &h)
{
    const int x = i % g.nx, line = i / g.nx, y = line % g.ny, z = line / g.ny;
    const int a = g.tab[x], b = g.tab[g.nx + y], c = g.tab[g.nx + g.ny + z];
    h = (a & 0x7FFFFFFF) + (b & 0x7FFFFFFF) + (c & 0x7FFFFFFF);
    return (a & b & c) < 0;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_p_split(int n, SplitRows g, const T *__restrict__ p,
                                                    T *__restrict__ q)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int h;
    const bool f = split_row(g, i, h);
    const int64_t r = static_cast<int64_t>(i) * 8;
    for (int s = 0; s < 4; ++s) q[static_cast<int64_t>(i) * 4 + s] = p[r + s];
    if (f)
        for (int s = 0; s < 4; ++s)
            q[(static_cast<int64_t>(n) + h) * 4 + s] = p[r + 4 + s];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_p_merge(int n, SplitRows g, const T *__restrict__ q,
                                                    T *__restrict__ p)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int h;
    const bool f = split_row(g, i, h);
    const int64_t r = static_cast<int64_t>(i) * 8;
    for (int s = 0; s < 4; ++s) p[r + s] = q[static_cast<int64_t>(i) * 4 + s];
    for (int s = 0; s < 4; ++s)
        p[r + 4 + s] = f ? q[(static_cast<int64_t>(n) + h) * 4 + s] : T(0);
}

}  // namespace

void launch_p_split(hipStream_t s, int n, const SplitRows &g, bool fp32, const double *p64,
                    const float *p32, double *q64, float *q32)
{
    if (n <= 0) return;
    if (fp32)
        k_p_split<float><<<grid_n(n), kBlock, 0, s>>>(n, g, p32, q32);
    else
        k_p_split<double><<<grid_n(n), kBlock, 0, s>>>(n, g, p64, q64);
}

void launch_p_merge(hipStream_t s, int n, const SplitRows &g, bool fp32, const double *q64,
                    const float *q32, double *p64, float *p32)
{
    if (n <= 0) return;
    if (fp32)
        k_p_merge<float><<<grid_n(n), kBlock, 0, s>>>(n, g, q32, p32);
    else
        k_p_merge<double><<<grid_n(n), kBlock, 0, s>>>(n, g, q64, p64);
}

GridOrder grid_order_for(int n, const DiaOffsets &d)
{
    GridOrder g;
    if (d.n != 7) return g;
    const int a = d.off[6], b = d.off[5];
    const bool stencil = d.off[0] == -a && d.off[1] == -b && d.off[2] == -1 && d.off[3] == 0 &&
                         d.off[4] == 1 && b >= 2 && a > b && a % b == 0;
    if (!stencil || n % a != 0) return g;
    const int nx = b, ny = a / b, nz = n / a;
    if (nz < 2 || ny % 8 != 0 || (static_cast<int64_t>(ny / 8) * nx) % kBlock != 0) return g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.lines = ny / 8;
    g.bps = g.lines * nx / kBlock;
    return g;
}

// The same for a scalar stencil A whose DIA copy (ad, [jw][n], absent
// entries zero) has J's offsets: A is read diagonal by diagonal (coalesced)
// instead of row by row.  Dhat sums the off-diagonals in offset order, which
// is column order, so the values equal k_filter_jacobi's.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_filter_jacobi_dia(int n, int filter, double omega,
                                                              const double *__restrict__ ad,
                                                              DiaOffsets joff, int sym,
                                                              T *__restrict__ jv)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int jw = joff.n;
    int mid = 0;
    for (int o = 0; o < jw; ++o)
        if (joff.off[o] == 0) mid = o;
    double d = 0.0;
    for (int o = 0; o < jw; ++o) {
        if (o == mid) continue;
        double g = ad[static_cast<int64_t>(o) * n + i];
        if (filter && g > 0.0) g = 0.0;
        d -= g;
    }
    for (int o = 0; o < jw; ++o) {
        double v;
        if (sym) {
            if (o < mid) {
                v = 0.0;
            } else if (o == mid) {
                v = d == 0.0 ? 0.0 : -omega / d;
            } else {
                v = ad[static_cast<int64_t>(o) * n + i];
                if (filter && v > 0.0) v = 0.0;
            }
        } else if (d == 0.0) {
            v = o == mid ? 1.0 : 0.0;
        } else if (o == mid) {
            v = 1.0 - omega;
        } else {
            double g = ad[static_cast<int64_t>(o) * n + i];
            if (filter && g > 0.0) g = 0.0;
            v = g == 0.0 ? 0.0 : -omega * g / d;
        }
        jv[static_cast<int64_t>(o) * n + i] = static_cast<T>(v);
    }
}

// The same for a node-block operator (NodeStencil: a row's coefficients by
// node offset and component) when J's diagonals are the node offsets'
// same-component couplings in the same order: row i reads its 27 (say)
// couplings of component i mod BS from their node-offset planes instead of
// walking its whole CSR row.  d is summed over the couplings in ascending
// column order, as in k_filter_jacobi; a coupling of value zero (absent from
// the row, or filtered) gives a zero entry.
template <typename T, int BS>
__global__ __launch_bounds__(kBlock) void k_filter_jacobi_nbs(int n, int filter, double omega,
                                                              NodeStencil ns,
                                                              const double *__restrict__ nsv,
                                                              T *__restrict__ jv)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int ic = i % BS;
    auto coef = [&](int o) {
        double g = nsv[static_cast<int64_t>(o * BS + ic) * n + i];
        if (filter && g > 0.0) g = 0.0;
        return g;
    };
    double d = 0.0;
    for (int o = 0; o < ns.n; ++o)
        if (ns.off[o] != 0) d -= coef(o);
    for (int o = 0; o < ns.n; ++o) {
        double v;
        if (d == 0.0) {
            v = ns.off[o] == 0 ? 1.0 : 0.0;
        } else if (ns.off[o] == 0) {
            v = 1.0 - omega;
        } else {
            const double g = coef(o);
            v = g == 0.0 ? 0.0 : -omega * g / d;
        }
        jv[static_cast<int64_t>(o) * n + i] = static_cast<T>(v);
    }
}

void launch_filter_jacobi(hipStream_t s, int n, int bs, int filter, double omega, const int *rp,
                          const int *ci, const double *a, int jw, const DiaOffsets &joff,
                          bool use_dia, bool sym, double *jv64, float *jv32, const double *ad,
                          const NodeStencil *ns, const double *nsv)
{
    // node-block A whose node offsets are J's diagonals (times bs), in order
    bool nbs = ns && nsv && use_dia && !sym && ns->bs == bs && (bs == 2 || bs == 3) &&
               ns->n == jw && joff.n == jw;
    for (int o = 0; nbs && o < jw; ++o) nbs = joff.off[o] == ns->off[o] * bs;
    if (nbs) {
        auto go = [&](auto bsc) {
            constexpr int BS = decltype(bsc)::value;
            if (jv32)
                k_filter_jacobi_nbs<float, BS><<<grid_for(n), kBlock, 0, s>>>(n, filter, omega, *ns,
                                                                              nsv, jv32);
            else
                k_filter_jacobi_nbs<double, BS><<<grid_for(n), kBlock, 0, s>>>(n, filter, omega,
                                                                               *ns, nsv, jv64);
        };
        if (bs == 3) go(std::integral_constant<int, 3>{});
        else go(std::integral_constant<int, 2>{});
        return;
    }
    if (ad && use_dia && bs == 1) {
        if (jv32)
            k_filter_jacobi_dia<float><<<grid_for(n), kBlock, 0, s>>>(n, filter, omega, ad, joff,
                                                                      sym ? 1 : 0, jv32);
        else
            k_filter_jacobi_dia<double><<<grid_for(n), kBlock, 0, s>>>(n, filter, omega, ad, joff,
                                                                       sym ? 1 : 0, jv64);
        return;
    }
    if (jv32)
        k_filter_jacobi<float><<<grid_for(n), kBlock, 0, s>>>(n, bs, filter, omega, rp, ci, a, jw,
                                                              joff, use_dia ? 1 : 0, sym ? 1 : 0,
                                                              jv32);
    else
        k_filter_jacobi<double><<<grid_for(n), kBlock, 0, s>>>(n, bs, filter, omega, rp, ci, a,
                                                               jw, joff, use_dia ? 1 : 0,
                                                               sym ? 1 : 0, jv64);
}

void launch_init_basis(hipStream_t s, int n, int pw, const int *pcol, const int *part,
                       double *p64, float *p32)
{
    const int64_t m = static_cast<int64_t>(n) * pw;
    if (p32)
        k_init_basis<float><<<grid_for(m), kBlock, 0, s>>>(m, pw, pcol, part, p32);
    else
        k_init_basis<double><<<grid_for(m), kBlock, 0, s>>>(m, pw, pcol, part, p64);
}

void launch_smooth(hipStream_t s, const SmoothArgs &a, bool fp32, const double *jv64,
                   const float *jv32, const double *pin64, double *pout64, const float *pin32,
                   float *pout32)
{
    if (fp32)
        smooth_t<float>(s, a, jv32, pin32, pout32);
    else
        smooth_t<double>(s, a, jv64, pin64, pout64);
    if (a.eit_part) k_eit_final<<<1, 1024, 0, s>>>(grid_n(a.n), a.eit_part, a.eit_out);
}

void launch_basis_stats(hipStream_t s, int n, int pw, const int *pcol, bool fp32,
                        const double *p64, const float *p32, double *partials, double *out3)
{
    const int64_t m = static_cast<int64_t>(n) * pw;
    const int nb = std::min(2048, std::max(1, grid_for(pw == 4 || pw == 8 ? m : n)));
    if (pw == 8) {
        if (fp32)
            k_basis_stats_e<float, 8><<<nb, kBlock, 0, s>>>(m, pcol, p32, partials);
        else
            k_basis_stats_e<double, 8><<<nb, kBlock, 0, s>>>(m, pcol, p64, partials);
    } else if (pw == 4) {
        if (fp32)
            k_basis_stats_e<float, 4><<<nb, kBlock, 0, s>>>(m, pcol, p32, partials);
        else
            k_basis_stats_e<double, 4><<<nb, kBlock, 0, s>>>(m, pcol, p64, partials);
    } else if (fp32) {
        k_basis_stats<float><<<nb, kBlock, 0, s>>>(n, pw, pcol, p32, partials);
    } else {
        k_basis_stats<double><<<nb, kBlock, 0, s>>>(n, pw, pcol, p64, partials);
    }
    k_basis_stats_final<<<1, kBlock, 0, s>>>(nb, partials, out3);
}

void launch_p_convert(hipStream_t s, int64_t m, const float *src, double *dst)
{
    if (m > 0) k_convert<float, double><<<grid_for(m), kBlock, 0, s>>>(m, src, dst);
}

void launch_p_convert_down(hipStream_t s, int64_t m, const double *src, float *dst)
{
    if (m > 0) k_convert<double, float><<<grid_for(m), kBlock, 0, s>>>(m, src, dst);
}

void launch_ell_to_csr(hipStream_t s, int n, int pw, const int *prp, bool fp32,
                       const double *pe64, const float *pe32, double *pcsr)
{
    if (fp32)
        k_ell_to_csr<float><<<grid_for(n), kBlock, 0, s>>>(n, pw, prp, pe32, pcsr);
    else
        k_ell_to_csr<double><<<grid_for(n), kBlock, 0, s>>>(n, pw, prp, pe64, pcsr);
}

void launch_csr_to_ell(hipStream_t s, int n, int pw, const int *prp, const double *pcsr,
                       double *pe64)
{
    k_csr_to_ell<<<grid_for(n), kBlock, 0, s>>>(n, pw, prp, pcsr, pe64);
}

void launch_build_maps(hipStream_t s, int n, int pw, int jw, const DiaOffsets &joff,
                       const int *jcol, const int *jrp, const int *jci, const int *pcol,
                       uint32_t *maps)
{
    k_build_maps<<<grid_for(n), kBlock, 0, s>>>(n, pw, jw, joff, jcol, jrp, jci, pcol, maps);
}

}  // namespace msrsb
