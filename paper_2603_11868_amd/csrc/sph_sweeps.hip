// Pair sweeps of libsph: sorted sweep records, neighbour traversal (direct
// search over the 3^d nearest cells, Sec. 5 of the paper), the per-step
// neighbour list, and the density and force sweeps.
//
// Fluid sweep record, two 4-vectors per particle, rec[2k] = A, rec[2k+1] = B:
//   3D  A = (x, y, z, vx)   B = (vy, vz, rho, P)
//   2D  A = (x, y, vx, vy)  B = (rho, P, -, -)
// x is the FP64 position on the FP64 path.  On the mixed path it is the
// offset from the centre of the particle's cell as a 32-bit fixed-point
// number in units of 2^-30 cs (the bits of an int32 in the float slot), and
// every other component is FP32.  k_pack writes A and the velocity half of
// B; the density sweep writes (rho, P).  One particle's data for the force
// sweep is one 64-byte (FP64) or 32-byte (mixed) block.  Walls: wpos (FP64
// position, or the fixed-point offset).  Both paths keep FP32 offsets from the
// cell origin, in metres (cpos, wcpos), for cheap candidate tests.
//
// Mixed-path geometry.  Pair arithmetic runs in units of the cell size cs.
// A pair vector is t - q_j 2^-31, t = q_i 2^-31 - (c_j - c_i) in FP32 for
// the force and the continuity term; the density summation forms the exact
// integer difference (q_i - (c_j - c_i) 2^31) - q_j in FP64 and evaluates
// the kernel there: the summation density sets the pressure
// p = c0^2 (rho - rho0), which magnifies its rounding by rho0 / (rho - rho0),
// so it needs the FP64 sum of FP64 kernel values, while the force sum does not.
#include "sph_step_common.h"

#include <type_traits>

namespace sphx {

// Neighbour-list entries, 32 bits: source slot in bits 0..24; on the mixed path
// the source cell's offset from the target cell in bits 25..30 (two bits per
// axis, offset + 1); wall flag in bit 31.
// List walks gather records cooperatively (walk_coop).
constexpr bool kCoopWalk = true;
template <int DIM, bool MIXED> constexpr bool use_coop() { return kCoopWalk; }
// List positions fetched at a time by the cooperative walks (1, 2, 4, 6 or 8;
// six and eight read three and two quads of entries per iteration).  Measured
// on the 2.0 M-particle 3D dam break: eight in the density walks (FP64
// 739 -> 630 us, mixed 500 -> 420 us) and the 3D mixed force (528 -> 417 us);
// six in the 3D FP64 force (716 -> 673 us; eight leave two waves per SIMD:
// 782 us); four in the 2D forces (64-instance 2D batch: mixed 554 -> 589 us
// with eight, FP64 795 -> 916 us with six) and in the dual scheme's sweeps
// (six: no change; eight: 5 % slower).  On the 29 M-particle case, eight
// stay best in the mixed density walk (six: +17 %, four: +29 %) and equal
// six in the mixed force.
constexpr int kCoopRoundsWalk = 8, kCoopRoundsDual = 4;
template <int DIM, bool MIXED> constexpr int coop_rounds_force() { return DIM == 3 ? (MIXED ? 8 : 6) : 4; }
// List entries in flight per lane in the per-lane walks (walk_list: every
// walk when the cooperative gather is off).  Deep prefetch beats occupancy in these L1-bound walks: measured on
// the 2.0 M-particle 3D dam break, 16 entries in flight at 2 waves per SIMD
// (FP64) were faster than 8 at 3 or 4 at 5.
template <int DIM, bool MIXED> constexpr int skin_walk_u() { return 16; }
template <int DIM, bool MIXED> constexpr int force_walk_u() { return MIXED && DIM == 3 ? 16 : 8; }
constexpr int kDualWalkU = 4;          // the sub-step sweeps of the dual scheme (FP64): 8 was slower

constexpr int kSlotBits = 25;
constexpr unsigned kSlotMask = (1u << kSlotBits) - 1u;
constexpr unsigned kWallBit = 0x80000000u;

__device__ __forceinline__ unsigned offset_bits(int ox, int oy, int oz)
{
    return (unsigned)((ox + 1) | ((oy + 1) << 2) | ((oz + 1) << 4)) << kSlotBits;
}

// Element s of an array addressed with a 32-bit byte offset (list sweeps only:
// they handle fewer than 2^25 particles per kind, so s * sizeof(T) < 2^32).
template <class T>
__device__ __forceinline__ T ld32(const T *__restrict__ base, int s)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                        (uint32_t)s * (uint32_t)sizeof(T));
}

template <int DIM> struct Cand;
template <> struct Cand<2> { using t = fvec2; };
template <> struct Cand<3> { using t = fvec4; };

// Record access for one (dimension, precision).
template <int DIM, bool MIXED>
struct RV {
    using R = Rec<DIM, MIXED>;
    using real = typename R::real;
    using v4 = typename R::v4;
    using v2 = typename R::v2;
    using wpos_t = typename R::wpos_t;

    // position (mixed: offset from the cell centre in units of cs)
    __device__ __forceinline__ static real coord(real bits)
    {
        if constexpr (MIXED) return (float)__float_as_int(bits) * kQUnit;
        else return bits;
    }
    __device__ __forceinline__ static void pos(const v4 &A, real *p)
    {
        p[0] = coord(A.x);
        p[1] = coord(A.y);
        if constexpr (DIM == 3) p[2] = coord(A.z);
        else p[2] = 0;
    }
    __device__ __forceinline__ static void wall_pos(const wpos_t &w, real *p)
    {
        p[0] = coord(w.x);
        p[1] = coord(w.y);
        if constexpr (DIM == 3) p[2] = coord(w.z);
        else p[2] = 0;
    }
    // a wall record as the A vector of a source (position, zero velocity)
    __device__ __forceinline__ static v4 wall_A(const wpos_t &w)
    {
        v4 A{};
        A.x = w.x;
        A.y = w.y;
        if constexpr (DIM == 3) A.z = w.z;
        return A;
    }
    // fixed-point position (mixed path)
    __device__ __forceinline__ static void qpos(const v4 &A, int *q)
    {
        q[0] = __float_as_int((float)A.x);
        q[1] = __float_as_int((float)A.y);
        q[2] = DIM == 3 ? __float_as_int((float)A.z) : 0;
    }
    // velocity from A and the first half of B
    __device__ __forceinline__ static void vel(const v4 &A, const v4 &B, real *v)
    {
        if constexpr (DIM == 3) {
            v[0] = A.w;
            v[1] = B.x;
            v[2] = B.y;
        } else {
            v[0] = A.z;
            v[1] = A.w;
            v[2] = 0;
        }
    }
    __device__ __forceinline__ static real rho(const v4 &B) { if constexpr (DIM == 3) return B.z; else return B.x; }
    __device__ __forceinline__ static real P(const v4 &B) { if constexpr (DIM == 3) return B.w; else return B.y; }
    // the v2 slot of B that holds (rho, P), counted in v2 units from rec
    __device__ __forceinline__ static int64_t rhoP_slot(int k) { return 4 * (int64_t)k + (DIM == 3 ? 3 : 2); }
    // loads of A, the velocity half of B (3D), the whole B
    __device__ __forceinline__ static v4 loadA(const v4 *__restrict__ rec, int s) { return rec[2 * (int64_t)s]; }
    __device__ __forceinline__ static v4 loadB(const v4 *__restrict__ rec, int s)
    {
        if constexpr (DIM == 3) {
            return rec[2 * (int64_t)s + 1];
        } else {
            const v2 h = reinterpret_cast<const v2 *>(rec)[4 * (int64_t)s + 2];
            v4 B{};
            B.x = h.x;
            B.y = h.y;
            return B;
        }
    }
    __device__ __forceinline__ static v4 loadBv(const v4 *__restrict__ rec, int s)
    {
        v4 B{};
        if constexpr (DIM == 3) {
            const v2 h = reinterpret_cast<const v2 *>(rec)[4 * (int64_t)s + 2];
            B.x = h.x;
            B.y = h.y;
        }
        (void)rec;
        (void)s;
        return B;
    }
};

// Mixed path: squared distance of a pair from the fixed-point positions, in
// fixed-point units (2^-31 cs)^2.  qs: the target's offsets plus 2^31, as
// FP64; Aj: the source's A vector (or wall record); e: a list entry, whose
// bits 25..30 hold the source cell's offset from the target cell per axis,
// plus one.  The difference (q_i - (c_j - c_i) 2^31) - q_j is formed in FP64,
// where every term is an integer below 2^33 and exact, so the result has a
// single rounding per square and sum, for any pair.
template <int DIM>
__device__ __forceinline__ double exact_r2(const double *qs, const fvec4 &Aj, unsigned e)
{
    const int qj[3] = {__float_as_int(Aj.x), __float_as_int(Aj.y), DIM == 3 ? __float_as_int(Aj.z) : 0};
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned o1 = (e >> (25 + 2 * a)) & 3u;       // cell offset + 1
        const double d = fma((double)o1, -kQScale, qs[a]) - (double)qj[a];
        r2 = fma(d, d, r2);
    }
    return r2;
}

// The target side of exact_r2.
template <int DIM>
__device__ __forceinline__ void exact_target(const int *qi, double *qs)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) qs[a] = a < DIM ? (double)qi[a] + kQScale : 0.0;
}

// r^2 bound of the walks' pair test.  The FP64 path and the mixed force
// decide with it; the mixed density sweep (EXACT) widens it by 2e-6 and
// decides with exact_r2.
template <bool MIXED, bool EXACT = false>
__device__ __forceinline__ auto walk_cut2(const SimConst &sc)
{
    if constexpr (MIXED) return EXACT ? sc.ucut2 * 1.000002f : sc.ucut2;
    else return sc.cut2;
}

// Whether a density walk skips list entries at r^2 >= cut2 itself.  A list
// holds every pair its build found closer than the build radius with an FP32
// test and a margin of 1e-4 in r^2 -- a superset of the pairs -- so every walk
// decides each entry: the FP64 walks with r^2 < (2h)^2 in FP64, the forces
// with the r^2 of their own precision, and the mixed density sweep with the
// exact fixed-point test inside its pair function (with a skin, the FP32 test
// of the walk first skips the entries well beyond 2h).
template <bool MIXED, int LIST>
constexpr bool density_chk() { return !MIXED || LIST == 3; }

// How much of B a sweep needs from each fluid source.
enum { NEED_NONE = 0, NEED_VEL = 1, NEED_ALL = 2 };

template <int DIM, bool MIXED, int NEED>
__device__ __forceinline__ typename RV<DIM, MIXED>::v4 load_need(const typename RV<DIM, MIXED>::v4 *__restrict__ rec,
                                                                 int s)
{
    using V = RV<DIM, MIXED>;
    if constexpr (NEED == NEED_ALL) return V::loadB(rec, s);
    else if constexpr (NEED == NEED_VEL) return V::loadBv(rec, s);
    else return typename V::v4{};
}

// Pair vector r = t - x_j, where t is the target position seen from the
// source's cell.  FP64: positions are absolute and t = x_i.  FP32: offsets from
// the cell origins, and t = o_i - (c_j - c_i) cs with c_j - c_i in {-1, 0, 1}
// per axis; that product is exact, so t is one rounding of the difference
// whether or not the compiler fuses it.
template <int DIM, bool MIXED, class real>
__device__ __forceinline__ void shift_target(const real *pi, int ox, int oy, int oz, real cs, real *t)
{
    if constexpr (MIXED) {
        t[0] = pi[0] - (real)ox * cs;
        t[1] = pi[1] - (real)oy * cs;
        t[2] = DIM == 3 ? pi[2] - (real)oz * cs : (real)0;
    } else {
        (void)ox; (void)oy; (void)oz; (void)cs;
        t[0] = pi[0];
        t[1] = pi[1];
        t[2] = pi[2];
    }
}

template <int DIM, class real>
__device__ __forceinline__ void sub_vec(const real *t, const real *pj, real *r)
{
    r[0] = t[0] - pj[0];
    r[1] = t[1] - pj[1];
    r[2] = DIM == 3 ? t[2] - pj[2] : (real)0;
}

// Shifted targets of one stencil row: the row spans cells xlo..xhi (at most
// three), and a source slot s lies in cell xlo + (s >= b1) + (s >= b2).
template <int DIM, bool SHIFT, class real>
struct RowTarget {
    real x, cs, ty, tz;
    int b1, b2, ox0, oy, oz;
    __device__ __forceinline__ void init(const real *pi, int ox, int dy, int dz, real cs_, int b1_, int b2_)
    {
        b1 = b1_;
        b2 = b2_;
        ox0 = ox;
        oy = dy;
        oz = dz;
        cs = cs_;
        x = pi[0];
        real t[3];
        shift_target<DIM, SHIFT>(pi, ox, dy, dz, cs, t);
        ty = t[1];
        tz = t[2];
    }
    __device__ __forceinline__ int ox(int s) const { return ox0 + (s >= b1) + (s >= b2); }
    __device__ __forceinline__ void at(int s, real *t) const
    {
        if constexpr (SHIFT) t[0] = x - (real)ox(s) * cs;
        else t[0] = x;
        t[1] = ty;
        t[2] = tz;
    }
    // list-entry offset bits of slot s
    __device__ __forceinline__ unsigned bits(int s) const { return offset_bits(ox(s), oy, oz); }
};

template <int DIM, class real>
__device__ __forceinline__ real norm2(const real *r)
{
    if constexpr (DIM == 3) return dist2(r[0], r[1], r[2]);
    else return dist2(r[0], r[1]);
}

// ---------------------------------------------------------------------------
// sweep records
// ---------------------------------------------------------------------------

// Fixed-point offset of a coordinate from the centre of its cell, in units of
// 2^-31 cs, as the bits of an int32 (mixed path).  |q| < 0.75 2^31 for any
// particle inside the cells of its last build (it has moved less than
// skin / 2 <= cs / 4 out of them); a particle far outside them (a clamped
// key) saturates.
__device__ __forceinline__ float qfix(double off_origin, double cs, double inv_cs)
{
    double u = rint((off_origin - 0.5 * cs) * (inv_cs * kQScale));
    u = fmin(fmax(u, -2147483647.0), 2147483647.0);
    return __int_as_float((int)u);
}

template <int DIM>
__device__ __forceinline__ void cell_offset_f64(const SimConst &sc, const double *xi, const InstDev &I, int lk,
                                                double *o)
{
    int cx, cy, cz;
    cell_coords(sc, I, lk, cx, cy, cz);
    o[0] = xi[0] - (I.lo[0] + cx * sc.cs);
    o[1] = xi[1] - (I.lo[1] + cy * sc.cs);
    o[2] = DIM == 3 ? xi[2] - (I.lo[2] + cz * sc.cs) : 0.0;
}

template <int DIM, bool MIXED>
__global__ __launch_bounds__(kMaxBlock) void k_pack(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    double *__restrict__ x, double *__restrict__ v, const int *__restrict__ perm,
    const int *__restrict__ skey, int n, typename Rec<DIM, MIXED>::v4 *__restrict__ rec,
    typename Cand<DIM>::t *__restrict__ cpos, const int *__restrict__ gate,
    const double *__restrict__ a, const double *__restrict__ dt, int kick_on)
{
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    const InstDev &I = inst[ch.inst];
    const int i = perm[k];
    const int lk = skey[k] - I.cell_base;
    double xi[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        xi[c] = x[(int64_t)c * n + i];
        vi[c] = v[(int64_t)c * n + i];
    }
    // a step that reuses its cell table (no keys, no sort) kicks and drifts
    // here, on its way to the records: one pass over the state instead of two
    if (kick_on && gate != nullptr && *gate == 0) {
        const double dtb = dt[ch.inst];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            kick_drift(xi[c], vi[c], a[(int64_t)c * n + i], dtb);
            x[(int64_t)c * n + i] = xi[c];
            v[(int64_t)c * n + i] = vi[c];
        }
    }
    double od[3];
    cell_offset_f64<DIM>(sc, xi, I, lk, od);
    real p[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (MIXED) p[c] = qfix(od[c], sc.cs, sc.inv_cs);
        else p[c] = xi[c];
    }
    // whole records: (rho, P) get zeros here and their values from the density
    // sweep, which runs before anything reads them; writing every byte of the
    // record's sectors spares the memory a read-modify-write of partial ones
    typename V::v4 A, B{};
    if constexpr (DIM == 3) {
        A.x = p[0]; A.y = p[1]; A.z = p[2]; A.w = (real)vi[0];
        B.x = (real)vi[1];
        B.y = (real)vi[2];
    } else {
        A.x = p[0]; A.y = p[1]; A.z = (real)vi[0]; A.w = (real)vi[1];
    }
    rec[2 * (int64_t)k] = A;
    rec[2 * (int64_t)k + 1] = B;
    // the FP32 copies serve the candidate tests, which only a build runs
    if (gate == nullptr || *gate != 0) {
        typename Cand<DIM>::t cp;
        cp.x = (float)od[0];
        cp.y = (float)od[1];
        if constexpr (DIM == 3) { cp.z = (float)od[2]; cp.w = 0.0f; }
        cpos[k] = cp;
    }
}

template <int DIM, bool MIXED>
__global__ __launch_bounds__(kMaxBlock) void k_wall_pack(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const double *__restrict__ xw, const int *__restrict__ wperm, const int *__restrict__ wskey,
    int nw, typename Rec<DIM, MIXED>::wpos_t *__restrict__ wpos, typename Cand<DIM>::t *__restrict__ wcpos)
{
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    const InstDev &I = inst[ch.inst];
    const int j = wperm[k];
    double xj[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < DIM; ++c) xj[c] = xw[(int64_t)c * nw + j];
    double od[3];
    cell_offset_f64<DIM>(sc, xj, I, wskey[k] - I.cell_base, od);
    real p[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (MIXED) p[c] = qfix(od[c], sc.cs, sc.inv_cs);
        else p[c] = xj[c];
    }
    typename V::wpos_t w;
    w.x = p[0];
    w.y = p[1];
    if constexpr (DIM == 3) {
        w.z = p[2];
        w.w = 0;
    } else if constexpr (MIXED) {
        w.z = 0;                           // 16-byte record: zero velocity
        w.w = 0;
    }
    wpos[k] = w;
    typename Cand<DIM>::t cp;
    cp.x = (float)od[0];
    cp.y = (float)od[1];
    if constexpr (DIM == 3) { cp.z = (float)od[2]; cp.w = 0.0f; }
    wcpos[k] = cp;
}

template <int DIM, bool MIXED>
static void pack_dispatch(const SimConst &sc, const Dev &d, int kick_on, hipStream_t s)
{
    k_pack<DIM, MIXED><<<d.nfchunks, d.block, 0, s>>>(
        sc, d.fmap, d.inst, d.x, d.v, d.perm, d.skey, sc.N,
        static_cast<typename Rec<DIM, MIXED>::v4 *>(d.rec), static_cast<typename Cand<DIM>::t *>(d.cpos), d.gate,
        d.a, d.dt, kick_on);
}

hipError_t launch_pack(const SimConst &sc, const Dev &d, int mixed, hipStream_t s, int kick_on)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) pack_dispatch<2, true>(sc, d, kick_on, s); else pack_dispatch<2, false>(sc, d, kick_on, s); }
    else { if (mixed) pack_dispatch<3, true>(sc, d, kick_on, s); else pack_dispatch<3, false>(sc, d, kick_on, s); }
    return hipGetLastError();
}

template <int DIM, bool MIXED>
static void wall_pack_dispatch(const SimConst &sc, const Dev &d, hipStream_t s)
{
    k_wall_pack<DIM, MIXED><<<d.nwchunks, d.block, 0, s>>>(
        sc, d.wmap, d.inst, d.xw, d.wall_perm, d.wskey, sc.Nw,
        static_cast<typename Rec<DIM, MIXED>::wpos_t *>(d.wpos), static_cast<typename Cand<DIM>::t *>(d.wcpos));
}

hipError_t launch_wall_pack(const SimConst &sc, const Dev &d, int mixed, hipStream_t s)
{
    if (d.nwchunks <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) wall_pack_dispatch<2, true>(sc, d, s); else wall_pack_dispatch<2, false>(sc, d, s); }
    else { if (mixed) wall_pack_dispatch<3, true>(sc, d, s); else wall_pack_dispatch<3, false>(sc, d, s); }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stencil geometry
// ---------------------------------------------------------------------------

struct CellPos {
    int cx, cy, cz;
};

__device__ __forceinline__ CellPos decode_cell(const SimConst &sc, const InstDev &I, int lk)
{
    CellPos c;
    cell_coords(sc, I, lk, c.cx, c.cy, c.cz);
    return c;
}

// Slot ranges of the cells xlo..xhi of stencil row (yy, zz).  Row-major keys:
// one range (the row is contiguous), split at cells b1, b2.  Tiled Morton
// keys: one range per cell.
struct RowSeg {
    int s0, s1, b1, b2, x0;
};

__device__ __forceinline__ int row_segments(const SimConst &sc, int xlo, int xhi)
{
    return sc.key_order == 0 ? 1 : xhi - xlo + 1;
}

__device__ __forceinline__ RowSeg row_segment(const SimConst &sc, const InstDev &I, const int *__restrict__ st,
                                              int g, int xlo, int xhi, int yy, int zz, bool split)
{
    RowSeg r;
    if (sc.key_order == 0) {
        const int row = I.cell_base + (yy + I.ncell[1] * zz) * I.ncell[0];
        r.s0 = st[row + xlo];
        r.s1 = st[row + xhi + 1];
        r.b1 = split && xlo + 1 <= xhi ? st[row + xlo + 1] : r.s1;
        r.b2 = split && xlo + 2 <= xhi ? st[row + xlo + 2] : r.s1;
        r.x0 = xlo;
    } else {
        const int kc = I.cell_base + cell_key(sc, I, xlo + g, yy, zz);
        r.s0 = st[kc];
        r.s1 = st[kc + 1];
        r.b1 = r.s1;
        r.b2 = r.s1;
        r.x0 = xlo + g;
    }
    return r;
}

// Offsets of a target inside its own cell, per axis (in [0, cs) up to rounding).
template <int DIM, bool MIXED>
__device__ __forceinline__ void target_offsets(const SimConst &sc, const InstDev &I, const CellPos &c,
                                               const typename RV<DIM, MIXED>::real *pi,
                                               typename RV<DIM, MIXED>::real *o)
{
    if constexpr (MIXED) {
        // pi: offsets from the cell centre in units of cs
        o[0] = pi[0] + 0.5f;
        o[1] = pi[1] + 0.5f;
        o[2] = DIM == 3 ? pi[2] + 0.5f : 0.0f;
    } else {
        o[0] = pi[0] - (I.lo[0] + c.cx * sc.cs);
        o[1] = pi[1] - (I.lo[1] + c.cy * sc.cs);
        o[2] = DIM == 3 ? pi[2] - (I.lo[2] + c.cz * sc.cs) : 0.0;
    }
}

// Stencil row (dy, dz) of a target with in-cell offsets o: false when every
// point of the row is at least 2h + skin away, else the x range of cells that
// can hold a neighbour.  cut2m is (2h + skin)^2 enlarged by a margin far above
// the rounding of o, so a skipped cell never holds a particle that passes the
// r^2 < (2h + skin)^2 predicate.  With a skin the cells are those of the last
// build and particles have moved by less than skin / 2 since, so a particle
// closer than 2h is never skipped either.
template <class real>
__device__ __forceinline__ bool row_cells(const real *o, real cs, real cut2m, int dy, int dz, int cx,
                                          int ncx, int &xlo, int &xhi)
{
    real d2 = 0;
    if (dy < 0) d2 += o[1] * o[1];
    else if (dy > 0) { const real t = cs - o[1]; d2 += t * t; }
    if (dz < 0) d2 += o[2] * o[2];
    else if (dz > 0) { const real t = cs - o[2]; d2 += t * t; }
    if (d2 >= cut2m) return false;
    xlo = (cx > 0 && o[0] * o[0] + d2 < cut2m) ? cx - 1 : cx;
    const real t = cs - o[0];
    xhi = (cx < ncx - 1 && t * t + d2 < cut2m) ? cx + 1 : cx;
    return true;
}

template <bool MIXED>
__device__ __forceinline__ auto cull_margin(const SimConst &sc)
{
    if constexpr (MIXED) return sc.ubcut2 * (float)(1.0 + 1e-5);     // units of cs
    else return sc.bcut2 * (1.0 + 1e-9);
}

// ---------------------------------------------------------------------------
// direct search: fn(wall, s, r, r2, A_j, B_j, e) for every neighbour of target
// k (r^2 < cut2), fluid slots of a stencil row first, then its wall slots;
// rows in z, y order.  e carries the source's list-entry bits (wall flag, slot
// and the source cell's offset from the target cell).
// ---------------------------------------------------------------------------

template <int DIM, bool MIXED, int NEED, class Fn>
__device__ __forceinline__ void for_neighbours(const SimConst &sc, const InstDev &I, int lk, int k,
                                               const typename RV<DIM, MIXED>::real *pi,
                                               const int *__restrict__ cstart, const int *__restrict__ wstart,
                                               const typename RV<DIM, MIXED>::v4 *__restrict__ rec,
                                               const typename RV<DIM, MIXED>::wpos_t *__restrict__ wpos,
                                               typename RV<DIM, MIXED>::real cut2, Fn &&fn)
{
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    using v4 = typename V::v4;
    const CellPos c = decode_cell(sc, I, lk);
    const int ncx = I.ncell[0], ncy = I.ncell[1], ncz = I.ncell[2];
    const real cs = MIXED ? (real)1 : (real)sc.cs;
    const real cut2m = cull_margin<MIXED>(sc);
    real o[3];
    target_offsets<DIM, MIXED>(sc, I, c, pi, o);
    const int dz_lo = (DIM == 3 && c.cz > 0) ? -1 : 0;
    const int dz_hi = (DIM == 3 && c.cz < ncz - 1) ? 1 : 0;
    for (int dz = dz_lo; dz <= dz_hi; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = c.cy + dy;
            if (yy < 0 || yy >= ncy) continue;
            int xlo, xhi;
            if (!row_cells(o, cs, cut2m, dy, dz, c.cx, ncx, xlo, xhi)) continue;
            const int nseg = row_segments(sc, xlo, xhi);
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                const int *__restrict__ st = pass == 0 ? cstart : wstart;
              for (int g = 0; g < nseg; ++g) {
                // cell boundaries inside the row matter only for the FP32 offsets
                const RowSeg sg = row_segment(sc, I, st, g, xlo, xhi, yy, c.cz + dz, MIXED);
                const int s0 = sg.s0, s1 = sg.s1;
                RowTarget<DIM, MIXED, real> rt;
                rt.init(pi, sg.x0 - c.cx, dy, dz, cs, sg.b1, sg.b2);
                for (int s = s0; s < s1; ++s) {
                    if (pass == 0 && s == k) continue;
                    const v4 A = pass == 0 ? V::loadA(rec, s) : V::wall_A(wpos[s]);
                    real pj[3], t[3], r[3];
                    V::pos(A, pj);
                    rt.at(s, t);
                    sub_vec<DIM>(t, pj, r);
                    const real r2 = norm2<DIM>(r);
                    if (r2 < cut2) {
                        const unsigned e = (pass == 0 ? 0u : kWallBit) | (unsigned)s | rt.bits(s);
                        if (pass == 0) fn(false, s, r, r2, A, load_need<DIM, MIXED, NEED>(rec, s), e);
                        else fn(true, s, r, r2, A, v4{}, e);
                    }
                }
              }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// neighbour list
//
// The density sweep tests the candidates once and writes each target's hits to
// a slot-major list of 16-byte quads, quad q of target k at nlist[q * N + k];
// its own pair loop and the whole force sweep then walk that list: the force
// sweep tests no candidates, and a wave reads 1 KiB contiguous per quad.  A
// target with more than `cap` neighbours walks the stencil instead (the same
// neighbours, in the direct search's row order) and raises SPH_FLAG_CAPACITY.
// A list holds the fluid slots of the target's own stencil row first, then
// the other rows in z, y order, fluid then wall slots: the nearest sources,
// whose records sit beside the target's, are gathered first.
// ---------------------------------------------------------------------------

// Phase 1: candidate tests of target k, hits appended to its list.  Returns the
// number of hits (possibly above cap; only the first cap are stored).
//
// Candidates are read as FP32 offsets from their cell's origin (the cpos and
// wcpos copies), U per lane in flight, with the index clamped instead of
// branched.  A candidate is a hit when its FP32 r^2 is below the build radius
// (2h + skin)^2 times (1 + 1e-4); the FP32 r^2 of a pair is within ~1e-5 of
// the exact one, so the list holds every pair closer than the build radius
// and a few just beyond it, which the walks skip with their own exact test.
// On the FP64 path a target far outside its cell (a clamped particle) takes
// the FP64 test for every candidate.  Hits enter a four-entry shift register
// that is stored as one quad whenever it fills.
template <int DIM, bool MIXED, int U>
__device__ __forceinline__ int build_list(const SimConst &sc, const InstDev &I, int lk, int k,
                                          const typename RV<DIM, MIXED>::real *pi, const float *ci,
                                          const int *__restrict__ cstart, const int *__restrict__ wstart,
                                          const typename RV<DIM, MIXED>::v4 *__restrict__ rec,
                                          const typename RV<DIM, MIXED>::wpos_t *__restrict__ wpos,
                                          const typename Cand<DIM>::t *__restrict__ cpos,
                                          const typename Cand<DIM>::t *__restrict__ wcpos,
                                          uint4 *__restrict__ nlist, int cap, int n)
{
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    const CellPos c = decode_cell(sc, I, lk);
    const int ncx = I.ncell[0], ncy = I.ncell[1], ncz = I.ncell[2];
    // row culling: FP64 offsets on the FP64 path, the FP32 copies (metres) on
    // the mixed path
    const real cs = MIXED ? (real)sc.fcs : (real)sc.cs;
    const real cut2m = MIXED ? (real)(sc.fbcut2 * (float)(1.0 + 1e-5)) : (real)(sc.bcut2 * (1.0 + 1e-9));
    const float fcs = sc.fcs, fcut2 = sc.fbcut2;       // the build radius (2h + skin)
    real o[3];
    if constexpr (MIXED) {
        o[0] = ci[0];
        o[1] = ci[1];
        o[2] = ci[2];
    } else {
        target_offsets<DIM, MIXED>(sc, I, c, pi, o);
    }
    const float hi = fcut2 * (1.0f + 1e-4f);
    bool far = false;
    if constexpr (!MIXED) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) far |= fabs((double)o[a]) > 4.0 * sc.cs;
    }
    int m = 0;
    uint4 buf = make_uint4(0u, 0u, 0u, 0u);
    const int dz_lo = (DIM == 3 && c.cz > 0) ? -1 : 0;
    const int dz_hi = (DIM == 3 && c.cz < ncz - 1) ? 1 : 0;
    // the fluid (PASS 0) or wall (PASS 1) slots of stencil row (dy, dz)
    auto row = [&](int dz, int dy, auto passc) __attribute__((always_inline)) {
            constexpr int pass = decltype(passc)::value;
            const int yy = c.cy + dy;
            if (yy < 0 || yy >= ncy) return;
            int xlo, xhi;
            if (!row_cells(o, cs, cut2m, dy, dz, c.cx, ncx, xlo, xhi)) return;
            // a needed row is scanned whole: targets of one cell then read the
            // same candidates at the same time, one cache line for all of them
            xlo = c.cx > 0 ? c.cx - 1 : c.cx;
            xhi = c.cx < ncx - 1 ? c.cx + 1 : c.cx;
            const int nseg = row_segments(sc, xlo, xhi);
            {
                const int *__restrict__ st = pass == 0 ? cstart : wstart;
                const unsigned wall_bit = pass == 1 ? kWallBit : 0u;
              for (int g = 0; g < nseg; ++g) {
                const RowSeg sg = row_segment(sc, I, st, g, xlo, xhi, yy, c.cz + dz, true);
                const int s0 = sg.s0, s1 = sg.s1;
                RowTarget<DIM, true, float> rf;      // FP32 candidate test
                rf.init(ci, sg.x0 - c.cx, dy, dz, fcs, sg.b1, sg.b2);
                for (int t0 = s0; t0 < s1; t0 += U) {
                    float cj[U][3];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int s = min(t0 + u, s1 - 1);
                        const typename Cand<DIM>::t w = pass == 0 ? ld32(cpos, s) : ld32(wcpos, s);
                        cj[u][0] = w.x;
                        cj[u][1] = w.y;
                        if constexpr (DIM == 3) cj[u][2] = w.z;
                        else cj[u][2] = 0.0f;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int s = t0 + u;
                        float t[3], r[3];
                        rf.at(s, t);
                        sub_vec<DIM>(t, cj[u], r);
                        const float r2f = norm2<DIM>(r);
                        bool hit = s < s1 && !(pass == 0 && s == k);
                        if constexpr (MIXED) {
                            hit = hit && r2f < hi;
                        } else if (!far) {
                            hit = hit && r2f < hi;
                        } else if (hit) {
                            real pj[3], rr[3];
                            if (pass == 0) V::pos(V::loadA(rec, s), pj);
                            else V::wall_pos(wpos[s], pj);
                            sub_vec<DIM>(pi, pj, rr);
                            hit = norm2<DIM>(rr) < (real)sc.bcut2;
                        }
                        if (hit) {
                            unsigned e = wall_bit | (unsigned)s;
                            if constexpr (MIXED) e |= rf.bits(s);
                            buf.x = buf.y;
                            buf.y = buf.z;
                            buf.z = buf.w;
                            buf.w = e;
                            ++m;
                            if ((m & 3) == 0 && m <= cap) nlist[(int64_t)((m >> 2) - 1) * n + k] = buf;
                        }
                    }
                }
              }
            }
    };
    // the centre row's fluid first (it holds the target's own cell), then the
    // other rows in z, y order, fluid then wall slots: the order of the
    // cell-pair build's sequence
    using std::integral_constant;
    row(0, 0, integral_constant<int, 0>{});
    for (int dz = dz_lo; dz <= dz_hi; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            if (dz != 0 || dy != 0) row(dz, dy, integral_constant<int, 0>{});
            row(dz, dy, integral_constant<int, 1>{});
        }
    }
    // the last partial quad: its entries sit in the top (m & 3) words
    const int rest = m & 3;
    if (rest != 0 && m <= cap) {
        uint4 q;
        q.x = rest == 1 ? buf.w : (rest == 2 ? buf.z : buf.y);
        q.y = rest == 2 ? buf.w : buf.z;
        q.z = buf.w;
        q.w = 0u;
        nlist[(int64_t)(m >> 2) * n + k] = q;
    }
    return m;
}

// Phase 2: fn(wall, s, r, r2, A_j, B_j, e) for the first m (<= cap) entries
// of target k; the records of U entries (U = 1, 2, 4, 8 or 16; above 4 a
// round reads U / 4 quads) are fetched before any of them is used.
// CHK: entries with r^2 >= cut2 are skipped (the list is a superset of the
// pairs: built with a margin, or with a skin).
template <int DIM, bool MIXED, int U, int NEED, bool CHK = false, class Fn>
__device__ __forceinline__ void walk_list(const SimConst &sc, int k, int m,
                                          const typename RV<DIM, MIXED>::real *pi,
                                          const typename RV<DIM, MIXED>::v4 *__restrict__ rec,
                                          const typename RV<DIM, MIXED>::wpos_t *__restrict__ wpos,
                                          const uint4 *__restrict__ nlist, int n,
                                          typename RV<DIM, MIXED>::real cut2, Fn &&fn)
{
    static_assert(U == 1 || U == 2 || U == 4 || U == 8 || U == 16, "entries come in quads");
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    using v4 = typename V::v4;
    constexpr int QN = U > 4 ? U / 4 : 1;      // quads per round
    const real cs = MIXED ? (real)1 : (real)sc.cs;
    for (int q0 = 0; q0 < m; q0 += 4 * QN) {
        unsigned eq[4 * QN];
#pragma unroll
        for (int g = 0; g < QN; ++g) {
            // a second quad past the end is not read (its entries are >= m)
            uint4 quad = make_uint4(0u, 0u, 0u, 0u);
            if (g == 0 || q0 + 4 * g < m) quad = nlist[(int64_t)((q0 >> 2) + g) * n + k];
            eq[4 * g] = quad.x;
            eq[4 * g + 1] = quad.y;
            eq[4 * g + 2] = quad.z;
            eq[4 * g + 3] = quad.w;
        }
#pragma unroll
        for (int h = 0; h < 4 * QN; h += U) {
            v4 A[U], B[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (q0 + h + u < m) {
                    const unsigned e = eq[h + u];
                    const int s = (int)(e & kSlotMask);
                    if (e & kWallBit) {             // position only, zero velocity
                        A[u] = V::wall_A(ld32(wpos, s));
                        B[u] = v4{};
                    } else {
                        A[u] = ld32(rec, 2 * s);
                        if constexpr (NEED == NEED_ALL && DIM == 3) B[u] = ld32(rec, 2 * s + 1);
                        else B[u] = load_need<DIM, MIXED, NEED>(rec, s);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (q0 + h + u < m) {
                    const unsigned e = eq[h + u];
                    real pj[3], t[3], r[3];
                    V::pos(A[u], pj);
                    if constexpr (MIXED) {
                        const int ox = (int)((e >> kSlotBits) & 3u) - 1;
                        const int oy = (int)((e >> (kSlotBits + 2)) & 3u) - 1;
                        const int oz = (int)((e >> (kSlotBits + 4)) & 3u) - 1;
                        shift_target<DIM, true>(pi, ox, oy, oz, cs, t);
                    } else {
                        shift_target<DIM, false>(pi, 0, 0, 0, cs, t);
                    }
                    sub_vec<DIM>(t, pj, r);
                    const real r2 = norm2<DIM>(r);
                    if (!CHK || r2 < cut2) fn((e & kWallBit) != 0u, (int)(e & kSlotMask), r, r2, A[u], B[u], e);
                }
            }
        }
    }
}

// Cooperative list walk.  Walks with one record per lane are bound by L1 tag
// lookups: each 16-byte load instruction of a wave touches about 64 cache
// lines.  Here the G lanes of a group (G = 16-byte parts of a record:
// 4 for FP64, 2 for the mixed path's 32-byte records) fetch the parts of each
// other's records: instruction i loads, on lane G g + p, part p of the record
// that lane G g + i needs, so one instruction touches 64 / G lines for whole
// records.  An LDS exchange (stride G + 1 parts: no bank conflicts) then hands
// every lane its own record.  All loads of R list positions are issued before
// any is used.  The wall records follow the fluid records in memory
// (SimConst::wrec_off), so that an entry is one 32-bit byte offset from the
// records' base: the lane that owns the entry forms it, and the group reads
// it with one DPP broadcast per part, fused with the add of the lane's part
// offset.  Parts past the end of a (shorter) wall record are read from the
// records after it (the region ends with 64 bytes of padding) and zeroed on
// the way out of the LDS; a position without an entry reads record 0 and is
// not used.  Every lane of the wave must call this, with m = 0 for a lane
// with nothing to walk.

// Value of lane G * (lane / G) + I within groups of G = 4 or 2 lanes (DPP
// quad permutation); 0 from a disabled lane.
template <int G, int I>
__device__ __forceinline__ unsigned group_bcast(int v)
{
    constexpr int ctrl = G == 4 ? I * 0x55 : (I | (I << 2) | ((2 + I) << 4) | ((2 + I) << 6));
    return (unsigned)__builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, true);
}

// An empty register constraint on a loaded part: the load stays a load into
// registers where it is written.  A load whose value only goes to an LDS
// store becomes a global-to-LDS copy placed at the store, after the previous
// position's pairs, which leaves one position's loads in flight instead of R.
__device__ __forceinline__ void in_registers(dvec2 &v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }
__device__ __forceinline__ void in_registers(fvec4 &v) { asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w)); }

template <int DIM, bool MIXED, int NEED, bool CHK, int R, class Fn>
__device__ __forceinline__ void walk_coop(const SimConst &sc, int k, int m,
                                          const typename RV<DIM, MIXED>::real *pi,
                                          const typename RV<DIM, MIXED>::v4 *__restrict__ rec,
                                          const uint4 *__restrict__ nlist, int n,
                                          typename RV<DIM, MIXED>::real cut2, Fn &&fn)
{
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    using v4 = typename V::v4;
    using part_t = std::conditional_t<MIXED, fvec4, dvec2>;     // 16 bytes
    static_assert(R == 1 || R == 2 || R == 4 || R == 6 || R == 8, "positions per batch: 1, 2, 4, 6 or 8");
    constexpr int G = MIXED ? 2 : 4;
    // 16-byte parts a sweep needs, of a fluid record and of a wall record
    constexpr int NP = MIXED ? (NEED != NEED_NONE ? 2 : 1)
                             : (DIM == 3 ? (NEED == NEED_ALL ? 4 : (NEED == NEED_VEL ? 3 : 2))
                                         : (NEED == NEED_ALL ? 3 : 2));
    constexpr int NPW = (MIXED || DIM == 2) ? 1 : 2;
    constexpr uint32_t RBYTES = MIXED ? 32u : 64u;
    constexpr uint32_t WBYTES = sizeof(typename V::wpos_t);
    constexpr int STRIDE = G + 1;                     // parts per record in LDS
    constexpr int RS = 64 * STRIDE;
    __shared__ part_t xch[kMaxBlock / 64][RS];
    part_t *X = xch[threadIdx.x >> 6];
    const int lane = lane_id();
    const int p = lane & (G - 1);
    const int gb = lane & ~(G - 1);
    const char *base = reinterpret_cast<const char *>(rec);
    const uint32_t woff = (uint32_t)sc.wrec_off;
    const uint32_t p16 = (uint32_t)p * 16u;
    const real cs = MIXED ? (real)1 : (real)sc.cs;
    int mmax = m;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mmax = max(mmax, __shfl_xor(mmax, off, 64));
    constexpr int QN = R == 6 ? 3 : (R > 4 ? R / 4 : 1);   // quads of entries per iteration
    for (int q0 = 0; q0 < mmax; q0 += 4 * QN) {
        unsigned eq[4 * QN];
#pragma unroll
        for (int g = 0; g < QN; ++g) {
            uint4 quad = make_uint4(0u, 0u, 0u, 0u);
            if (q0 + 4 * g < m) quad = nlist[(int64_t)((q0 >> 2) + g) * n + k];
            eq[4 * g] = quad.x;
            eq[4 * g + 1] = quad.y;
            eq[4 * g + 2] = quad.z;
            eq[4 * g + 3] = quad.w;
        }
#pragma unroll
        for (int h0 = 0; h0 < 4 * QN; h0 += R) {
            part_t raw[R][G];
#pragma unroll
            for (int h = 0; h < R; ++h) {
                const bool valid = q0 + h0 + h < m;
                const unsigned e = eq[h0 + h];
                const uint32_t sl = e & kSlotMask;
                uint32_t off = (e & kWallBit) ? woff + sl * WBYTES : sl * RBYTES;
                off = valid ? off : 0u;
                uint32_t og[G];
                og[0] = group_bcast<G, 0>((int)off);
                og[1] = group_bcast<G, 1>((int)off);
                if constexpr (G == 4) {
                    og[2] = group_bcast<G, 2>((int)off);
                    og[3] = group_bcast<G, 3>((int)off);
                }
#pragma unroll
                for (int i = 0; i < G; ++i) raw[h][i] = *reinterpret_cast<const part_t *>(base + (og[i] + p16));
            }
#pragma unroll
            for (int h = 0; h < R; ++h) {
#pragma unroll
                for (int i = 0; i < G; ++i) {
                    in_registers(raw[h][i]);
                    X[(gb + i) * STRIDE + p] = raw[h][i];
                }
                // LDS operations of one wave execute in order: the reads below
                // see the stores above, and the next stores come after them;
                // the barriers only keep the compiler from reordering them
                __builtin_amdgcn_wave_barrier();
                if (q0 + h0 + h < m) {
                    const unsigned e = eq[h0 + h];
                    const bool wl = (e & kWallBit) != 0u;
                    const part_t *mine = X + lane * STRIDE;
                    v4 A, B;
                    if constexpr (MIXED) {
                        A = mine[0];
                        B = NP > 1 && !wl ? mine[1] : fvec4{};
                    } else {
                        const dvec2 p0 = mine[0];
                        const dvec2 p1 = NPW > 1 || !wl ? mine[1] : dvec2{0.0, 0.0};
                        const dvec2 p2 = NP > 2 && !wl ? mine[2] : dvec2{0.0, 0.0};
                        const dvec2 p3 = NP > 3 && !wl ? mine[3] : dvec2{0.0, 0.0};
                        A.x = p0.x; A.y = p0.y; A.z = p1.x; A.w = p1.y;
                        B.x = p2.x; B.y = p2.y; B.z = p3.x; B.w = p3.y;
                    }
                    real pj[3], t[3], r[3];
                    V::pos(A, pj);
                    if constexpr (MIXED) {
                        const int ox = (int)((e >> kSlotBits) & 3u) - 1;
                        const int oy = (int)((e >> (kSlotBits + 2)) & 3u) - 1;
                        const int oz = (int)((e >> (kSlotBits + 4)) & 3u) - 1;
                        shift_target<DIM, true>(pi, ox, oy, oz, cs, t);
                    } else {
                        shift_target<DIM, false>(pi, 0, 0, 0, cs, t);
                    }
                    sub_vec<DIM>(t, pj, r);
                    const real r2 = norm2<DIM>(r);
                    if (!CHK || r2 < cut2) fn(wl, (int)(e & kSlotMask), r, r2, A, B, e);
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// density sweep
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Cell-pair list build.
//
// The lanes of a wave hold 64 sources, the targets are taken one at a time:
// a wave owns 64 consecutive targets (sorted slots) and walks them cell by
// cell.  For one cell, the sources of its 3^d stencil -- the fluid slots of
// the centre row's three cells first (they hold the targets themselves),
// then the rest in z, y row order, per row the fluid slots of its three
// cells, then their wall slots -- form one sequence of S sources held in the
// first nch = ceil(S / 64) of CH register chunks: lane l of chunk j holds
// element 64 j + l, as its FP32 position p relative to the centre of the
// target cell, scaled by -2, its |p|^2, and its list entry.  A target t
// of the cell (wave-uniform, so its position is a scalar operand) then tests a
// chunk with three FMAs and a compare, |p|^2 - 2 t.p < R^2 (1 + 1e-4) - |t|^2
// with R the build radius 2h + skin (positions within 1.5 cells of the
// centre: the rounding stays below 1e-5 R^2), and one compare against its
// own entry; the hits append to the target's list in sequence (slot) order
// through a ballot and mbcnt, into a staging area in LDS written out as
// quads when the target is done.  The loop over a cell's targets exists in
// one fully unrolled copy per chunk count (the fewest counts share one copy,
// whose surplus chunks never hit), chosen once per cell, so the chunk tests
// carry no branches.  Source loads happen once per cell, not once per target.  The list is the superset of build_list's kind (every pair
// closer than R, and a few within the margin beyond it, which the walks skip).
//
// Cells whose stencil holds more than CH * 64 sources, and targets far
// outside their cell, are marked (lcount = -1) for k_build, which follows
// with FALLBACK = true and builds only those; tiled Morton keys (stencil rows
// not contiguous) and capacities above kCpListMax use k_build alone.
// ---------------------------------------------------------------------------

// Register chunks of 64 sources.  3D: with h = 1.3 dx a stencil of cells of
// 2h spans 7 or 8 lattice planes per axis (at most 512 sources, walls
// included, while the fluid stays near its rest density); cells of 2h + skin
// reach 9 planes.
template <int DIM, bool SKIN> constexpr int cp_chunks() { return DIM == 3 ? (SKIN ? 10 : 8) : 4; }
constexpr int kCpListMax = 255;        // list capacity the cell-pair build supports
constexpr int kNSelf = 2;              // chunks that may hold a target's own entry

// Value of `v` on lane `src` (lane-varying source lane).
__device__ __forceinline__ int lane_value(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }

template <int DIM, bool MIXED, bool SKIN>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(SKIN ? 5 : 6))) void k_build_cp(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ cstart, const int *__restrict__ wstart,
    const typename Cand<DIM>::t *__restrict__ cpos, uint32_t wcpos_off,
    uint4 *__restrict__ nlist, int *__restrict__ lcount, int cap, unsigned *__restrict__ flags,
    const int *__restrict__ gate)
{
    using CT = typename Cand<DIM>::t;
    constexpr int NR = DIM == 3 ? 18 : 6;                 // (row, kind) ranges of a stencil
    if constexpr (SKIN) {
        if (*gate == 0) return;
    }
    constexpr int CH = cp_chunks<DIM, SKIN>();
    // staging: a whole stencil of hits, and room past it for the writes of
    // the lanes without a hit
    constexpr int kCpStage = CH * 64;
    static_assert(((kCpListMax + 3) & ~3) <= kCpStage + 64, "the quads of a full list stay inside the staging");
    __shared__ __align__(16) unsigned stage[kMaxBlock / 64][kCpStage + 128];
    const Chunk ch = map[blockIdx.x];
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w0 = ch.begin + wv * 64;
    const int nt = min(64, ch.end - w0);                  // targets of the wave
    if (nt <= 0) return;                                  // the whole wave
    unsigned *lst = stage[wv];
    const InstDev &I = inst[ch.inst];
    const int ncx = I.ncell[0], ncy = I.ncell[1], ncz = I.ncell[2];
    const float fcs = sc.fcs, hcs = 0.5f * sc.fcs;
    const float bhi = sc.fbcut2 * (1.0f + 1e-4f);        // the build radius^2 with its margin
    const char *cbase = reinterpret_cast<const char *>(cpos);
    const int n = sc.N;

    // the wave's targets, one per lane: cell key, position relative to the
    // centre of its cell, R^2 (1 + 1e-4) - |t|^2
    const bool tv = lane < nt;
    const int tl = w0 + (tv ? lane : 0);
    const int kl = skey[tl];
    const CT ol = cpos[tl];
    const float txl = ol.x - hcs, tyl = ol.y - hcs;
    float tzl = 0.0f;
    if constexpr (DIM == 3) tzl = ol.z - hcs;
    const float ctl = bhi - (txl * txl + tyl * tyl + tzl * tzl);
    // targets far outside their cell (clamped keys) are left to k_build
    const uint64_t farm = __builtin_amdgcn_ballot_w64(
        tv && (fabsf(txl) > 4.0f * fcs || fabsf(tyl) > 4.0f * fcs || fabsf(tzl) > 4.0f * fcs));
    // the first target of each cell: lane 0 and the lanes whose key differs
    // from the one before
    const int kup = lane_value(kl, lane > 0 ? lane - 1 : 0);
    uint64_t starts = __builtin_amdgcn_ballot_w64(tv && (lane == 0 || kl != kup));
    int lc = -1;                                          // list length of the lane's target (-1: k_build)
    int mmax = 0;                                         // the longest list of the wave

    // the cell of the lane's target (instance-local key)
    const int lkl = kl - I.cell_base;
    // lane r < NR describes range r = 2 row + kind of the stencil of cell
    // (cx, cy, cz): its first slot, length, the slots where the second and
    // third cell of the row begin, and the row's cell offsets (x of its first
    // cell, y, z; each plus one).  The loads are unconditional (a row outside
    // the grid reads the instance's first row and is emptied afterwards), so
    // that they stay in flight until the values are used.
    // Lane 0 describes the centre row's fluid range, which holds every target
    // of the cell, so that a target's own entry lies in the first kNSelf
    // chunks and only those need the test against it; lanes 1.. describe the
    // other ranges in row order.
    constexpr int RC = NR / 2 - 1;                        // range of the centre row's fluid
    const int rr = lane == 0 ? RC : (lane <= RC ? lane - 1 : lane);
    const int rrow = rr >> 1, rkind = rr & 1;
    const int rdy = (DIM == 3 ? rrow % 3 : rrow) - 1;
    const int rdz = DIM == 3 ? rrow / 3 - 1 : 0;
    const int *rst = rkind ? wstart : cstart;
    struct Ranges { int start, end, b1, b2, sh; bool ok; };
    auto ranges = [&](int lk) __attribute__((always_inline)) {
        const int cx = lk % ncx, cy = (lk / ncx) % ncy, cz = lk / (ncx * ncy);
        Ranges R;
        const int yy = cy + rdy, zz = cz + rdz;
        R.ok = lane < NR && yy >= 0 && yy < ncy && zz >= 0 && zz < ncz;
        const int xlo = cx > 0 ? cx - 1 : cx, xhi = cx < ncx - 1 ? cx + 1 : cx;
        const int rk = I.cell_base + (R.ok ? (yy + ncy * zz) * ncx : 0);
        R.start = rst[rk + xlo];
        R.end = rst[rk + xhi + 1];
        R.b1 = rst[rk + min(xlo + 1, xhi + 1)];
        R.b2 = rst[rk + min(xlo + 2, xhi + 1)];
        R.sh = (xlo - cx + 1) | ((rdy + 1) << 2) | ((rdz + 1) << 4) | (rkind << 6);
        return R;
    };

    // list output, one target behind: the quads of the last target are read
    // from the staging before the next target's tests write it (a wave's LDS
    // operations execute in order) and stored after them.  Entries of the
    // last quad past the list length are stored as the staging holds them:
    // the walks never read past it.
    int pend_t = -1, pend_mm = 0;
    auto store_pending = [&](const uint4 &o) __attribute__((always_inline)) {
        if (pend_t >= 0 && lane < ((pend_mm + 3) >> 2)) nlist[(int64_t)lane * n + pend_t] = o;
    };

    Ranges R = ranges(__builtin_amdgcn_readlane(lkl, 0));
    while (true) {
        const int a = (int)__builtin_ctzll(starts);      // the cell's first and last + 1 lanes
        starts &= starts - 1;
        const int b = starts ? (int)__builtin_ctzll(starts) : nt;
        const int rstart = R.ok ? R.start : 0, rlen = R.ok ? R.end - R.start : 0;
        const int rb1 = R.b1, rb2 = R.b2, rsh = R.sh;
        const int rend_seq = wave_inclusive_scan(rlen);  // end of range r in the sequence
        const int S = __builtin_amdgcn_readlane(rend_seq, 63);
        const int nch = (S + 63) >> 6;
        // the chunks: -2 p, |p|^2 and the entry of every source (a cell with
        // more sources than the registers hold is left to k_build)
        float qx[CH], qy[CH], qz[CH], pp[CH];
        unsigned ent[CH];
        int rc = 0;                                       // ranges ending at or before 64 j
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            qx[j] = qy[j] = qz[j] = 0.0f;
            pp[j] = 3.0e38f;                              // no hit
            ent[j] = 0u;
            if (j < nch && nch <= CH) {
                const int g = 64 * j + lane;
                while (rc < NR && __builtin_amdgcn_readlane(rend_seq, rc) <= 64 * j) ++rc;
                // the range of g: rc plus the ranges ending inside the chunk at or before g
                int r = rc;
                for (int q = rc; q < NR; ++q) {
                    const int e = __builtin_amdgcn_readlane(rend_seq, q);
                    if (e > 64 * j + 63) break;
                    r += e <= g ? 1 : 0;
                }
                const int pre = lane_value(rend_seq - rlen, r);
                const int slot = lane_value(rstart, r) + (g - pre);
                const int sh = lane_value(rsh, r);
                const int ox = (sh & 3) - 1 + (slot >= lane_value(rb1, r) ? 1 : 0) + (slot >= lane_value(rb2, r) ? 1 : 0);
                const int oy = ((sh >> 2) & 3) - 1, oz = ((sh >> 4) & 3) - 1;
                const bool wall = (sh >> 6) & 1;
                const bool valid = g < S;
                const uint32_t off = valid ? (wall ? wcpos_off : 0u) + (uint32_t)slot * (uint32_t)sizeof(CT) : 0u;
                const CT c = *reinterpret_cast<const CT *>(cbase + off);
                if (valid) {
                    // the candidate copies hold offsets from the cell's origin
                    const float sx = fmaf((float)ox - 0.5f, fcs, c.x);
                    const float sy = fmaf((float)oy - 0.5f, fcs, c.y);
                    float sz = 0.0f;
                    if constexpr (DIM == 3) sz = fmaf((float)oz - 0.5f, fcs, c.z);
                    qx[j] = -2.0f * sx;
                    qy[j] = -2.0f * sy;
                    qz[j] = -2.0f * sz;
                    pp[j] = sx * sx + sy * sy + sz * sz;
                    ent[j] = (wall ? kWallBit : 0u) | (unsigned)slot | (MIXED ? offset_bits(ox, oy, oz) : 0u);
                }
            }
        }
        // the next cell's ranges, loaded while this cell's targets are tested
        const int nb = starts ? b : a;
        R = ranges(__builtin_amdgcn_readlane(lkl, nb));
        // the targets of the cell against the first NC chunks (NC >= nch;
        // chunks past nch never hit): one unrolled copy per chunk count
        auto targets = [&](auto ncc) __attribute__((always_inline)) {
            constexpr int NC = decltype(ncc)::value;
            // the cell's targets a..b-1 without the far ones (left to k_build)
            uint64_t todo = (b - a >= 64 ? ~0ull : ((1ull << (b - a)) - 1ull)) << a;
            todo &= ~farm;
            while (todo) {
                const int l = (int)__builtin_ctzll(todo);
                todo &= todo - 1ull;
                const uint4 o = reinterpret_cast<const uint4 *>(lst)[lane];   // the pending quads
                const float ttx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(txl), l));
                const float tty = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tyl), l));
                float ttz = 0.0f;
                if constexpr (DIM == 3) ttz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tzl), l));
                const float ct = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ctl), l));
                // the target's own entry, the one source that is not a pair
                unsigned eself = (unsigned)(w0 + l) | (MIXED ? offset_bits(0, 0, 0) : 0u);
                // an opaque scalar: no induction variable per chunk
                asm volatile("" : "+s"(eself));
                unsigned *lp = lst;                       // the target's next list place
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    float d = fmaf(qx[j], ttx, pp[j]);
                    d = fmaf(qy[j], tty, d);
                    if constexpr (DIM == 3) d = fmaf(qz[j], ttz, d);
                    const bool near = d < ct, other = j >= kNSelf || ent[j] != eself;
                    const uint64_t hm = __builtin_amdgcn_ballot_w64(near) & __builtin_amdgcn_ballot_w64(other);
                    int pos = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(hm >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)hm, 0u));
                    // every lane writes: a hit at its place in the list, any
                    // other lane past the places this chunk's hits can take
                    // (later hits overwrite it, or it lies past the list)
                    asm volatile("" : "+v"(pos));
                    lp[near && other ? pos : 64 + lane] = ent[j];
                    lp += __popcll(hm);
                }
                const int m = (int)(lp - lst);
                store_pending(o);
                pend_t = w0 + l;
                pend_mm = min(m, cap);
                lc = lane == l ? m : lc;
                mmax = max(mmax, m);
            }
        };
        using std::integral_constant;
        // the cell is built here when its sources fit the chunks and its
        // centre range the chunks that test the targets' own entries
        if (nch <= CH && __builtin_amdgcn_readlane(rlen, 0) <= 64 * kNSelf) {
            if constexpr (CH >= 5) {
                if (nch <= CH - 4) targets(integral_constant<int, CH - 4>{});
                else if (nch == CH - 3) targets(integral_constant<int, CH - 3>{});
                else if (nch == CH - 2) targets(integral_constant<int, CH - 2>{});
                else if (nch == CH - 1) targets(integral_constant<int, CH - 1>{});
                else targets(integral_constant<int, CH>{});
            } else {
                if (nch <= 2) targets(integral_constant<int, 2>{});
                else if (nch == 3) targets(integral_constant<int, 3>{});
                else targets(integral_constant<int, CH>{});
            }
        }
        if (!starts) break;
    }
    store_pending(reinterpret_cast<const uint4 *>(lst)[lane]);
    if (tv) lcount[w0 + lane] = lc;
    if (mmax > cap && lane == 0) atomicOr(flags, 4u);
}

// Candidate tests and list build (a lane per target): lists of every target
// and their lengths (lcount); a list longer than cap raises
// SPH_FLAG_CAPACITY (its target searches the cells in the sweeps).  SKIN:
// with radius 2h + skin, on build steps only (*gate != 0).
template <int DIM, bool MIXED, bool SKIN, int PF, bool FALLBACK>
__global__ __launch_bounds__(kMaxBlock) void k_build(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ cstart, const int *__restrict__ wstart,
    const typename Rec<DIM, MIXED>::v4 *__restrict__ rec, const typename Rec<DIM, MIXED>::wpos_t *__restrict__ wpos,
    const typename Cand<DIM>::t *__restrict__ cpos, const typename Cand<DIM>::t *__restrict__ wcpos,
    uint4 *__restrict__ nlist, int *__restrict__ lcount, int cap, unsigned *__restrict__ flags,
    const int *__restrict__ gate)
{
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    using v4 = typename V::v4;
    if constexpr (SKIN) {
        if (*gate == 0) return;
    }
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    // after k_build_cp: only the targets it left (lcount = -1)
    if constexpr (FALLBACK) {
        if (lcount[k] != -1) return;
    }
    const InstDev &I = inst[ch.inst];
    const int lk = skey[k] - I.cell_base;
    const v4 Ai = V::loadA(rec, k);
    real pi[3];
    V::pos(Ai, pi);
    float ci[3];
    const typename Cand<DIM>::t cp = cpos[k];
    ci[0] = cp.x;
    ci[1] = cp.y;
    if constexpr (DIM == 3) ci[2] = cp.z;
    else ci[2] = 0.0f;
    const int m = build_list<DIM, MIXED, PF>(sc, I, lk, k, pi, ci, cstart, wstart, rec, wpos, cpos, wcpos,
                                             nlist, cap, sc.N);
    lcount[k] = m;
    if (m > cap) atomicOr(flags, 4u);
}

// LIST = 0: direct search.  LIST = 5: walk the list of this step's build
// (launch_build).  LIST = 3 (Verlet skin): walk the list of the last build,
// skipping the entries at 2h or beyond.  A target whose list overflowed
// searches the cells instead.
template <int DIM, bool MIXED, int LIST>
__global__ __launch_bounds__(kMaxBlock) void k_density(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ perm, const int *__restrict__ cstart,
    const int *__restrict__ wstart, typename Rec<DIM, MIXED>::v4 *__restrict__ rec,
    const typename Rec<DIM, MIXED>::wpos_t *__restrict__ wpos, double *__restrict__ rho, int *__restrict__ count,
    const double *__restrict__ dt, int use_dt, const uint4 *__restrict__ nlist, const int *__restrict__ lcount,
    int cap)
{
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    using v4 = typename V::v4;
    static_assert(LIST == 0 || LIST == 3 || LIST == 5, "density sweeps: direct search or a list walk");
    constexpr int NEED = DIM == 3 ? NEED_VEL : NEED_NONE;
    // the cooperative walk needs every lane of the wave, targets or not
    constexpr bool COOP = LIST != 0 && use_coop<DIM, MIXED>();
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    const bool act = k < ch.end;
    if (!COOP && !act) return;
    const int kk = act ? k : ch.begin;
    const int n = sc.N;
    const InstDev &I = inst[ch.inst];
    const int lk = skey[kk] - I.cell_base;
    const v4 Ai = V::loadA(rec, kk);
    const v4 Bi = load_need<DIM, MIXED, NEED>(rec, kk);
    real pi[3], vi[3];
    V::pos(Ai, pi);
    V::vel(Ai, Bi, vi);
    double qs[3] = {0.0, 0.0, 0.0};
    if constexpr (MIXED) {
        int qi[3];
        V::qpos(Ai, qi);
        exact_target<DIM>(qi, qs);
    }
    // the summation density in FP64 on both paths (see exact_r2)
    double sigma = MIXED ? 0.0 : sc.W0;
    real drho = 0;
    int cnt = 0;
    const real cut2 = walk_cut2<MIXED, true>(sc);
    auto pair = [&](bool wall, int, const real *r, real r2, const v4 &Aj, const v4 &Bj, unsigned e)
        __attribute__((always_inline)) {
        (void)wall;                        // wall records carry zero velocity
        real vj[3];
        V::vel(Aj, Bj, vj);
        real vr = (vi[0] - vj[0]) * r[0] + (vi[1] - vj[1]) * r[1];
        if constexpr (DIM == 3) vr += (vi[2] - vj[2]) * r[2];
        if constexpr (MIXED) {
            // exact pair test and kernel value on the fixed-point positions;
            // the continuity term in FP32 (lengths in units of cs)
            const double r2q = exact_r2<DIM>(qs, Aj, e);
            if (r2q < sc.qcut2) {
                double W;
                float F;
                kernel_WF_exact(r2q, sc.qinv_h, sc.kW, sc.kF, W, F);
                sigma += W;
                drho += vr * F;
                ++cnt;
            }
        } else {
            (void)e;
            (void)vr;
            density_pair<DIM, real>(r, r2, vi, vj, (real)sc.inv_h, (real)sc.kW, (real)sc.kF, sigma, drho, cnt);
        }
    };
    if constexpr (COOP && (LIST == 3 || LIST == 5)) {
        const int m = act ? lcount[k] : 0;
        walk_coop<DIM, MIXED, NEED, density_chk<MIXED, LIST>(), kCoopRoundsWalk>(sc, kk, m <= cap ? m : 0, pi, rec, nlist, n, cut2, pair);
        if (act && m > cap) for_neighbours<DIM, MIXED, NEED>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, cut2, pair);
        if (!act) return;
    } else if constexpr (LIST == 3 || LIST == 5) {
        const int m = lcount[k];
        if (m <= cap) walk_list<DIM, MIXED, skin_walk_u<DIM, MIXED>(), NEED, density_chk<MIXED, LIST>()>(sc, k, m, pi, rec, wpos, nlist, n, cut2, pair);
        else for_neighbours<DIM, MIXED, NEED>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, cut2, pair);
    } else {
        for_neighbours<DIM, MIXED, NEED>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, cut2, pair);
    }
    const int i = perm[k];
    const double sig = MIXED ? sc.W0 + sigma : sigma;
    const double dtb = use_dt ? dt[ch.inst] : 0.0;
    // mixed path: the continuity sum is in units of cs
    const double mscale = MIXED ? sc.mass * sc.cs : sc.mass;
    double rn, P;
    density_update(rho[i], sig, mscale * (double)drho, dtb, sc.mass, sc.rho0, I.c0, rn, P);
    rho[i] = rn;
    count[i] = cnt;
    typename V::v2 out;
    out.x = (real)rn;
    out.y = (real)P;
    reinterpret_cast<typename V::v2 *>(rec)[V::rhoP_slot(k)] = out;
}

template <int DIM, bool MIXED, int LIST>
static void density_dispatch(const SimConst &sc, const Dev &d, int use_dt, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    k_density<DIM, MIXED, LIST><<<d.nfchunks, d.block, 0, s>>>(
        sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start, static_cast<typename R::v4 *>(d.rec),
        static_cast<const typename R::wpos_t *>(d.wpos), d.rho, d.count, d.dt, use_dt, d.nlist, d.lcount,
        d.list_cap);
}

template <int DIM, bool MIXED, bool SKIN, int PF>
static void build_dispatch(const SimConst &sc, const Dev &d, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    using CT = typename Cand<DIM>::t;
    const auto *rec = static_cast<const typename R::v4 *>(d.rec);
    const auto *wp = static_cast<const typename R::wpos_t *>(d.wpos);
    const auto *cp = static_cast<const CT *>(d.cpos);
    const auto *wcp = static_cast<const CT *>(d.wcpos);
    const int64_t woff = static_cast<const char *>(d.wcpos) - static_cast<const char *>(d.cpos);
    const bool cell_pair = d.cell_pair && sc.key_order == 0 && d.list_cap <= kCpListMax && woff >= 0 &&
                           woff < (int64_t)UINT32_MAX;
    if (cell_pair) {
        k_build_cp<DIM, MIXED, SKIN><<<d.nfchunks, d.block, 0, s>>>(
            sc, d.fmap, d.inst, d.skey, d.cell_start, d.wall_start, cp, (uint32_t)woff, d.nlist,
            d.lcount, d.list_cap, d.flags, d.gate);
        k_build<DIM, MIXED, SKIN, PF, true><<<d.nfchunks, d.block, 0, s>>>(
            sc, d.fmap, d.inst, d.skey, d.cell_start, d.wall_start, rec, wp, cp, wcp, d.nlist, d.lcount,
            d.list_cap, d.flags, d.gate);
    } else {
        k_build<DIM, MIXED, SKIN, PF, false><<<d.nfchunks, d.block, 0, s>>>(
            sc, d.fmap, d.inst, d.skey, d.cell_start, d.wall_start, rec, wp, cp, wcp, d.nlist, d.lcount,
            d.list_cap, d.flags, d.gate);
    }
}

template <int DIM, bool MIXED>
static void build_variant(const SimConst &sc, const Dev &d, hipStream_t s)
{
    if (d.gate) {
        if (d.prefetch == 4) build_dispatch<DIM, MIXED, true, 4>(sc, d, s);
        else build_dispatch<DIM, MIXED, true, 8>(sc, d, s);
    } else {
        if (d.prefetch == 4) build_dispatch<DIM, MIXED, false, 4>(sc, d, s);
        else build_dispatch<DIM, MIXED, false, 8>(sc, d, s);
    }
}

hipError_t launch_build(const SimConst &sc, const Dev &d, int mixed, hipStream_t s)
{
    if (d.nfchunks <= 0 || d.list_cap <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) build_variant<2, true>(sc, d, s); else build_variant<2, false>(sc, d, s); }
    else { if (mixed) build_variant<3, true>(sc, d, s); else build_variant<3, false>(sc, d, s); }
    return hipGetLastError();
}

template <int DIM, bool MIXED>
static void density_variant(const SimConst &sc, const Dev &d, int use_dt, hipStream_t s)
{
    // the lists come from launch_build
    if (d.list_cap <= 0) density_dispatch<DIM, MIXED, 0>(sc, d, use_dt, s);
    else if (d.gate) density_dispatch<DIM, MIXED, 3>(sc, d, use_dt, s);
    else density_dispatch<DIM, MIXED, 5>(sc, d, use_dt, s);
}

hipError_t launch_density(const SimConst &sc, const Dev &d, int mixed, int use_dt, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) density_variant<2, true>(sc, d, use_dt, s); else density_variant<2, false>(sc, d, use_dt, s); }
    else { if (mixed) density_variant<3, true>(sc, d, use_dt, s); else density_variant<3, false>(sc, d, use_dt, s); }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// force sweep (+ half 2 and all partials when fused)
// ---------------------------------------------------------------------------

// LIST = 0: direct search.  LIST = 1: walk the list of this step's density
// sweep.  LIST = 2: the same with a Verlet skin (entries at 2h or beyond skipped).
template <int DIM, bool MIXED, bool FUSED, int LIST>
__global__ __launch_bounds__(kMaxBlock) void k_force(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ perm, const int *__restrict__ cstart,
    const int *__restrict__ wstart, const typename Rec<DIM, MIXED>::v4 *__restrict__ rec,
    const typename Rec<DIM, MIXED>::wpos_t *__restrict__ wpos, double *__restrict__ a,
    double *__restrict__ v, const double *__restrict__ x, const double *__restrict__ rho,
    const double *__restrict__ dt, double *__restrict__ partials, const uint4 *__restrict__ nlist,
    const int *__restrict__ lcount, int cap)
{
    using V = RV<DIM, MIXED>;
    using real = typename V::real;
    using v4 = typename V::v4;
    constexpr int U = force_walk_u<DIM, MIXED>();
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    const bool act = k < ch.end;
    const int n = sc.N;
    const InstDev &I = inst[ch.inst];
    const int kk = act ? k : ch.begin;
    const v4 Ai = V::loadA(rec, kk);
    const v4 Bi = V::loadB(rec, kk);
    real pi[3], vi[3];
    V::pos(Ai, pi);
    V::vel(Ai, Bi, vi);
    const real rho_i = V::rho(Bi), P_i = V::P(Bi);
    const real p_i = P_i * rho_i * rho_i;
    const real inv_rho_i2 = (real)1 / (rho_i * rho_i);
    // mixed path: lengths in units of cs (the sums are scaled back below)
    const real inv_h = MIXED ? (real)sc.uinv_h : (real)sc.inv_h;
    const real kF = MIXED ? (real)sc.fkF : (real)sc.kF;
    const real visc_a = MIXED ? (real)(sc.uvisc_scale * (float)I.c0) : (real)(sc.alpha * I.c0 * sc.h);
    const real eps_h2 = MIXED ? (real)sc.ueps_h2 : (real)sc.eps_h2;
    const real gx = MIXED ? (real)sc.ug[0] : (real)sc.g[0];
    const real gy = MIXED ? (real)sc.ug[1] : (real)sc.g[1];
    const real gz = MIXED ? (real)sc.ug[2] : (real)sc.g[2];
    const real cut2 = walk_cut2<MIXED>(sc);
    real acc[3] = {0, 0, 0}, aff[3] = {0, 0, 0};
    int cnt = 0;
    auto pair = [&](bool wall, int, const real *r, real r2, const v4 &Aj, const v4 &Bj, unsigned)
        __attribute__((always_inline)) {
        real vj[3];
        V::vel(Aj, Bj, vj);                // zero for walls
        force_pair<DIM, real>(wall, r, r2, vi, vj, rho_i, P_i, p_i, inv_rho_i2, V::rho(Bj), V::P(Bj), inv_h, kF,
                              visc_a, eps_h2, gx, gy, gz, acc, aff, cnt);
    };
    if constexpr (LIST && use_coop<DIM, MIXED>()) {
        // every lane takes part in the cooperative walk
        const int m = act ? lcount[k] : 0;
        walk_coop<DIM, MIXED, NEED_ALL, true, coop_rounds_force<DIM, MIXED>()>(sc, kk, m <= cap ? m : 0, pi, rec, nlist, n, cut2, pair);
        if (act && m > cap)
            for_neighbours<DIM, MIXED, NEED_ALL>(sc, I, skey[k] - I.cell_base, k, pi, cstart, wstart, rec, wpos, cut2, pair);
    } else if (act) {
        const int lk = skey[k] - I.cell_base;
        if constexpr (LIST) {
            const int m = lcount[k];
            if (m <= cap) walk_list<DIM, MIXED, U, NEED_ALL, true>(sc, k, m, pi, rec, wpos, nlist, n, cut2, pair);
            else for_neighbours<DIM, MIXED, NEED_ALL>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, cut2, pair);
        } else {
            for_neighbours<DIM, MIXED, NEED_ALL>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, cut2, pair);
        }
    }
    double vals[kNPart];
#pragma unroll
    for (int q = 0; q < kNPart; ++q) vals[q] = 0.0;
    if (act) {
        const int i = perm[k];
        const double mscale = MIXED ? sc.mass * sc.cs : sc.mass;
        double an[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            an[c] = sc.g[c] + mscale * (double)acc[c];
            a[(int64_t)c * n + i] = an[c];
            vals[P_FF + c] = sc.mass * (mscale * (double)aff[c]);
        }
        vals[P_PAIRS] = (double)cnt;
        if constexpr (FUSED) {
            const double dtb = dt[ch.inst];
            double vn[DIM], xi[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                vn[c] = kick(v[(int64_t)c * n + i], an[c], dtb);
                v[(int64_t)c * n + i] = vn[c];
                xi[c] = x[(int64_t)c * n + i];
            }
            state_partials<DIM>(sc, I, vn, an, xi, rho[i], vals);
        }
    }
    double *out = partials + (int64_t)ch.id * kNPart;
    if constexpr (FUSED) block_partials<0, P_BAD + 1>(vals, out);
    else block_partials<P_FF, P_PAIRS + 1>(vals, out);
}

template <int DIM, bool MIXED, bool FUSED, int LIST>
static void force_dispatch(const SimConst &sc, const Dev &d, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    k_force<DIM, MIXED, FUSED, LIST><<<d.nfchunks, d.block, 0, s>>>(
        sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start,
        static_cast<const typename R::v4 *>(d.rec), static_cast<const typename R::wpos_t *>(d.wpos), d.a, d.v,
        d.x, d.rho, d.dt, d.partials, d.nlist, d.lcount, d.list_cap);
}

template <int DIM, bool MIXED>
static void force_variant(const SimConst &sc, const Dev &d, int fused, int list, hipStream_t s)
{
    if (list && d.gate) {
        if (fused) force_dispatch<DIM, MIXED, true, 2>(sc, d, s);
        else force_dispatch<DIM, MIXED, false, 2>(sc, d, s);
    } else if (fused) { if (list) force_dispatch<DIM, MIXED, true, 1>(sc, d, s); else force_dispatch<DIM, MIXED, true, 0>(sc, d, s); }
    else { if (list) force_dispatch<DIM, MIXED, false, 1>(sc, d, s); else force_dispatch<DIM, MIXED, false, 0>(sc, d, s); }
}

hipError_t launch_force(const SimConst &sc, const Dev &d, int mixed, int fused, int list, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) force_variant<2, true>(sc, d, fused, list, s); else force_variant<2, false>(sc, d, fused, list, s); }
    else { if (mixed) force_variant<3, true>(sc, d, fused, list, s); else force_variant<3, false>(sc, d, fused, list, s); }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dual-criteria scheme: acoustic sub-steps
//
// An advection step rebuilds the cell table, packs the sweep records at the
// current positions and resets the density by summation (the density sweep
// above with dt = 0); the records' positions then stay frozen for the
// acoustic sub-steps, which relax pressure and density against that
// configuration with interface states from the linearised Riemann problem
// along each pair (the published scheme of the library behind the paper:
// Zhang, Hu & Adams 2017; Zhang, Rezavand & Hu 2021).  A sub-step is
//   first half    rho += dt/2 Drho; p = max(0, c0^2 (rho - rho0)); x += dt/2 v
//   pressure      a_i = g - 2 m sum_j P*_ij / (rho_i rho_j) F_ij r_ij; v += dt a
//   second half   x += dt/2 v
//   density       Drho_i = 2 rho_i m sum_j (v_i - v*_ij).F_ij r_ij / rho_j;
//                 rho += dt/2 Drho
// with, along e = r_ij / |r_ij|, U_L = -v_i.e, U_R = -v_j.e, Z = rho c0,
// beta = min(eta max(U_L - U_R, 0) / c0, 1),
// P* = (Z_L p_R + Z_R p_L + Z_L Z_R beta (U_L - U_R)) / (Z_L + Z_R),
// v_i - v* = Z_R (v_i - v_j) / (Z_L + Z_R) + (p_L - p_R) / (Z_L + Z_R) e,
// and a wall j mirroring the target (rho_j = rho_i, v_j = 0,
// p_j = max(0, p_i + rho_i g.(x_j - x_i))).  The sweeps read velocities,
// densities and pressures from the records and write the FP64 state, so every
// target sees the values of the start of the sweep; the per-particle kernels
// in between refresh the records.  FP64 only.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double half_update(double y, double rate, double dt)
{
#pragma clang fp contract(off)
    return y + 0.5 * dt * rate;
}

__device__ __forceinline__ double full_update(double y, double rate, double dt)
{
#pragma clang fp contract(off)
    return y + dt * rate;
}

// First half (sorted order): density and pressure of the sub-step, half drift.
template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_dual_first(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ perm, double *__restrict__ x, const double *__restrict__ v,
    double *__restrict__ rho, const double *__restrict__ drho, const int *__restrict__ nsub,
    const double *__restrict__ dtsub, int sub, typename Rec<DIM, false>::v4 *__restrict__ rec)
{
    using V = RV<DIM, false>;
    const Chunk ch = map[blockIdx.x];
    if (sub >= nsub[ch.inst]) return;
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    const int n = sc.N;
    const InstDev &I = inst[ch.inst];
    const double dt = dtsub[ch.inst];
    const int i = perm[k];
    const double r = half_update(rho[i], drho[i], dt);
    double p = I.c0 * I.c0 * (r - sc.rho0);
    if (p < 0.0) p = 0.0;
    rho[i] = r;
#pragma unroll
    for (int c = 0; c < DIM; ++c) x[(int64_t)c * n + i] = half_update(x[(int64_t)c * n + i], v[(int64_t)c * n + i], dt);
    // (rho, p) go into the record with the whole 32-byte half around them (3D:
    // the velocities as held; 2D: padding), so no sector is written in part
    typename V::v4 B{};
    if constexpr (DIM == 3) {
        B = rec[2 * (int64_t)k + 1];
        B.z = r;
        B.w = p;
    } else {
        B.x = r;
        B.y = p;
    }
    rec[2 * (int64_t)k + 1] = B;
}

// Second half (sorted order): half drift with the new velocity, and the new
// velocity into the records.
template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_dual_second(
    SimConst sc, const Chunk *__restrict__ map, const int *__restrict__ perm, double *__restrict__ x,
    const double *__restrict__ v, const int *__restrict__ nsub, const double *__restrict__ dtsub, int sub,
    typename Rec<DIM, false>::v4 *__restrict__ rec)
{
    const Chunk ch = map[blockIdx.x];
    if (sub >= nsub[ch.inst]) return;
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    const int n = sc.N;
    const double dt = dtsub[ch.inst];
    const int i = perm[k];
    double vi[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        vi[c] = v[(int64_t)c * n + i];
        x[(int64_t)c * n + i] = half_update(x[(int64_t)c * n + i], vi[c], dt);
    }
    // the velocities go into the record with the whole 32-byte halves around
    // them (positions, (rho, p) as held), so no sector is written in part
    typename Rec<DIM, false>::v4 A = rec[2 * (int64_t)k];
    if constexpr (DIM == 3) {
        typename Rec<DIM, false>::v4 B = rec[2 * (int64_t)k + 1];
        A.w = vi[0];
        B.x = vi[1];
        B.y = vi[2];
        rec[2 * (int64_t)k + 1] = B;
    } else {
        A.z = vi[0];
        A.w = vi[1];
    }
    rec[2 * (int64_t)k] = A;
}

// Pair state shared by both sweeps.
template <int DIM>
struct DualPair {
    double e[3], ul, ur, rho_j, p_j, vj[3];
};

template <int DIM>
__device__ __forceinline__ void dual_pair(const SimConst &sc, bool wall, const double *r, double r2,
                                          const double *vi, double rho_i, double p_i,
                                          const typename RV<DIM, false>::v4 &Aj,
                                          const typename RV<DIM, false>::v4 &Bj, DualPair<DIM> &q)
{
    using V = RV<DIM, false>;
    V::vel(Aj, Bj, q.vj);                  // zero for walls
    double gr = sc.g[0] * r[0] + sc.g[1] * r[1];
    if constexpr (DIM == 3) gr += sc.g[2] * r[2];
    double p_m = p_i - rho_i * gr;         // wall mirror: p_i + rho_i g.(x_j - x_i)
    p_m = p_m < 0.0 ? 0.0 : p_m;
    q.rho_j = wall ? rho_i : V::rho(Bj);
    q.p_j = wall ? p_m : V::P(Bj);
    const double rr = root(r2);
    const double inv = rr > 0.0 ? recip(rr) : 0.0;
    q.ul = 0.0;
    q.ur = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        q.e[c] = r[c] * inv;
        q.ul -= vi[c] * q.e[c];
        q.ur -= q.vj[c] * q.e[c];
    }
}

// Pressure relaxation (sorted order): a and v of the FP64 state; the
// fluid-fluid force and pair counts go to the per-chunk partials.
template <int DIM, int LIST>
__global__ __launch_bounds__(kMaxBlock) void k_dual_pressure(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ perm, const int *__restrict__ cstart,
    const int *__restrict__ wstart, const typename Rec<DIM, false>::v4 *__restrict__ rec,
    const typename Rec<DIM, false>::wpos_t *__restrict__ wpos, double *__restrict__ a,
    double *__restrict__ v, const int *__restrict__ nsub, const double *__restrict__ dtsub, int sub,
    double *__restrict__ partials, const uint4 *__restrict__ nlist, const int *__restrict__ lcount, int cap)
{
    using V = RV<DIM, false>;
    using v4 = typename V::v4;
    const Chunk ch = map[blockIdx.x];
    if (sub >= nsub[ch.inst]) return;      // uniform over the block
    const int k = ch.begin + threadIdx.x;
    const bool act = k < ch.end;
    const int n = sc.N;
    const InstDev &I = inst[ch.inst];
    const int kk = act ? k : ch.begin;
    const v4 Ai = V::loadA(rec, kk);
    const v4 Bi = V::loadB(rec, kk);
    double pi[3], vi[3];
    V::pos(Ai, pi);
    V::vel(Ai, Bi, vi);
    const double rho_i = V::rho(Bi), p_i = V::P(Bi);
    const double c0 = I.c0, inv_c0 = 1.0 / c0;
    double acc[3] = {0, 0, 0}, aff[3] = {0, 0, 0};
    int cnt = 0;
    auto pair = [&](bool wall, int, const double *r, double r2, const v4 &Aj, const v4 &Bj, unsigned)
        __attribute__((always_inline)) {
        DualPair<DIM> q;
        dual_pair<DIM>(sc, wall, r, r2, vi, rho_i, p_i, Aj, Bj, q);
        const double zl = rho_i * c0, zr = q.rho_j * c0;
        const double du = q.ul - q.ur;
        double beta = sc.eta * (du > 0.0 ? du : 0.0) * inv_c0;
        beta = beta > 1.0 ? 1.0 : beta;
        const double ps = (zl * q.p_j + zr * p_i + zl * zr * beta * du) * recip(zl + zr);
        double F;
        kernel_F(r2, sc.inv_h, sc.kF, F);
        const double coef = 2.0 * ps * recip(rho_i * q.rho_j) * F;
        const double coef_ff = wall ? 0.0 : coef;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            acc[c] -= coef * r[c];
            aff[c] -= coef_ff * r[c];
        }
        ++cnt;
    };
    if constexpr (LIST && kCoopWalk) {
        // every lane takes part in the cooperative walk
        const int m = act ? lcount[k] : 0;
        walk_coop<DIM, false, NEED_ALL, true, kCoopRoundsDual>(sc, kk, m <= cap ? m : 0, pi, rec, nlist, n, sc.cut2, pair);
        if (act && m > cap)
            for_neighbours<DIM, false, NEED_ALL>(sc, I, skey[k] - I.cell_base, k, pi, cstart, wstart, rec, wpos, sc.cut2, pair);
    } else if (act) {
        const int lk = skey[k] - I.cell_base;
        if constexpr (LIST) {
            const int m = lcount[k];
            if (m <= cap) walk_list<DIM, false, kDualWalkU, NEED_ALL, true>(sc, k, m, pi, rec, wpos, nlist, n, sc.cut2, pair);
            else for_neighbours<DIM, false, NEED_ALL>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, sc.cut2, pair);
        } else {
            for_neighbours<DIM, false, NEED_ALL>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, sc.cut2, pair);
        }
    }
    double vals[kNPart];
#pragma unroll
    for (int q = 0; q < kNPart; ++q) vals[q] = 0.0;
    if (act) {
        const int i = perm[k];
        const double dt = dtsub[ch.inst];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const double an = sc.g[c] + sc.mass * acc[c];
            a[(int64_t)c * n + i] = an;
            v[(int64_t)c * n + i] = full_update(v[(int64_t)c * n + i], an, dt);
            vals[P_FF + c] = sc.mass * (sc.mass * aff[c]);
        }
        vals[P_PAIRS] = (double)cnt;
    }
    block_partials<P_FF, P_PAIRS + 1>(vals, partials + (int64_t)ch.id * kNPart);
}

// Density relaxation (sorted order): Drho and rho of the FP64 state.
template <int DIM, int LIST>
__global__ __launch_bounds__(kMaxBlock) void k_dual_density(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ perm, const int *__restrict__ cstart,
    const int *__restrict__ wstart, const typename Rec<DIM, false>::v4 *__restrict__ rec,
    const typename Rec<DIM, false>::wpos_t *__restrict__ wpos, double *__restrict__ rho,
    double *__restrict__ drho, const int *__restrict__ nsub, const double *__restrict__ dtsub, int sub,
    const uint4 *__restrict__ nlist, const int *__restrict__ lcount, int cap)
{
    using V = RV<DIM, false>;
    using v4 = typename V::v4;
    const Chunk ch = map[blockIdx.x];
    if (sub >= nsub[ch.inst]) return;
    const int k = ch.begin + threadIdx.x;
    const bool act = k < ch.end;
    if (!(LIST && kCoopWalk) && !act) return;
    const int kk = act ? k : ch.begin;
    const int n = sc.N;
    const InstDev &I = inst[ch.inst];
    const v4 Ai = V::loadA(rec, kk);
    const v4 Bi = V::loadB(rec, kk);
    double pi[3], vi[3];
    V::pos(Ai, pi);
    V::vel(Ai, Bi, vi);
    const double rho_i = V::rho(Bi), p_i = V::P(Bi);
    const double c0 = I.c0;
    double sum = 0.0;
    auto pair = [&](bool wall, int, const double *r, double r2, const v4 &Aj, const v4 &Bj, unsigned)
        __attribute__((always_inline)) {
        DualPair<DIM> q;
        dual_pair<DIM>(sc, wall, r, r2, vi, rho_i, p_i, Aj, Bj, q);
        const double zl = rho_i * c0, zr = q.rho_j * c0, zs = zl + zr;
        const double izs = recip(zs);
        double dot = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const double dv = zr * (vi[c] - q.vj[c]) * izs + (p_i - q.p_j) * izs * q.e[c];
            dot += dv * r[c];
        }
        double F;
        kernel_F(r2, sc.inv_h, sc.kF, F);
        sum += dot * F * recip(q.rho_j);
    };
    const int lk = skey[kk] - I.cell_base;
    if constexpr (LIST && kCoopWalk) {
        const int m = act ? lcount[k] : 0;
        walk_coop<DIM, false, NEED_ALL, true, kCoopRoundsDual>(sc, kk, m <= cap ? m : 0, pi, rec, nlist, n, sc.cut2, pair);
        if (act && m > cap) for_neighbours<DIM, false, NEED_ALL>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, sc.cut2, pair);
        if (!act) return;
    } else if constexpr (LIST) {
        const int m = lcount[k];
        if (m <= cap) walk_list<DIM, false, kDualWalkU, NEED_ALL, true>(sc, k, m, pi, rec, wpos, nlist, n, sc.cut2, pair);
        else for_neighbours<DIM, false, NEED_ALL>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, sc.cut2, pair);
    } else {
        for_neighbours<DIM, false, NEED_ALL>(sc, I, lk, k, pi, cstart, wstart, rec, wpos, sc.cut2, pair);
    }
    const int i = perm[k];
    const double d = 2.0 * rho_i * (sc.mass * sum);
    drho[i] = d;
    rho[i] = half_update(rho[i], d, dtsub[ch.inst]);
}

template <int DIM>
static void dual_dispatch(const SimConst &sc, const Dev &d, int sub, int list, hipStream_t s, int part)
{
    // LIST = 2: lists built with a skin (entries at 2h or beyond skipped)
    using R = Rec<DIM, false>;
    auto *rec = static_cast<typename R::v4 *>(d.rec);
    auto *wpos = static_cast<const typename R::wpos_t *>(d.wpos);
    switch (part) {
    case 0:
        k_dual_first<DIM><<<d.nfchunks, d.block, 0, s>>>(sc, d.fmap, d.inst, d.perm, d.x, d.v, d.rho, d.drho,
                                                         d.nsub, d.dtsub, sub, rec);
        break;
    case 1:
        if (list && d.gate)
            k_dual_pressure<DIM, 2><<<d.nfchunks, d.block, 0, s>>>(
                sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start, rec, wpos, d.a, d.v, d.nsub,
                d.dtsub, sub, d.partials, d.nlist, d.lcount, d.list_cap);
        else if (list)
            k_dual_pressure<DIM, 1><<<d.nfchunks, d.block, 0, s>>>(
                sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start, rec, wpos, d.a, d.v, d.nsub,
                d.dtsub, sub, d.partials, d.nlist, d.lcount, d.list_cap);
        else
            k_dual_pressure<DIM, 0><<<d.nfchunks, d.block, 0, s>>>(
                sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start, rec, wpos, d.a, d.v, d.nsub,
                d.dtsub, sub, d.partials, d.nlist, d.lcount, d.list_cap);
        break;
    case 2:
        k_dual_second<DIM><<<d.nfchunks, d.block, 0, s>>>(sc, d.fmap, d.perm, d.x, d.v, d.nsub, d.dtsub, sub, rec);
        break;
    default:
        if (list && d.gate)
            k_dual_density<DIM, 2><<<d.nfchunks, d.block, 0, s>>>(
                sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start, rec, wpos, d.rho, d.drho, d.nsub,
                d.dtsub, sub, d.nlist, d.lcount, d.list_cap);
        else if (list)
            k_dual_density<DIM, 1><<<d.nfchunks, d.block, 0, s>>>(
                sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start, rec, wpos, d.rho, d.drho, d.nsub,
                d.dtsub, sub, d.nlist, d.lcount, d.list_cap);
        else
            k_dual_density<DIM, 0><<<d.nfchunks, d.block, 0, s>>>(
                sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start, rec, wpos, d.rho, d.drho, d.nsub,
                d.dtsub, sub, d.nlist, d.lcount, d.list_cap);
        break;
    }
}

hipError_t launch_dual_substep(const SimConst &sc, const Dev &d, int sub, int list, hipStream_t s, int part)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) dual_dispatch<2>(sc, d, sub, list, s, part);
    else dual_dispatch<3>(sc, d, sub, list, s, part);
    return hipGetLastError();
}

}  // namespace sphx
