// The DSMC flow loop around the collision step (section "Results and
// Discussion": the Couette channel between diffuse walls and the lid-driven
// cavity): free flight with wall events and the cell index, the gather of
// particle arrays into cell order, per-cell moment sampling and the
// macroscopic fields.  The paper gives no formulas for this part; the
// standard method is used (Bird 1994): ballistic motion, periodic / specular
// / diffuse sides, the diffuse re-emission drawn from the wall Maxwellian
// (normal component from the flux-weighted half-range Maxwellian, tangential
// components Maxwellian about the wall velocity).  The move and the field
// formulas run in FP64 whatever the storage type, without contraction, so
// they reproduce the reference arithmetic operation by operation.
#include <math.h>

#include "common.hpp"

namespace dsmc {

constexpr uint32_t SLOT_WALL0 = 6, SLOT_WALL1 = 7;
constexpr int MAX_WALL_EVENTS = 8;
constexpr double BOLTZMANN = 1.380649e-23;

struct DomainDev {
    int32_t nx, ny;
    double Lx, Ly, cx, cy;      // cx = nx / Lx, cy = ny / Ly
    int32_t kind[4];
    double sw[4];               // sqrt(k T_w / m)
    double uw0[4], uw1[4], uw2[4];   // wall velocity components per side
};

// Entry `side` of a per-side array of the by-value domain, by selects (a
// dynamic index into a kernel argument would go through scratch memory).
template <typename V>
__device__ __forceinline__ V side_of(const V (&a)[4], int side)
{
    return side == 0 ? a[0] : side == 1 ? a[1] : side == 2 ? a[2] : a[3];
}

// Diffuse re-emission at `side` for wall event h of the particle in slot s:
// Philox(s, h, step, slot 6) -> U1, U2 and (.., slot 7) -> U3.
__device__ __forceinline__ void wall_velocity(const DomainDev& D, int side, const dsmc_rng& rng,
                                              uint32_t s, uint32_t h, double& ux, double& uy,
                                              double& uz)
{
    const U4 r0 = draw(rng, s, h, SLOT_WALL0);
    const U4 r1 = draw(rng, s, h, SLOT_WALL1);
    const double U1 = unif53(r0.a, r0.b), U2 = unif53(r0.c, r0.d), U3 = unif53(r1.a, r1.b);
    const double sw = side_of(D.sw, side);
    const double vn = sw * sqrt(-2.0 * log(1.0 - U1));
    double n1, n2;
    box_muller(U2, U3, n1, n2);
    const double w0 = side_of(D.uw0, side), w1 = side_of(D.uw1, side), w2 = side_of(D.uw2, side);
    if (side < 2) {
        ux = side == 0 ? vn : -vn;
        uy = w1 + sw * n1;
        uz = w2 + sw * n2;
    } else {
        uy = side == 2 ? vn : -vn;
        ux = w0 + sw * n1;
        uz = w2 + sw * n2;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_move(int32_t n, V3<T> pos, V3<T> v, DomainDev D, double dt, dsmc_rng rng,
       int32_t* __restrict__ cell_of, dsmc_status* st)
{
    int limit = 0, events = 0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = (uint32_t)p;
        double x = pos.x[p], y = pos.y[p], ux = v.x[p], uy = v.y[p], uz = v.z[p];
        double t = dt;
        int h = 0;
        for (;;) {
            double tx = INFINITY, ty = INFINITY;
            if (ux > 0.0) tx = (D.Lx - x) / ux;
            else if (ux < 0.0) tx = -x / ux;
            if (uy > 0.0) ty = (D.Ly - y) / uy;
            else if (uy < 0.0) ty = -y / uy;
            if (tx >= t && ty >= t) {
                x = x + ux * t;
                y = y + uy * t;
                break;
            }
            if (h == MAX_WALL_EVENTS) {
                ++limit;
                x = x + ux * t;
                y = y + uy * t;
                break;
            }
            int side;
            double th;
            if (tx <= ty) {
                side = ux > 0.0 ? 1 : 0;
                th = tx > 0.0 ? tx : 0.0;
                y = y + uy * th;
                x = side == 1 ? D.Lx : 0.0;
            } else {
                side = uy > 0.0 ? 3 : 2;
                th = ty > 0.0 ? ty : 0.0;
                x = x + ux * th;
                y = side == 3 ? D.Ly : 0.0;
            }
            t = t - th;
            const int kind = side_of(D.kind, side);
            if (kind == DSMC_WALL_PERIODIC) {
                if (side == 0) x = D.Lx;
                else if (side == 1) x = 0.0;
                else if (side == 2) y = D.Ly;
                else y = 0.0;
            } else if (kind == DSMC_WALL_SPECULAR) {
                if (side < 2) ux = -ux; else uy = -uy;
            } else {
                wall_velocity(D, side, rng, s, (uint32_t)h, ux, uy, uz);
            }
            ++h;
            ++events;
        }
        if (x < 0.0) x = 0.0;
        if (x > D.Lx) x = D.Lx;
        if (y < 0.0) y = 0.0;
        if (y > D.Ly) y = D.Ly;
        // stored positions stay inside the box in the storage type too
        T xs = (T)x, ys = (T)y;
        if constexpr (sizeof(T) == 4) {
            if ((double)xs > D.Lx) xs = nextafterf(xs, 0.0f);
            if ((double)ys > D.Ly) ys = nextafterf(ys, 0.0f);
        }
        pos.x[p] = xs;
        pos.y[p] = ys;
        v.x[p] = (T)ux;
        v.y[p] = (T)uy;
        v.z[p] = (T)uz;
        // cell of the stored position
        int32_t ix = (int32_t)((double)xs * D.cx);
        int32_t iy = (int32_t)((double)ys * D.cy);
        ix = ix < 0 ? 0 : (ix >= D.nx ? D.nx - 1 : ix);
        iy = iy < 0 ? 0 : (iy >= D.ny ? D.ny - 1 : iy);
        cell_of[p] = iy * D.nx + ix;
    }
    if (st) {
        const int wl = wave_sum_i(limit), we = wave_sum_i(events);
        if ((threadIdx.x & 63) == 0) {
            if (we) atomicAdd(reinterpret_cast<unsigned long long*>(&st->wall_events),
                              (unsigned long long)we);
            if (wl) {
                atomicAdd(&st->wall_limit, wl);
                atomicOr(&st->flags, (uint32_t)DSMC_ST_WALL_LIMIT);
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_gather(int32_t n, const int32_t* __restrict__ perm, const T* __restrict__ a,
         const T* __restrict__ b, const T* __restrict__ c, T* __restrict__ oa,
         T* __restrict__ ob, T* __restrict__ oc)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = perm[s];
        if (a) oa[s] = a[q];
        if (b) ob[s] = b[q];
        if (c) oc[s] = c[q];
    }
}

// One wave per cell: the 13 raw sums (count, v_i, v_i v_j, |v|^2 v_i), lanes
// strided over the cell's slots, fixed butterfly, added to acc.
constexpr int SAMPLE_SUMS = 13;

template <typename T>
__global__ void __launch_bounds__(256)
k_sample(const int32_t* __restrict__ cell_start, int32_t n_cells, V3<const T> v, double* acc)
{
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    for (int32_t k = blockIdx.x * wpb + (threadIdx.x >> 6); k < n_cells; k += gridDim.x * wpb) {
        const int32_t s0 = cell_start[k], s1 = cell_start[k + 1];
        double m[SAMPLE_SUMS] = {};
        for (int32_t s = s0 + lane; s < s1; s += 64) {
            const double x = v.x[s], y = v.y[s], z = v.z[s];
            const double e = x * x + y * y + z * z;
            m[0] += 1.0;
            m[1] += x; m[2] += y; m[3] += z;
            m[4] += x * x; m[5] += y * y; m[6] += z * z;
            m[7] += x * y; m[8] += x * z; m[9] += y * z;
            m[10] += e * x; m[11] += e * y; m[12] += e * z;
        }
#pragma unroll
        for (int q = 0; q < SAMPLE_SUMS; ++q) m[q] = wave_sum(m[q]);
        if (lane < SAMPLE_SUMS) {
            double mine = m[0];
#pragma unroll
            for (int q = 1; q < SAMPLE_SUMS; ++q)
                if (lane == q) mine = m[q];
            acc[(size_t)SAMPLE_SUMS * k + lane] += mine;
        }
    }
}

// Fields per cell from the sums: (n, ux, uy, uz, T, tau_xy, qx, qy, qz).
__global__ void __launch_bounds__(256)
k_fields(int32_t n_cells, const double* __restrict__ acc, double n_samples, double mass,
         double fnum_per_volume, double* __restrict__ out)
{
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_cells;
         k += gridDim.x * blockDim.x) {
        const double* a = acc + (size_t)SAMPLE_SUMS * k;
        double* f = out + 9 * (size_t)k;
        const double N = a[0];
        if (!(N > 0.0)) {
            for (int q = 0; q < 9; ++q) f[q] = 0.0;
            continue;
        }
        const double u0 = a[1] / N, u1 = a[2] / N, u2 = a[3] / N;
        const double xx = a[4] / N, yy = a[5] / N, zz = a[6] / N;
        const double xy = a[7] / N, xz = a[8] / N, yz = a[9] / N;
        const double e2 = xx + yy + zz;
        const double uu = u0 * u0 + u1 * u1 + u2 * u2;
        const double cc = e2 - uu;
        const double dens = N / n_samples * fnum_per_volume;
        const double rho = dens * mass;
        // <|c|^2 c_i> = <|v|^2 v_i> - u_i <|v|^2> - 2 u_j <v_j v_i> + 2 |u|^2 u_i
        const double e30 = a[10] / N, e31 = a[11] / N, e32 = a[12] / N;
        const double c30 = e30 - u0 * e2 - 2.0 * (u0 * xx + u1 * xy + u2 * xz) + 2.0 * uu * u0;
        const double c31 = e31 - u1 * e2 - 2.0 * (u0 * xy + u1 * yy + u2 * yz) + 2.0 * uu * u1;
        const double c32 = e32 - u2 * e2 - 2.0 * (u0 * xz + u1 * yz + u2 * zz) + 2.0 * uu * u2;
        f[0] = dens;
        f[1] = u0; f[2] = u1; f[3] = u2;
        f[4] = mass * cc / (3.0 * BOLTZMANN);
        f[5] = -rho * (xy - u0 * u1);
        f[6] = 0.5 * rho * c30;
        f[7] = 0.5 * rho * c31;
        f[8] = 0.5 * rho * c32;
    }
}

static int grid_for(int64_t items, int threads)
{
    const int pb = persistent_blocks(threads);
    int64_t b = (items + threads - 1) / threads;
    if (b < 1) b = 1;
    return (int)(b > pb ? pb : b);
}

static int check_domain(const dsmc_domain* dom, DomainDev* D)
{
    if (!dom) return arg_error("dsmc_move: null domain");
    if (dom->nx < 1 || dom->ny < 1 || !(dom->Lx > 0) || !(dom->Ly > 0) || !(dom->m > 0))
        return arg_error("dsmc_move: bad domain (nx=%d ny=%d)", dom->nx, dom->ny);
    D->nx = dom->nx; D->ny = dom->ny; D->Lx = dom->Lx; D->Ly = dom->Ly;
    D->cx = (double)dom->nx / dom->Lx;
    D->cy = (double)dom->ny / dom->Ly;
    for (int q = 0; q < 4; ++q) {
        const int k = dom->kind[q];
        if (k != DSMC_WALL_PERIODIC && k != DSMC_WALL_SPECULAR && k != DSMC_WALL_DIFFUSE)
            return arg_error("dsmc_move: side %d kind %d", q, k);
        if (k == DSMC_WALL_DIFFUSE && !(dom->T_w[q] > 0))
            return arg_error("dsmc_move: side %d wall temperature %g", q, dom->T_w[q]);
        D->kind[q] = k;
        D->sw[q] = k == DSMC_WALL_DIFFUSE ? sqrt(BOLTZMANN * dom->T_w[q] / dom->m) : 0.0;
        D->uw0[q] = dom->u_w[q][0];
        D->uw1[q] = dom->u_w[q][1];
        D->uw2[q] = dom->u_w[q][2];
    }
    if ((dom->kind[0] == DSMC_WALL_PERIODIC) != (dom->kind[1] == DSMC_WALL_PERIODIC) ||
        (dom->kind[2] == DSMC_WALL_PERIODIC) != (dom->kind[3] == DSMC_WALL_PERIODIC))
        return arg_error("dsmc_move: a periodic side needs a periodic opposite side");
    if ((int64_t)dom->nx * dom->ny >= INT32_MAX)
        return arg_error("dsmc_move: too many cells");
    return DSMC_OK;
}

}  // namespace dsmc

using namespace dsmc;

extern "C" int dsmc_move(int32_t n, int32_t dtype, dsmc_vec3 pos, dsmc_vec3 v,
                         const dsmc_domain* dom, double dt, dsmc_rng rng, int32_t* cell_of,
                         dsmc_status* st, dsmc_stream_t stream)
{
    DomainDev D;
    int rc = check_domain(dom, &D);
    if (rc) return rc;
    if (n < 0) return arg_error("dsmc_move: n=%d", n);
    if (!(dt >= 0)) return arg_error("dsmc_move: dt=%g", dt);
    if (n == 0) return DSMC_OK;
    if (!pos.x || !pos.y || !v.x || !v.y || !v.z || !cell_of)
        return arg_error("dsmc_move: null pointer");
    hipStream_t s = as_stream(stream);
    const int blocks = grid_for(n, 256);
    if (dtype == DSMC_F64)
        k_move<double><<<blocks, 256, 0, s>>>(n, v3<double>(pos), v3<double>(v), D, dt, rng,
                                               cell_of, st);
    else if (dtype == DSMC_F32)
        k_move<float><<<blocks, 256, 0, s>>>(n, v3<float>(pos), v3<float>(v), D, dt, rng,
                                              cell_of, st);
    else
        return arg_error("dsmc_move: dtype %d", dtype);
    DSMC_LAUNCH_CHECK("move");
    return DSMC_OK;
}

extern "C" int dsmc_gather(int32_t n, int32_t dtype, const int32_t* perm, dsmc_vec3 in,
                           dsmc_vec3 out, dsmc_stream_t stream)
{
    if (n < 0) return arg_error("dsmc_gather: n=%d", n);
    if (n == 0) return DSMC_OK;
    if (!perm) return arg_error("dsmc_gather: null perm");
    if ((!in.x) != (!out.x) || (!in.y) != (!out.y) || (!in.z) != (!out.z))
        return arg_error("dsmc_gather: in and out must name the same components");
    if ((in.x && in.x == out.x) || (in.y && in.y == out.y) || (in.z && in.z == out.z))
        return arg_error("dsmc_gather: in and out must be distinct buffers");
    hipStream_t s = as_stream(stream);
    const int blocks = grid_for(n, 256);
    if (dtype == DSMC_F64)
        k_gather<double><<<blocks, 256, 0, s>>>(
            n, perm, (const double*)in.x, (const double*)in.y, (const double*)in.z,
            (double*)out.x, (double*)out.y, (double*)out.z);
    else if (dtype == DSMC_F32)
        k_gather<float><<<blocks, 256, 0, s>>>(
            n, perm, (const float*)in.x, (const float*)in.y, (const float*)in.z,
            (float*)out.x, (float*)out.y, (float*)out.z);
    else
        return arg_error("dsmc_gather: dtype %d", dtype);
    DSMC_LAUNCH_CHECK("gather");
    return DSMC_OK;
}

extern "C" int dsmc_sample(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                           dsmc_vec3 v, double* acc, dsmc_stream_t stream)
{
    if (n_cells < 1) return arg_error("dsmc_sample: n_cells=%d", n_cells);
    if (!cell_start || !acc || !v.x || !v.y || !v.z)
        return arg_error("dsmc_sample: null pointer");
    hipStream_t s = as_stream(stream);
    const int pb = persistent_blocks(256);
    int blocks = (n_cells + 3) / 4;
    blocks = blocks > pb ? pb : blocks;
    if (dtype == DSMC_F64)
        k_sample<double><<<blocks, 256, 0, s>>>(cell_start, n_cells, v3<const double>(v), acc);
    else if (dtype == DSMC_F32)
        k_sample<float><<<blocks, 256, 0, s>>>(cell_start, n_cells, v3<const float>(v), acc);
    else
        return arg_error("dsmc_sample: dtype %d", dtype);
    DSMC_LAUNCH_CHECK("sample");
    return DSMC_OK;
}

extern "C" int dsmc_sample_fields(int32_t n_cells, const double* acc, double n_samples,
                                  double mass, double fnum_per_volume, double* fields,
                                  dsmc_stream_t stream)
{
    if (n_cells < 1) return arg_error("dsmc_sample_fields: n_cells=%d", n_cells);
    if (!acc || !fields) return arg_error("dsmc_sample_fields: null pointer");
    if (!(n_samples > 0) || !(mass > 0))
        return arg_error("dsmc_sample_fields: n_samples=%g mass=%g", n_samples, mass);
    k_fields<<<grid_for(n_cells, 256), 256, 0, as_stream(stream)>>>(n_cells, acc, n_samples,
                                                                    mass, fnum_per_volume,
                                                                    fields);
    DSMC_LAUNCH_CHECK("sample_fields");
    return DSMC_OK;
}
