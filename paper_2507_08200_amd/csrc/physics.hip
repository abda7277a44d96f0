// Explicit terms of the semi-implicit step: electric field and transport,
// WENO5 drift-flux divergence with wall fluxes, chemical sources, Poisson
// charge density.  FP64 throughout (the rate polynomials cancel
// catastrophically in lower precision).
#include "vd_internal.hpp"
#include "physics.hpp"

namespace vd {

// ----------------------------------------------------- electric field
// E along direction d at the face between row positions p-1 and p (face
// index p in 0..n): interior -(phi_R - phi_L)/h; Dirichlet face with value
// g: one-sided over half a cell; Neumann/wall: 0; periodic: wrapped.
__device__ __forceinline__ double e_face(const GridDev &G, const double *__restrict__ phi, int d, int c, int pos, int fidx) {
    const int n = G.n[d];
    const long st = G.stride[d];
    const double ih = G.ih[d];
    const long c0 = c - (long)pos * st;     // index of row position 0
    if (fidx > 0 && fidx < n) {
        // masked step: a covered cell's potential is the Dirichlet value of
        // its faces with valid cells (one-sided over half a cell); no field
        // between two covered cells
        if (G.mask) {
            const bool vl = gld(G.mask, c0 + (fidx - 1) * st) != 0, vr = gld(G.mask, c0 + fidx * st) != 0;
            if (!vl && !vr) return 0.0;
            if (vl != vr) return -(gld(phi, c0 + fidx * st) - gld(phi, c0 + (fidx - 1) * st)) * (2.0 * ih);
        }
        return -(gld(phi, c0 + fidx * st) - gld(phi, c0 + (fidx - 1) * st)) * ih;
    }
    const int f = 2 * d + (fidx == 0 ? 0 : 1);
    const int kind = G.phi_kind[f];
    if (kind == VD_BC_PERIODIC) return -(gld(phi, c0) - gld(phi, c0 + (n - 1) * st)) * ih;
    if (kind == VD_BC_DIRICHLET) {
        const double g = G.phi_val[f];
        if (fidx == 0) return -(gld(phi, c0) - g) * (2.0 * ih);
        return -(g - gld(phi, c0 + (n - 1) * st)) * (2.0 * ih);
    }
    return 0.0;
}

__device__ __forceinline__ void e_cell(const GridDev &G, const double *__restrict__ phi, int c, const int pos[3], double E[3]) {
    for (int d = 0; d < 3; d++) E[d] = 0.5 * (e_face(G, phi, d, c, pos[d], pos[d]) + e_face(G, phi, d, c, pos[d], pos[d] + 1));
}

constexpr double kTd = 1e-21;
constexpr double kENFloor = 1e-3;     // reduced-field floor before the log

__device__ __forceinline__ double mu_electron(double en_td, double N) {
    double en = en_td < kENFloor ? kENFloor : en_td;
    return exp(0.05481 - 2.911 * tanh(0.289 * log(en) + 0.543)) * (1.1296e25 / N);
}

__device__ __forceinline__ double te_lfa(const double *__restrict__ tab, int npts, double ln_min, double ln_max, double en_td) {
    double en = en_td < kENFloor ? kENFloor : en_td;
    double x = log(en);
    if (x <= ln_min) return gld(tab, 0);
    if (x >= ln_max) return gld(tab, npts - 1);
    double t = (x - ln_min) / ((ln_max - ln_min) / (double)(npts - 1));
    int i0 = (int)floor(t);
    i0 = i0 > npts - 2 ? npts - 2 : (i0 < 0 ? 0 : i0);
    double w = t - (double)i0;
    return (1.0 - w) * gld(tab, i0) + w * gld(tab, i0 + 1);
}

// Per cell: E/N, Te (fixed / table / from the electron energy) and, for the
// species with a field-dependent mobility, signed mu and D.
__global__ void __launch_bounds__(kBlock) k_transport(TransportArgs a) {
    const GridDev &G = a.g;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= G.ncell) return;
    int pos[3];
    pos[2] = c / G.nxy;
    int r = c - pos[2] * G.nxy;
    pos[1] = r / G.n[0];
    pos[0] = r - pos[1] * G.n[0];
    double E[3];
    e_cell(G, a.phi, c, pos, E);
    double en = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]) / a.N_gas / kTd;
    double Te;
    if (a.te_mode == VD_TE_LFA) {
        Te = te_lfa(a.lfa, a.lfa_n, a.lfa_ln_min, a.lfa_ln_max, en);
        gst(a.Te, c, Te);
    } else if (a.te_mode == VD_TE_ENERGY) {
        double ne = gld(a.ne, c);
        double t = ne > 0.0 ? gld(a.Ee, c) / (1.5 * ne * a.kB) : a.Tg;
        Te = ne > 0.0 ? (t < a.Tg ? a.Tg : (t > a.Te_max ? a.Te_max : t)) : a.Tg;
        gst(a.Te, c, Te);
    } else {
        Te = gld(a.Te, c);
    }
    for (int v = 0; v < a.nvar; v++) {
        double m = mu_electron(en, a.N_gas);
        gst(a.mu, (long)v * G.ncell + c, a.var_sign[v] * m);
        double D = m * a.kB * Te / a.qe;
        gst(a.D, (long)v * G.ncell + c, D);
        if (a.beta_e && v == a.e_var) gst(a.beta_e, c, 5.0 / 3.0 * D);
    }
}

// ------------------------------------------------------------- WENO5
// Jiang-Shu WENO5 value at the right face of the middle cell of
// (a, b, c, d, e), epsilon 1e-6, power 2.  The normalised weights
// alpha_k / sum(alpha) are evaluated with a single division by clearing the
// three denominators (algebraically identical).
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e) {
    const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
    const double q1 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
    const double q2 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
    const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, u1 = b - d;
    const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
    const double s0 = 1e-6 + (13.0 / 12.0) * t0 * t0 + 0.25 * u0 * u0;
    const double s1 = 1e-6 + (13.0 / 12.0) * t1 * t1 + 0.25 * u1 * u1;
    const double s2 = 1e-6 + (13.0 / 12.0) * t2 * t2 + 0.25 * u2 * u2;
    const double p0 = s0 * s0, p1 = s1 * s1, p2 = s2 * s2;
    const double w0 = 0.1 * (p1 * p2), w1 = 0.6 * (p0 * p2), w2 = 0.3 * (p0 * p1);
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

// value of field u at row position p along d (may be up to 3 outside):
// mirror at Neumann/wall faces, odd reflection about g at Dirichlet faces,
// wrap at periodic faces
__device__ __forceinline__ double u_at(const GridDev &G, const int *kind, const double *gval, const double *__restrict__ u,
                                       int d, long c0, int p) {
    const int n = G.n[d];
    const long st = G.stride[d];
    if (p >= 0 && p < n) return gld(u, c0 + p * st);
    // constant-index selects (no dynamic indexing of the descriptor arrays)
    const int kd = p < 0 ? (d == 0 ? kind[0] : d == 1 ? kind[2] : kind[4]) : (d == 0 ? kind[1] : d == 1 ? kind[3] : kind[5]);
    if (kd == VD_BC_PERIODIC) return gld(u, c0 + (p < 0 ? p + n : p - n) * st);
    const int q = p < 0 ? -1 - p : 2 * n - 1 - p;
    const double v = gld(u, c0 + q * st);
    const double g = p < 0 ? (d == 0 ? gval[0] : d == 1 ? gval[2] : gval[4]) : (d == 0 ? gval[1] : d == 1 ? gval[3] : gval[5]);
    return kd == VD_BC_DIRICHLET ? 2.0 * g - v : v;
}

// Masked step: the five upwind values of face fidx's WENO5 stencil (up:
// positions fidx-3 .. fidx+1, else fidx+2 down to fidx-2).  The nearest
// covered cell on each side, within reach, closes the valid run like a
// homogeneous Dirichlet domain face: a position past it takes minus the
// value mirrored across that face, 0 when the mirror leaves the run.
__device__ __forceinline__ void stencil5_masked(const GridDev &G, const FieldDesc &F, int d, long c0, int fidx, bool up,
                                                double s[5]) {
    const int n = G.n[d];
    const long st = G.stride[d];
    int lo = -1, hi = -1;
    for (int p = fidx - 1; p >= fidx - 3 && p >= 0; p--)
        if (!gld(G.mask, c0 + p * st)) { lo = p + 1; break; }
    for (int p = fidx; p <= fidx + 2 && p < n; p++)
        if (!gld(G.mask, c0 + p * st)) { hi = p; break; }
#pragma unroll
    for (int m = 0; m < 5; m++) {
        const int p = up ? fidx - 3 + m : fidx + 2 - m;
        const int fb = (lo >= 0 && p < lo) ? lo : ((hi >= 0 && p >= hi) ? hi : -1);
        if (fb < 0) { s[m] = u_at(G, F.kind, F.gval, F.u, d, c0, p); continue; }
        const int q = 2 * fb - 1 - p;
        const bool inrun = q >= 0 && q < n && (lo < 0 || q >= lo) && (hi < 0 || q < hi) && gld(G.mask, c0 + q * st) != 0;
        s[m] = inrun ? -gld(F.u, c0 + q * st) : 0.0;
    }
}

__device__ __forceinline__ double wall_flux(int wk, double uc, double mu, double e_n, double Te, double Tg, double mass,
                                            double kB, double me) {
    switch (wk) {
    case VD_WALL_ELECTRON: return uc * 0.25 * sqrt(8.0 * kB * Te / (M_PI * me));
    case VD_WALL_ION: { double f = mu * uc * e_n; return f > 0.0 ? f : 0.0; }
    case VD_WALL_NEUTRAL: return uc * 0.25 * sqrt(8.0 * kB * Tg / (M_PI * mass));
    default: return 0.0;
    }
}

// Outward wall flux of field F at its boundary cell cb with F's wall
// variants (Sec. 2.2): sticking scales the neutral flux; secondary emission
// returns gamma times the ions' wall fluxes of the face to the gas
__device__ __forceinline__ double wall_flux_f(const FieldDesc &F, long cb, double uc, double mu, double e_n, double Te,
                                              double Tg, double kB, double me) {
    double fl = wall_flux(F.wall, uc, mu, e_n, Te, Tg, F.mass, kB, me);
    if (F.wall == VD_WALL_NEUTRAL) fl = F.stick * fl;
    if (F.wall == VD_WALL_ELECTRON && F.see_gamma != 0.0) {
        double ions = 0.0;
        for (int q = 0; q < F.nion; q++) {
            const double mi = F.ion_mu[q] ? gld(F.ion_mu[q], cb) : F.ion_mu_c[q];
            ions += wall_flux(VD_WALL_ION, gld(F.ion_n[q], cb), mi, e_n, Te, Tg, 0.0, kB, me);
        }
        fl = fl - F.see_gamma * ions;
    }
    return fl;
}

// Drift flux along +d at a non-wall face fidx of the row through c: face
// velocity mu_f E_f (mu_f the mean of the two cells, the boundary cell's on
// a domain face) times the upwind WENO5 value.
__device__ __forceinline__ double face_drift(const GridDev &G, const FieldDesc &F, const double *__restrict__ phi, int d, int c,
                                             int pos, int fidx) {
    const int n = G.n[d];
    const long st = G.stride[d];
    const long c0 = c - (long)pos * st;
    const bool boundary = (fidx == 0 || fidx == n);
    const int kd = fidx == 0 ? (d == 0 ? F.kind[0] : d == 1 ? F.kind[2] : F.kind[4])
                             : (d == 0 ? F.kind[1] : d == 1 ? F.kind[3] : F.kind[5]);
    const double *__restrict__ u = F.u;
    if (!F.mu && F.mu_c == 0.0) return 0.0;
    // masked step: validity of the face's two cells (a domain face has one)
    bool vl = true, vr = true;
    if (G.mask) {
        vl = fidx > 0 && gld(G.mask, c0 + (fidx - 1) * st) != 0;
        vr = fidx < n && gld(G.mask, c0 + fidx * st) != 0;
        if (!vl && !vr) return 0.0;
    }
    const double Ef = e_face(G, phi, d, c, pos, fidx);
    double muf;
    if (F.mu) {
        const int pl = fidx - 1, pr = fidx;
        if (boundary && kd != VD_BC_PERIODIC) muf = fidx == 0 ? gld(F.mu, c0) : gld(F.mu, c0 + (n - 1) * st);
        else if (vl != vr) muf = vl ? gld(F.mu, c0 + pl * st) : gld(F.mu, c0 + pr * st);   // the valid cell's
        else {
            const int ql = pl < 0 ? pl + n : pl, qr = pr >= n ? pr - n : pr;
            muf = 0.5 * (gld(F.mu, c0 + ql * st) + gld(F.mu, c0 + qr * st));
        }
    } else {
        muf = F.mu_c;
    }
    const double v = muf * F.mu_scale * Ef;
    if (v == 0.0) return 0.0;
    if (G.mask) {
        double sm[5];
        stencil5_masked(G, F, d, c0, fidx, v > 0.0, sm);
        return v * weno5(sm[0], sm[1], sm[2], sm[3], sm[4]);
    }
    double s0, s1, s2, s3, s4;
    if (v > 0.0) {
        const int b = fidx - 3;
        s0 = u_at(G, F.kind, F.gval, u, d, c0, b);
        s1 = u_at(G, F.kind, F.gval, u, d, c0, b + 1);
        s2 = u_at(G, F.kind, F.gval, u, d, c0, b + 2);
        s3 = u_at(G, F.kind, F.gval, u, d, c0, b + 3);
        s4 = u_at(G, F.kind, F.gval, u, d, c0, b + 4);
    } else {
        const int b = fidx + 2;
        s0 = u_at(G, F.kind, F.gval, u, d, c0, b);
        s1 = u_at(G, F.kind, F.gval, u, d, c0, b - 1);
        s2 = u_at(G, F.kind, F.gval, u, d, c0, b - 2);
        s3 = u_at(G, F.kind, F.gval, u, d, c0, b - 3);
        s4 = u_at(G, F.kind, F.gval, u, d, c0, b - 4);
    }
    return v * weno5(s0, s1, s2, s3, s4);
}

// Drift-flux divergence of one field at cell c (faces x-, x+, y-, y+, z-, z+).
__device__ double drift_div_cell(const GridDev &G, const FieldDesc &F, const double *__restrict__ phi,
                                 const double *__restrict__ Te, double Tg, double kB, double me, int c, const int pos[3]) {
    double total = 0.0;
    if (G.mask && !gld(G.mask, (long)c)) return 0.0;     // covered: no balance
    const double *__restrict__ u = F.u;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int n = G.n[d];
        double Fs[2];
#pragma unroll
        for (int side = 0; side < 2; side++) {
            const int fidx = pos[d] + side;
            const bool boundary = (fidx == 0 || fidx == n);
            const int kd = F.kind[2 * d + side];
            if (boundary && kd == VD_BC_NEUMANN) { Fs[side] = 0.0; continue; }
            const double Ef = e_face(G, phi, d, c, pos[d], fidx);
            if (boundary && kd == VD_BC_WALLFLUX) {
                const double e_n = fidx == 0 ? -Ef : Ef;
                double fl;
                if (F.ne_wall) {
                    fl = 2.0 * kB * gld(Te, c) * wall_flux(VD_WALL_ELECTRON, gld(F.ne_wall, c), 0.0, e_n, gld(Te, c), Tg, me, kB, me);
                } else {
                    const double muc = F.mu ? gld(F.mu, c) : F.mu_c;
                    fl = wall_flux_f(F, c, gld(u, c), muc, e_n, gld(Te, c), Tg, kB, me);
                }
                Fs[side] = fidx == 0 ? -fl : fl;
                continue;
            }
            Fs[side] = face_drift(G, F, phi, d, c, pos[d], fidx);
        }
        total += (Fs[1] - Fs[0]) * G.ihl[d];
    }
    return total;
}

// Complete flux along +d through face fidx of the row starting at c0:
// Neumann faces carry nothing, wall faces the wall flux of the adjacent
// boundary cell (sign of the outward normal folded in), other faces the
// upwind WENO5 drift flux.
__device__ __forceinline__ double face_flux(const GridDev &G, const FieldDesc &F, const double *__restrict__ phi,
                                            const double *__restrict__ Te, double Tg, double kB, double me, int d,
                                            long c0, int fidx) {
    const int n = G.n[d];
    if (fidx == 0 || fidx == n) {
        const int kd = fidx == 0 ? (d == 0 ? F.kind[0] : d == 1 ? F.kind[2] : F.kind[4])
                                 : (d == 0 ? F.kind[1] : d == 1 ? F.kind[3] : F.kind[5]);
        if (kd == VD_BC_NEUMANN) return 0.0;
        if (kd == VD_BC_WALLFLUX) {
            const long cb = c0 + (fidx == 0 ? 0 : (long)(n - 1) * G.stride[d]);
            const double Ef = e_face(G, phi, d, (int)c0, 0, fidx);
            const double e_n = fidx == 0 ? -Ef : Ef;
            double fl;
            if (F.ne_wall) fl = 2.0 * kB * gld(Te, cb) * wall_flux(VD_WALL_ELECTRON, gld(F.ne_wall, cb), 0.0, e_n, gld(Te, cb), Tg, me, kB, me);
            else fl = wall_flux_f(F, cb, gld(F.u, cb), F.mu ? gld(F.mu, cb) : F.mu_c, e_n, gld(Te, cb), Tg, kB, me);
            return fidx == 0 ? -fl : fl;
        }
    }
    return face_drift(G, F, phi, d, (int)c0, 0, fidx);
}

// Value of field u at row position p (up to 3 outside), as u_at, with
// every branch turned into a select: one load from a valid index, so the
// loads of a face stencil are issued together.
__device__ __forceinline__ double u_at_bf(const GridDev &G, const FieldDesc &F, int d, long c0, int p) {
    const int n = G.n[d];
    const bool lo = p < 0, hi = p >= n;
    const int kd = lo ? (d == 0 ? F.kind[0] : d == 1 ? F.kind[2] : F.kind[4])
                      : (d == 0 ? F.kind[1] : d == 1 ? F.kind[3] : F.kind[5]);
    const bool per = kd == VD_BC_PERIODIC;
    int q = lo ? (per ? p + n : -1 - p) : (hi ? (per ? p - n : 2 * n - 1 - p) : p);
    q = q < 0 ? 0 : (q >= n ? n - 1 : q);
    const double v = gld(F.u, c0 + q * G.stride[d]);
    const double g = lo ? (d == 0 ? F.gval[0] : d == 1 ? F.gval[2] : F.gval[4])
                        : (d == 0 ? F.gval[1] : d == 1 ? F.gval[3] : F.gval[5]);
    return ((lo || hi) && kd == VD_BC_DIRICHLET) ? 2.0 * g - v : v;
}

// face_flux for an interior face (0 < fidx < n) without branches around
// loads: phi at the two cells, the two cells' mobilities (the field itself
// stands in as a valid address when the mobility is constant) and the six
// stencil values of both upwind directions are loaded together, the upwind
// side is then selected.  Domain faces fall back to face_flux.
__device__ __forceinline__ double face_flux_fast(const GridDev &G, const FieldDesc &F, const double *__restrict__ phi,
                                                 const double *__restrict__ Te, double Tg, double kB, double me, int d,
                                                 long c0, int fidx, bool drift) {
    const int n = G.n[d];
    if (fidx == 0 || fidx == n) return face_flux(G, F, phi, Te, Tg, kB, me, d, c0, fidx);
    if (!drift) return 0.0;
    const long st = G.stride[d];
    const long cl = c0 + (long)(fidx - 1) * st, cr = cl + st;
    const double Ef = -(gld(phi, cr) - gld(phi, cl)) * G.ih[d];
    const double *__restrict__ mup = F.mu ? F.mu : F.u;
    const double ml = gld(mup, cl), mr = gld(mup, cr);
    double w[6];
#pragma unroll
    for (int m = 0; m < 6; m++) w[m] = u_at_bf(G, F, d, c0, fidx - 3 + m);
    const double muf = F.mu ? 0.5 * (ml + mr) : F.mu_c;
    const double v = muf * F.mu_scale * Ef;
    const bool up = v > 0.0;
    return v * weno5(up ? w[0] : w[5], up ? w[1] : w[4], up ? w[2] : w[3], up ? w[3] : w[2], up ? w[4] : w[1]);
}

// Tiled drift divergence: a workgroup owns a kTX x kTY tile of an x-y plane
// and marches kKZ planes in z.  Every face flux is evaluated once: x and y
// faces go through LDS (the tile-edge faces are remapped onto the first
// wave), the z face is carried from one plane to the next in a register.
constexpr int kTX = 32, kTY = 8;

__global__ void __launch_bounds__(kBlock) k_drift_tiled(DriftArgs a, int kz) {
    __shared__ double fx[kTY * (kTX + 1)];
    __shared__ double fy[(kTY + 1) * kTX];
    const GridDev &G = a.g;
    const FieldDesc F = a.f[blockIdx.y];
    if (F.rhs_done) return;
    const int nx = G.n[0], ny = G.n[1];
    const int tiles_x = nx / kTX, tiles_y = ny / kTY;
    int b = blockIdx.x;
    const int bx = b % tiles_x;
    b /= tiles_x;
    const int by = b % tiles_y;
    const int bz = b / tiles_y;
    const int tx = threadIdx.x & (kTX - 1), ty = threadIdx.x / kTX;
    const int i0 = bx * kTX, j0 = by * kTY, k0 = bz * kz;
    const int i = i0 + tx, j = j0 + ty;
    const long nxy = G.nxy;
    const long col = i + (long)nx * j;                  // (i, j, 0)
    // x faces: face f of row r of the tile, f in 0..kTX (kTY*(kTX+1) faces)
    const int nfx = kTY * (kTX + 1), nfy = (kTY + 1) * kTX;
    const bool drift = F.mu || F.mu_c != 0.0;
    double fz_lo = face_flux_fast(G, F, a.phi, a.Te, a.Tg, a.kB, a.me, 2, col, k0, drift);
    for (int k = k0; k < k0 + kz; k++) {
        const long pl = nxy * k;
        for (int q = threadIdx.x; q < nfx; q += kBlock) {
            const int r = q / (kTX + 1), f = q - r * (kTX + 1);
            fx[q] = face_flux_fast(G, F, a.phi, a.Te, a.Tg, a.kB, a.me, 0, pl + (long)nx * (j0 + r), i0 + f, drift);
        }
        for (int q = threadIdx.x; q < nfy; q += kBlock) {
            const int r = q / kTX, f = q - r * kTX;
            fy[q] = face_flux_fast(G, F, a.phi, a.Te, a.Tg, a.kB, a.me, 1, pl + i0 + f, j0 + r, drift);
        }
        const double fz_hi = face_flux_fast(G, F, a.phi, a.Te, a.Tg, a.kB, a.me, 2, col, k + 1, drift);
        __syncthreads();
        const double div = (fx[ty * (kTX + 1) + tx + 1] - fx[ty * (kTX + 1) + tx]) * G.ihl[0] +
                           (fy[(ty + 1) * kTX + tx] - fy[ty * kTX + tx]) * G.ihl[1] + (fz_hi - fz_lo) * G.ihl[2];
        const long c = col + pl;
        if (a.mode == 0) {
            gst(F.out, c, div);
        } else {
            double v = gld(F.u0, c) * a.inv_dt - div;
            if (F.src) v += gld(F.src, c);
            if (F.extra) v += gld(F.extra, c);
            gst(F.out, c, v);
        }
        fz_lo = fz_hi;
        __syncthreads();
    }
}

// ------------------------------------------- 2.5D LDS-staged WENO5 divergence
// A workgroup owns a 32 x 8 tile of x-y planes of one field and marches kz
// planes in z.  Per plane, the field (with a three-cell ring of ghost values:
// mirror, odd reflection or wrap, as u_at), phi and the mobility (one-cell
// rings) are staged in LDS from loads issued a plane ahead into registers;
// the z stencil of each thread's column lives in registers.  Every face
// flux is then arithmetic on staged values: domain faces are resolved by
// selects (a Neumann or wall face carries no drift flux here; the wall
// fluxes are added to the boundary cells by k_wall_div).  No global load
// sits in a branch, so the look-ahead loads overlap the face computations.
constexpr int kDX = 32, kDY = 8;
constexpr int kUX = kDX + 6, kUY = kDY + 6;          // field tile, ring 3
constexpr int kPX = kDX + 2, kPY = kDY + 2;          // phi / mobility tiles, ring 1
constexpr int kUN = kUX * kUY, kPN = kPX * kPY;
constexpr int kUPer = (kUN + kBlock - 1) / kBlock;   // 3
constexpr int kPPer = (kPN + kBlock - 1) / kBlock;   // 2

// ghost-mapped row position of the field along a direction: index of the
// cell to read and whether the value is reflected about g (Dirichlet)
__device__ __forceinline__ int ghost_pos(int p, int n, int klo, int khi, bool &odd, bool &hi_side) {
    const bool lo = p < 0, hi = p >= n;
    const int kd = lo ? klo : khi;
    const bool per = kd == VD_BC_PERIODIC;
    int q = lo ? (per ? p + n : -1 - p) : (hi ? (per ? p - n : 2 * n - 1 - p) : p);
    q = q < 0 ? 0 : (q >= n ? n - 1 : q);
    odd = (lo || hi) && kd == VD_BC_DIRICHLET;
    hi_side = hi;
    return q;
}

__device__ __forceinline__ int wrapc(int p, int n, bool per) {
    int q = per ? (p < 0 ? p + n : (p >= n ? p - n : p)) : p;
    return q < 0 ? 0 : (q >= n ? n - 1 : q);
}

// drift flux of one face from staged values: w the six stencil values
// (positions -3..+2 around the face), phi / mobility of the two cells.
// lo / hi mark a domain face; kf the field kind there, kp / gp phi's.
__device__ __forceinline__ double drift_face(const FieldDesc &F, double w0, double w1, double w2, double w3, double w4,
                                             double w5, double phl, double phr, double mul, double mur, double ih, bool lo,
                                             bool hi, int kf, int kp, double gp) {
    double Ef = -(phr - phl) * ih;
    const bool per = kp == VD_BC_PERIODIC;
    if ((lo || hi) && !per) Ef = kp == VD_BC_DIRICHLET ? (lo ? -(phr - gp) * (2.0 * ih) : -(gp - phl) * (2.0 * ih)) : 0.0;
    double muf = F.mu ? 0.5 * (mul + mur) : F.mu_c;
    if (F.mu && (lo || hi) && kf != VD_BC_PERIODIC) muf = lo ? mur : mul;
    const double v = muf * F.mu_scale * Ef;
    const bool up = v > 0.0;
    const double fl = v * weno5(up ? w0 : w5, up ? w1 : w4, up ? w2 : w3, up ? w3 : w2, up ? w4 : w1);
    const bool none = (lo || hi) && (kf == VD_BC_NEUMANN || kf == VD_BC_WALLFLUX);
    return none ? 0.0 : fl;
}

__global__ void __launch_bounds__(kBlock) k_drift25(DriftArgs a, int kz) {
    __shared__ double U[kUN], P[kPN], M[kPN];
    __shared__ double fx[kDY * (kDX + 1)];
    __shared__ double fy[(kDY + 1) * kDX];
    const GridDev &G = a.g;
    const FieldDesc F = a.f[blockIdx.y];
    if (F.rhs_done) return;
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const int tiles_x = nx / kDX, tiles_y = ny / kDY;
    int b = blockIdx.x;
    const int bx = b % tiles_x;
    b /= tiles_x;
    const int by = b % tiles_y;
    const int bz = b / tiles_y;
    const int tid = threadIdx.x;
    const int tx = tid & (kDX - 1), ty = tid / kDX;
    const int i0 = bx * kDX, j0 = by * kDY, k0 = bz * kz;
    const int i = i0 + tx, j = j0 + ty;
    const long nxy = G.nxy;
    const long col = i + (long)nx * j;
    const bool drift = F.mu || F.mu_c != 0.0;
    if (!drift) {
        // a field without mobility has no drift flux: its divergence is 0;
        // four planes' loads are issued before their stores
        const long c0 = col + nxy * k0;
        double *__restrict__ out = F.out;
        const double *__restrict__ pu0 = F.u0 ? F.u0 : F.u;
        const double *__restrict__ psrc = F.src;
        const double *__restrict__ pex = F.extra;
        for (int k = 0; k < kz; k += 4) {
            double v[4];
            if (a.mode == 0) {
#pragma unroll
                for (int m = 0; m < 4; m++) v[m] = 0.0;
            } else {
                double s0[4], e0[4];
#pragma unroll
                for (int m = 0; m < 4; m++) {
                    const long c = c0 + nxy * (k + m);
                    v[m] = gld(pu0, c);
                    s0[m] = psrc ? gld(psrc, c) : 0.0;
                    e0[m] = pex ? gld(pex, c) : 0.0;
                }
#pragma unroll
                for (int m = 0; m < 4; m++) {
                    v[m] = v[m] * a.inv_dt - 0.0;
                    if (psrc) v[m] += s0[m];
                    if (pex) v[m] += e0[m];
                }
            }
#pragma unroll
            for (int m = 0; m < 4; m++) gst(out, c0 + nxy * (k + m), v[m]);
        }
        return;
    }
    const double *__restrict__ u = F.u;
    const double *__restrict__ mup = F.mu ? F.mu : F.u;      // valid address when the mobility is constant
    const double *__restrict__ phi = a.phi;
    // per-thread x-y parts of the staged loads (plane-invariant)
    long uo[kUPer], po[kPPer];
    bool uodd[kUPer], uhi[kUPer];
    int ud[kUPer];                                   // direction whose ghost rule applies (0 x, 1 y, -1 none)
#pragma unroll
    for (int m = 0; m < kUPer; m++) {
        const int e = min(tid + m * kBlock, kUN - 1);
        const int ri = e % kUX, rj = e / kUX;
        const int gi = i0 - 3 + ri, gj = j0 - 3 + rj;
        bool oi, hi_i, oj, hi_j;
        const int qi = ghost_pos(gi, nx, F.kind[0], F.kind[1], oi, hi_i);
        const int qj = ghost_pos(gj, ny, F.kind[2], F.kind[3], oj, hi_j);
        uo[m] = qi + (long)nx * qj;
        // corner ghosts are never read by a face stencil; an x ghost takes
        // the x rule, a y ghost the y rule
        ud[m] = (gi < 0 || gi >= nx) ? 0 : ((gj < 0 || gj >= ny) ? 1 : -1);
        uodd[m] = ud[m] == 0 ? oi : (ud[m] == 1 ? oj : false);
        uhi[m] = ud[m] == 0 ? hi_i : hi_j;
    }
    // phi's ring wraps by phi's boundary kinds, the mobility's by the field's
    const bool pxp = G.phi_kind[0] == VD_BC_PERIODIC, pyp = G.phi_kind[2] == VD_BC_PERIODIC;
    const bool fxp = F.kind[0] == VD_BC_PERIODIC, fyp = F.kind[2] == VD_BC_PERIODIC;
    long mo[kPPer];
#pragma unroll
    for (int m = 0; m < kPPer; m++) {
        const int e = min(tid + m * kBlock, kPN - 1);
        const int ri = e % kPX, rj = e / kPX;
        po[m] = wrapc(i0 - 1 + ri, nx, pxp) + (long)nx * wrapc(j0 - 1 + rj, ny, pyp);
        mo[m] = wrapc(i0 - 1 + ri, nx, fxp) + (long)nx * wrapc(j0 - 1 + rj, ny, fyp);
    }
    const double gu_xlo = F.gval[0], gu_xhi = F.gval[1], gu_ylo = F.gval[2], gu_yhi = F.gval[3];
    double gsel[kUPer];
#pragma unroll
    for (int m = 0; m < kUPer; m++) gsel[m] = ud[m] == 0 ? (uhi[m] ? gu_xhi : gu_xlo) : (uhi[m] ? gu_yhi : gu_ylo);
    // staged tile values of one plane (registers) and their LDS store
#define VD_STAGE(K, US0, US1, US2, PS0, PS1, MS0, MS1)                                      \
    {                                                                                       \
        const long pl_ = nxy * min(max((K), 0), nz - 1);                                    \
        double v_;                                                                          \
        v_ = gld(u, uo[0] + pl_); US0 = uodd[0] ? 2.0 * gsel[0] - v_ : v_;                  \
        v_ = gld(u, uo[1] + pl_); US1 = uodd[1] ? 2.0 * gsel[1] - v_ : v_;                  \
        v_ = gld(u, uo[2] + pl_); US2 = uodd[2] ? 2.0 * gsel[2] - v_ : v_;                  \
        PS0 = gld(phi, po[0] + pl_); PS1 = gld(phi, po[1] + pl_);                           \
        MS0 = gld(mup, mo[0] + pl_); MS1 = gld(mup, mo[1] + pl_);                           \
    }
    static_assert(kUPer == 3 && kPPer == 2, "staging is written for 3 + 2 values per thread");
    // z column of this thread: field at planes k-3..k+3 (ghost rule in z),
    // phi and mobility at planes k-1..k+1
    bool zodd;
    bool zhi;
    auto zu = [&](int k) -> double {
        const int q = ghost_pos(k, nz, F.kind[4], F.kind[5], zodd, zhi);
        const double v = gld(u, col + nxy * q);
        return zodd ? 2.0 * (zhi ? F.gval[5] : F.gval[4]) - v : v;
    };
    const bool pzp = G.phi_kind[4] == VD_BC_PERIODIC, fzp = F.kind[4] == VD_BC_PERIODIC;
    auto zp = [&](int k) -> double { return gld(phi, col + nxy * wrapc(k, nz, pzp)); };
    auto zm = [&](int k) -> double { return gld(mup, col + nxy * wrapc(k, nz, fzp)); };
    const double ihx = G.ih[0], ihy = G.ih[1], ihz = G.ih[2];
    const bool inner = bx > 0 && bx < tiles_x - 1 && by > 0 && by < tiles_y - 1;
    // the z face above plane k from the column registers
    // column registers: z1..z6 = field at planes k-2 .. k+3
    double z1, z2, z3, z4, z5, z6;
    auto zface = [&](double ph0, double ph1, double mu0, double mu1, int k) -> double {
        const bool lo = (k + 1) == 0, hi = (k + 1) == nz;
        const int kf = lo ? F.kind[4] : F.kind[5];
        const int kp = lo ? G.phi_kind[4] : G.phi_kind[5];
        const double gp = lo ? G.phi_val[4] : G.phi_val[5];
        return drift_face(F, z1, z2, z3, z4, z5, z6, ph0, ph1, mu0, mu1, ihz, lo, hi, kf, kp, gp);
    };
    double ph_m = zp(k0 - 1), ph_c = zp(k0), ph_p = zp(k0 + 1);
    double mu_m = zm(k0 - 1), mu_c = zm(k0), mu_p = zm(k0 + 1);
    // flux below plane k0: face k0-1/2, stencil planes k0-3 .. k0+2
    double fz_lo;
    {
        const double a3 = zu(k0 - 3), a2 = zu(k0 - 2), a1 = zu(k0 - 1), b0 = zu(k0), b1 = zu(k0 + 1), b2 = zu(k0 + 2);
        fz_lo = drift_face(F, a3, a2, a1, b0, b1, b2, ph_m, ph_c, mu_m, mu_c, ihz, k0 == 0, false, F.kind[4], G.phi_kind[4],
                           G.phi_val[4]);
        if (!drift) fz_lo = 0.0;
        z1 = a2; z2 = a1; z3 = b0; z4 = b1; z5 = b2;
        z6 = zu(k0 + 3);
    }
    double us0, us1, us2, ps0, ps1, ms0, ms1;
    VD_STAGE(k0, us0, us1, us2, ps0, ps1, ms0, ms1);
    double u0v = 0.0, srcv = 0.0, exv = 0.0;
    const double *__restrict__ u0p = F.u0 ? F.u0 : u;
    const double *__restrict__ srcp = F.src ? F.src : u;
    const double *__restrict__ exp_ = F.extra ? F.extra : u;
    for (int k = k0; k < k0 + kz; k++) {
        lst(U, tid, us0);
        lst(U, tid + kBlock, us1);
        if (tid + 2 * kBlock < kUN) lst(U, tid + 2 * kBlock, us2);
        lst(P, tid, ps0);
        lst(M, tid, ms0);
        if (tid + kBlock < kPN) { lst(P, tid + kBlock, ps1); lst(M, tid + kBlock, ms1); }
        // look-ahead loads: next plane's tiles, the column's next values,
        // this plane's right-hand-side inputs
        double nus0, nus1, nus2, nps0, nps1, nms0, nms1;
        VD_STAGE(k + 1, nus0, nus1, nus2, nps0, nps1, nms0, nms1);
        const double cnext = zu(k + 4);
        const double ph_n = zp(k + 2), mu_n = zm(k + 2);
        const long c = col + nxy * k;
        u0v = gld(u0p, c);
        srcv = gld(srcp, c);
        exv = gld(exp_, c);
        __syncthreads();
        // x faces (tile rows 0..7, faces 0..32) and y faces (rows 0..8)
        // x faces (tile rows 0..7, faces 0..32) then y faces (rows 0..8) in
        // one loop, with the direction chosen by selects: a wavefront
        // holding both kinds evaluates each face once
        constexpr int kNFX = kDY * (kDX + 1), kNFY = (kDY + 1) * kDX;
        if (inner) {
            // a tile away from the x and y domain faces: no boundary rules
            for (int q = tid; q < kNFX + kNFY; q += kBlock) {
                const bool xf = q < kNFX;
                const int qy = q - kNFX;
                const int r = xf ? q / (kDX + 1) : qy / kDX;
                const int f = xf ? q - r * (kDX + 1) : qy - r * kDX;
                const int ub = xf ? (r + 3) * kUX + f : r * kUX + f + 3;
                const int us = xf ? 1 : kUX;
                const int pb = xf ? (r + 1) * kPX + f : r * kPX + f + 1;
                const int ps = xf ? 1 : kPX;
                const double fl = drift_face(F, lld(U, ub), lld(U, ub + us), lld(U, ub + 2 * us), lld(U, ub + 3 * us),
                                             lld(U, ub + 4 * us), lld(U, ub + 5 * us), lld(P, pb), lld(P, pb + ps),
                                             lld(M, pb), lld(M, pb + ps), xf ? ihx : ihy, false, false, 0, 0, 0.0);
                lst(xf ? fx : fy, xf ? q : qy, fl);
            }
        } else for (int q = tid; q < kNFX + kNFY; q += kBlock) {
            const bool xf = q < kNFX;
            const int qy = q - kNFX;
            const int r = xf ? q / (kDX + 1) : qy / kDX;
            const int f = xf ? q - r * (kDX + 1) : qy - r * kDX;
            const int g = xf ? i0 + f : j0 + r;            // face between cells g-1 and g along the direction
            const int ub = xf ? (r + 3) * kUX + f : r * kUX + f + 3;   // U index of cell g-3
            const int us = xf ? 1 : kUX;
            const int pb = xf ? (r + 1) * kPX + f : r * kPX + f + 1;   // P index of cell g-1
            const int ps = xf ? 1 : kPX;
            const bool lo = g == 0, hi = g == (xf ? nx : ny);
            const int kf = xf ? (lo ? F.kind[0] : F.kind[1]) : (lo ? F.kind[2] : F.kind[3]);
            const int kp = xf ? (lo ? G.phi_kind[0] : G.phi_kind[1]) : (lo ? G.phi_kind[2] : G.phi_kind[3]);
            const double gp = xf ? (lo ? G.phi_val[0] : G.phi_val[1]) : (lo ? G.phi_val[2] : G.phi_val[3]);
            const double fl = drift_face(F, lld(U, ub), lld(U, ub + us), lld(U, ub + 2 * us), lld(U, ub + 3 * us),
                                         lld(U, ub + 4 * us), lld(U, ub + 5 * us), lld(P, pb), lld(P, pb + ps), lld(M, pb),
                                         lld(M, pb + ps), xf ? ihx : ihy, lo, hi, kf, kp, gp);
            lst(xf ? fx : fy, xf ? q : qy, drift ? fl : 0.0);
        }
        const double fz_hi = drift ? zface(ph_c, ph_p, mu_c, mu_p, k) : 0.0;
        __syncthreads();
        const double div = (lld(fx, ty * (kDX + 1) + tx + 1) - lld(fx, ty * (kDX + 1) + tx)) * G.ihl[0] +
                           (lld(fy, (ty + 1) * kDX + tx) - lld(fy, ty * kDX + tx)) * G.ihl[1] + (fz_hi - fz_lo) * G.ihl[2];
        if (a.mode == 0) {
            gst(F.out, c, div);
        } else {
            double v = u0v * a.inv_dt - div;
            if (F.src) v += srcv;
            if (F.extra) v += exv;
            gst(F.out, c, v);
        }
        fz_lo = fz_hi;
        z1 = z2; z2 = z3; z3 = z4; z4 = z5; z5 = z6; z6 = cnext;
        ph_m = ph_c; ph_c = ph_p; ph_p = ph_n;
        mu_m = mu_c; mu_c = mu_p; mu_p = mu_n;
        us0 = nus0; us1 = nus1; us2 = nus2;
        ps0 = nps0; ps1 = nps1; ms0 = nms0; ms1 = nms1;
    }
#undef VD_STAGE
}

// Wall fluxes (Sec. 2.2, Eqs. (14)-(16)) of the WALLFLUX domain faces along direction
// d, added to the boundary cells' divergence after k_drift25 (mode 0: out +=
// contribution; mode 1: out -= it).  One thread per boundary line handles
// both ends, so no cell is updated twice in a launch.
__global__ void __launch_bounds__(kBlock) k_wall_div(DriftArgs a, int d) {
    const GridDev &G = a.g;
    const FieldDesc F = a.f[blockIdx.y];
    const int n = G.n[d];
    const int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
    const int na = G.n[da], nb = G.n[db];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= na * nb) return;
    const int pa = t % na, pb = t / na;
    long base = (long)pa * G.stride[da] + (long)pb * G.stride[db];
    for (int side = 0; side < 2; side++) {
        const int kd = side == 0 ? (d == 0 ? F.kind[0] : d == 1 ? F.kind[2] : F.kind[4])
                                 : (d == 0 ? F.kind[1] : d == 1 ? F.kind[3] : F.kind[5]);
        if (kd != VD_BC_WALLFLUX) continue;
        const long cb = base + (side == 0 ? 0 : (long)(n - 1) * G.stride[d]);
        const double Ef = e_face(G, a.phi, d, (int)base, 0, side == 0 ? 0 : n);
        const double e_n = side == 0 ? -Ef : Ef;
        double fl;
        if (F.ne_wall)
            fl = 2.0 * a.kB * gld(a.Te, cb) *
                 wall_flux(VD_WALL_ELECTRON, gld(F.ne_wall, cb), 0.0, e_n, gld(a.Te, cb), a.Tg, a.me, a.kB, a.me);
        else
            fl = wall_flux_f(F, cb, gld(F.u, cb), F.mu ? gld(F.mu, cb) : F.mu_c, e_n, gld(a.Te, cb), a.Tg, a.kB, a.me);
        // flux along +d through the face, and its share of the cell's divergence
        const double Fs = side == 0 ? -fl : fl;
        const double contrib = (side == 0 ? -Fs : Fs) * G.ihl[d];
        gst(F.out, cb, gld(F.out, cb) + (a.mode == 0 ? contrib : -contrib));
    }
}

// blockIdx.y = field.  mode 0: out = div.  mode 1 (species / energy
// right-hand side of the implicit solve): out = u0/dt - div + src + extra.
__global__ void __launch_bounds__(kBlock) k_drift(DriftArgs a) {
    const GridDev &G = a.g;
    const FieldDesc F = a.f[blockIdx.y];
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= G.ncell || F.rhs_done) return;
    int pos[3];
    pos[2] = c / G.nxy;
    int r = c - pos[2] * G.nxy;
    pos[1] = r / G.n[0];
    pos[0] = r - pos[1] * G.n[0];
    double div = drift_div_cell(G, F, a.phi, a.Te, a.Tg, a.kB, a.me, c, pos);
    if (a.mode == 0) {
        gst(F.out, c, div);
    } else {
        double v = gld(F.u0, c) * a.inv_dt - div;
        if (F.src) v += gld(F.src, c);
        if (F.extra) v += gld(F.extra, c);
        gst(F.out, c, v);
    }
}

// masked step: the cells flagged by k_mask_near get their divergence again
// from the mask-aware per-cell functions, after the unmasked kernels have
// filled every cell (elsewhere the masked formulas are the unmasked ones)
__global__ void __launch_bounds__(kBlock) k_drift_fix(DriftArgs a) {
    const GridDev &G = a.g;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= G.ncell || !gld(a.near, (long)c)) return;
    const FieldDesc F = a.f[blockIdx.y];
    if (F.rhs_done) return;
    int pos[3];
    pos[2] = c / G.nxy;
    int r = c - pos[2] * G.nxy;
    pos[1] = r / G.n[0];
    pos[0] = r - pos[1] * G.n[0];
    double div = drift_div_cell(G, F, a.phi, a.Te, a.Tg, a.kB, a.me, c, pos);
    if (a.mode == 0) {
        gst(F.out, c, div);
    } else {
        double v = gld(F.u0, c) * a.inv_dt - div;
        if (F.src) v += gld(F.src, c);
        if (F.extra) v += gld(F.extra, c);
        gst(F.out, c, v);
    }
}

__global__ void __launch_bounds__(kBlock) k_mask_near(GridDev G, uint8_t *__restrict__ near) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= G.ncell) return;
    int pos[3];
    pos[2] = c / G.nxy;
    const int r = c - pos[2] * G.nxy;
    pos[1] = r / G.n[0];
    pos[0] = r - pos[1] * G.n[0];
    bool f = !gld(G.mask, (long)c);
    for (int d = 0; d < 3 && !f; d++)
        for (int o = -3; o <= 3; o++) {
            const int p = pos[d] + o;
            if (o == 0 || p < 0 || p >= G.n[d]) continue;
            if (!gld(G.mask, (long)c + (long)o * G.stride[d])) { f = true; break; }
        }
    gst(near, (long)c, (uint8_t)(f ? 1 : 0));
}

void launch_mask_near(vd_ctx *ctx, const GridDev &G, uint8_t *near) {
    k_mask_near<<<ceil_div(G.ncell, kBlock), kBlock, 0, ctx->stream>>>(G, near);
    VD_HIP(hipGetLastError());
}

// ------------------------------------------------------------ chemistry
constexpr double kEvK = 11604.518;

// Ar-H2 mechanism, Tables A.1-A.3 (species e, Ar+, Ar2+, H+, H2+, H3+, ArH+,
// Ar*, Ar2*, H2(v1), H2(v2), H2(v3), H, Ar, H2).  R6 read as an ionization
// (Ar2+ + 2e), R11 as 2 Ar2* -> Ar2+ + 2 Ar + e, R24-R26 with Te in eV.
enum { SE = 0, SARP, SAR2P, SHP, SH2P, SH3P, SARHP, SARS, SAR2S, SH2V1, SH2V2, SH2V3, SH, SAR, SH2 };

__device__ __forceinline__ double vib(double L, double c0, double c1, double c2, double c3, double c4, double c5,
                                      double c6, double c7, double c8) {
    return exp(c0 + L * (c1 + L * (c2 + L * (c3 + L * (c4 + L * (c5 + L * (c6 + L * (c7 + L * c8))))))));
}

// rates of the 33 reactions at Te (K); units m^3/s, m^6/s, 1/s
__device__ void rates_arh2(double T, double k[33]) {
    const double Tev = T / kEvK, eps = 1.5 * Tev;
    const double ie = 1.0 / eps, it = 1.0 / T, iv = 1.0 / Tev;
    const double lT = log(T), lv = log(Tev);
    k[0] = exp(-37.44 + 1.407 * log(eps) + ie * (50.34 + ie * (-348.6 - 230.5 * ie)));
    k[1] = exp(14.37 - 8.641 * log(eps) + ie * (-622.9 + ie * (5341.0 - 0.1862e5 * ie)));
    k[2] = exp(-29.7 + it * (1.39e5 + it * (-3.34e10 + it * (3.38e15 + it * (-1.85e20 + it * (5.08e24 - 5.5e28 * it))))));
    k[3] = 5.0e-16;
    k[4] = exp(-4.82e4 * it - 32.46);
    k[5] = 1.29e-16 * exp(0.7 * lT - 0.4245e5 * it);
    k[6] = 1e-13;
    k[7] = 1.14e-44;
    k[8] = 2.5e-43;
    k[9] = 6e7;
    k[10] = 5e-16;
    k[11] = 43e-18 * exp(-0.5 * lT);
    k[12] = 9.75e-21 * exp(-4.5 * lT);
    k[13] = 25.9e-12 * exp(-0.66 * lT);
    k[14] = 8.4e-14 * exp(-0.45 * lv - 11.18 * iv);
    k[15] = 1.1e-14 * exp(0.29 * lv - 15.28 * iv);
    k[16] = 2.3e-14 * exp(0.19 * lv - 17.87 * iv);
    k[17] = 9.4e-16 * exp(0.45 * lv - 29.94 * iv);
    k[18] = 1.5e-13 * exp(-1.97 * iv);
    k[19] = 2.8e-15 * exp(0.48 * lv);
    k[20] = 1.6e-15 * exp(0.48 * lv);
    k[21] = 1.4e-15 * exp(0.43 * lv);
    k[22] = 20e-16;
    k[23] = 3.086e-15 * vib(lv, -0.714, 1.389, -0.897, 0.206, -0.00126, -0.0175, 0.000166, 0.00200, -0.000311);
    k[24] = 2.66e-16 * vib(lv, -1.379, 2.630, -1.838, 0.549, -0.107, 0.0966, -0.0731, 0.0210, -0.00203);
    k[25] = 2.5e-17 * vib(lv, -1.396, 2.937, -2.573, 1.206, -0.263, -0.0185, 0.0101, 0.00147, -0.00043);
    k[26] = 1e-15;
    k[27] = 6.3e-16;
    k[28] = 21.0e-16;
    k[29] = 2.0e-16;
    k[30] = 3.7e-16;
    k[31] = 8.7e-16;
    k[32] = 0.2e-16;
}

// Net production per species for the full mechanism (rates of progress r_i
// accumulated into the 15 species) and the inelastic electron loss.
__device__ void source_arh2(const double n[15], double T, double qe, double G[15], double *loss, double *ion) {
    double k[33];
    rates_arh2(T, k);
    const double e = n[SE];
    double r[33];
    r[0] = k[0] * e * n[SAR];
    r[1] = k[1] * e * n[SAR];
    r[2] = k[2] * e * n[SARS];
    r[3] = k[3] * n[SARS] * n[SARS];
    r[4] = k[4] * n[SARS] * e;
    r[5] = k[5] * n[SAR2S] * e;
    r[6] = k[6] * n[SAR2S] * e;
    r[7] = k[7] * n[SARS] * n[SAR] * n[SAR];
    r[8] = k[8] * n[SARP] * n[SAR] * n[SAR];
    r[9] = k[9] * n[SAR2S];
    r[10] = k[10] * n[SAR2S] * n[SAR2S];
    r[11] = k[11] * n[SARP] * e;
    r[12] = k[12] * n[SARP] * e * e;
    r[13] = k[13] * n[SAR2P] * e;
    r[14] = k[14] * e * n[SH2];
    r[15] = k[15] * e * n[SH];
    r[16] = k[16] * e * n[SH2];
    r[17] = k[17] * n[SH2] * e;
    r[18] = k[18] * n[SH2P] * e;
    r[19] = k[19] * n[SH3P] * e;
    r[20] = k[20] * n[SH3P] * e;
    r[21] = k[21] * n[SH2P] * e;
    r[22] = k[22] * n[SH2P] * n[SH2];
    r[23] = k[23] * e * n[SH2];
    r[24] = k[24] * e * n[SH2];
    r[25] = k[25] * e * n[SH2];
    r[26] = k[26] * e * n[SARHP];
    r[27] = k[27] * n[SARHP] * n[SH2];
    r[28] = k[28] * n[SH2P] * n[SAR];
    r[29] = k[29] * n[SH2P] * n[SAR];
    r[30] = k[30] * n[SH3P] * n[SAR];
    r[31] = k[31] * n[SARP] * n[SH2];
    r[32] = k[32] * n[SARP] * n[SH2];
    // net production, written species by species
    G[SE] = r[1] + r[2] + r[3] + r[5] + r[10] - r[11] - r[12] - r[13] + r[15] + r[16] + r[17] - r[19] - r[20] - r[21] - r[26];
    G[SARP] = r[1] + r[2] + r[3] - r[8] - r[11] - r[12] + r[29] - r[31] - r[32];
    G[SAR2P] = r[5] + r[8] + r[10] - r[13];
    G[SHP] = r[15] + r[17] + r[18];
    G[SH2P] = r[16] - r[18] - r[21] - r[22] - r[28] - r[29] + r[32];
    G[SH3P] = -r[19] - r[20] + r[22] + r[27] - r[30];
    G[SARHP] = -r[26] - r[27] + r[28] + r[30] + r[31];
    G[SARS] = r[0] - r[2] - 2.0 * r[3] - r[4] - r[7] + r[11] + r[12] + r[13];
    G[SAR2S] = -r[5] - r[6] + r[7] - r[9] - 2.0 * r[10];
    G[SH2V1] = r[23];
    G[SH2V2] = r[24];
    G[SH2V3] = r[25];
    G[SH] = 2.0 * r[14] - r[15] + r[17] + r[18] + 3.0 * r[19] + r[20] + 2.0 * r[21] + r[22] + r[26] + r[28] + r[31];
    G[SAR] = -r[0] - r[1] + r[3] + r[4] + 2.0 * r[6] - r[7] - r[8] + 2.0 * r[9] + 2.0 * r[10] + r[13] + r[26] + r[27] - r[28]
             - r[29] - r[30] + r[32];
    G[SH2] = -r[14] - r[16] - r[17] + r[20] - r[22] - r[23] - r[24] - r[25] - r[27] + r[29] + r[30] - r[31] - r[32];
    *loss = qe * (11.6 * r[0] + 15.759 * r[1] + 4.159 * r[2] + 4.2 * r[5] + 14.68 * r[14] + 13.6 * r[15] + 15.4 * r[16] +
                  28.08 * r[17] + 12.68 * r[18]);
    *ion = r[1];
}

// Argon subset on (e, Ar+, Ar*) with background Ar: R1-R5, R12, R13.
__device__ void source_ar3(const double n[3], double T, double nAr, double qe, double G[3], double *loss, double *ion) {
    const double Tev = T / kEvK, eps = 1.5 * Tev, ie = 1.0 / eps, it = 1.0 / T, lT = log(T);
    const double e = n[0], ip = n[1], ms = n[2];
    const double k1 = exp(-37.44 + 1.407 * log(eps) + ie * (50.34 + ie * (-348.6 - 230.5 * ie)));
    const double k2 = exp(14.37 - 8.641 * log(eps) + ie * (-622.9 + ie * (5341.0 - 0.1862e5 * ie)));
    const double k3 = exp(-29.7 + it * (1.39e5 + it * (-3.34e10 + it * (3.38e15 + it * (-1.85e20 + it * (5.08e24 - 5.5e28 * it))))));
    const double k5 = exp(-4.82e4 * it - 32.46);
    const double k12 = 43e-18 * exp(-0.5 * lT), k13 = 9.75e-21 * exp(-4.5 * lT);
    const double r1 = k1 * e * nAr, r2 = k2 * e * nAr, r3 = k3 * e * ms, r4 = 5.0e-16 * ms * ms, r5 = k5 * ms * e;
    const double r12 = k12 * ip * e, r13 = k13 * ip * e * e;
    G[0] = r2 + r3 + r4 - r12 - r13;
    G[1] = r2 + r3 + r4 - r12 - r13;
    G[2] = r1 - r3 - 2.0 * r4 - r5 + r12 + r13;
    *loss = qe * (11.6 * r1 + 15.759 * r2 + 4.159 * r3);
    *ion = r2;
}

__global__ void __launch_bounds__(kBlock) k_react(ReactArgs a) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    const long N = a.ncell;
    double loss = 0.0, ion = 0.0;
    // G of species s, or its right-hand side (the drift kernel's expression
    // for a field without drift: u0/dt - 0, then + G, then + extra).  u0 is
    // read again even when it is the rate state (a cache hit): holding the
    // densities in registers until here costs occupancy
    auto put = [&](int s, double g, double) {
        if ((a.rhs_mask >> s) & 1u) {
            double v = gld(a.u0, s * N + c) * a.inv_dt - 0.0;
            v += g;
            if (a.extra) v += gld(a.extra, s * N + c);
            gst(a.rhs, s * N + c, v);
        } else {
            gst(a.G, s * N + c, g);
        }
    };
    if (a.mech == VD_MECH_ARH2_15) {
        double n[15], G[15];
        for (int s = 0; s < 15; s++) n[s] = gld(a.n, s * N + c);
        source_arh2(n, gld(a.Te, c), a.qe, G, &loss, &ion);
        for (int s = 0; s < 15; s++) put(s, G[s], n[s]);
    } else if (a.mech == VD_MECH_AR3) {
        double n[3], G[3];
        for (int s = 0; s < 3; s++) n[s] = gld(a.n, s * N + c);
        source_ar3(n, gld(a.Te, c), a.bg0, a.qe, G, &loss, &ion);
        for (int s = 0; s < 3; s++) put(s, G[s], n[s]);
    } else if (a.mech == VD_MECH_DECAY) {
        for (int s = 0; s < a.S; s++) {
            const double nv = gld(a.n, s * N + c);
            put(s, -a.bg0 * nv, nv);
        }
    } else {
        for (int s = 0; s < a.S; s++) put(s, 0.0, 0.0);
    }
    if (a.S_inel) gst(a.S_inel, c, loss);
    if (a.ion) gst(a.ion, c, ion);
}

// rho = e sum_k Z_k n_k (optionally at the mid-point (n0 + n)/2)
__global__ void __launch_bounds__(kBlock) k_rho(RhoArgs a) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    double s = 0.0;
    for (int m = 0; m < a.S; m++) s += a.Z[m] * gld(a.n, a.idx[m] * a.ncell + c);
    gst(a.rho, c, a.qe * s);
}

// Photoionization right-hand sides (Sec. 2.1, Eqs. (9)-(12)): term q gets
// coef_q S_i, coef_q = A_q p_g^2 p_q / (p + p_q) xi nu_ratio (formed on the
// host)
__global__ void __launch_bounds__(kBlock) k_photo_rhs(PhotoArgs a) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    const double si = gld(a.ion, c);
    for (int q = 0; q < a.nterm; q++) {
        gst(a.rhs, q * a.ncell + c, (a.coef[q] * si) * a.inv_scale[q]);
        if (a.ratio[q] != 1.0) gst(a.S, q * a.ncell + c, gld(a.S, q * a.ncell + c) * a.ratio[q]);
    }
}

// S_ph = sum_q S_q into the electron and ion sources
__global__ void __launch_bounds__(kBlock) k_photo_add(PhotoArgs a) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    double s = 0.0;
    for (int q = 0; q < a.nterm; q++) s += gld(a.S, q * a.ncell + c) * a.scale[q];
    gst(a.Ge, c, gld(a.Ge, c) + s);
    gst(a.Gi, c, gld(a.Gi, c) + s);
}

__global__ void __launch_bounds__(kBlock) k_photo_max(const double *__restrict__ ion, long n, double *__restrict__ partial) {
    __shared__ double red[kBlock / 64];
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double m = c < n ? fabs(gld(ion, c)) : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
        const double v = __shfl_xor(m, o, 64);
        m = v > m ? v : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int w = 1; w < kBlock / 64; w++) r = red[w] > r ? red[w] : r;
        gst(partial, (long)blockIdx.x, r);
    }
}

__global__ void __launch_bounds__(kBlock) k_photo_unscale(PhotoArgs a, double *__restrict__ out) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    for (int q = 0; q < a.nterm; q++) gst(out, q * a.ncell + c, gld(a.S, q * a.ncell + c) * a.scale[q]);
}

// One dielectric face (Sec. 2.1, Eq. (13)), one thread per face position
// (a, b) with boundary cell (i, j, k).  update 0: rho += sigma / h with
// sigma at the corrector's mid-point (sig0, or (sig0 + sigma) / 2).
// update 1: sigma = sig0 + dt sum_s q_s Gamma_s . n_hat over the species
// with a wall face there, outward wall fluxes with the wall variants.
__global__ void __launch_bounds__(kBlock) k_sigma(SigmaArgs a, int update) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.na * a.nb) return;
    const GridDev &G = a.g;
    const int pa = t % a.na, pb = t / a.na;
    const int d = a.face / 2, hi = a.face & 1;
    const int n = G.n[d];
    int i, j, k;
    if (d == 0) { i = hi ? n - 1 : 0; j = pa; k = pb; }
    else if (d == 1) { i = pa; j = hi ? n - 1 : 0; k = pb; }
    else { i = pa; j = pb; k = hi ? n - 1 : 0; }
    const long cb = i + (long)G.n[0] * j + (long)G.nxy * k;
    const long q = a.off + t;
    if (!update) {
        const double sg = a.mid ? 0.5 * (gld(a.sig0, q) + gld(a.sigma, q)) : gld(a.sig0, q);
        gst(a.rho, cb, gld(a.rho, cb) + sg / a.h);
        return;
    }
    const int pos = d == 0 ? i : (d == 1 ? j : k);
    const double Ef = e_face(G, a.phi, d, (int)cb, pos, hi ? n : 0);
    const double e_n = hi ? Ef : -Ef;
    const double te = gld(a.Te, cb);
    double sum = 0.0;
    for (int s = 0; s < a.S; s++) {
        const FieldDesc &F = a.f[s];
        if (F.kind[a.face] != VD_BC_WALLFLUX) continue;
        const double fl = wall_flux_f(F, cb, gld(F.u, cb), F.mu ? gld(F.mu, cb) : F.mu_c, e_n, te, a.Tg, a.kB, a.me);
        sum += a.Z[s] * a.qe * fl;
    }
    gst(a.sigma, q, gld(a.sig0, q) + a.dt * sum);
}

// Time-step limits of Eq. (20) per cell, least over each workgroup
__global__ void __launch_bounds__(kBlock) k_dt_limit(DtArgs a) {
    __shared__ double red[kBlock / 64];
    const GridDev &G = a.g;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    double dt = a.dt_max;
    if (c < G.ncell && !(G.mask && !gld(G.mask, (long)c))) {     // masked step: valid cells only
        int pos[3];
        pos[2] = c / G.nxy;
        const int r = c - pos[2] * G.nxy;
        pos[1] = r / G.n[0];
        pos[0] = r - pos[1] * G.n[0];
        double E[3];
        e_cell(G, a.phi, c, pos, E);
        const double Em = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
        double mu = a.mu_c, D = a.D_c;
        if (a.fit) {
            mu = mu_electron(Em / a.N_gas / kTd, a.N_gas);
            D = mu * a.kB * gld(a.Te, c) / a.qe;
        }
        const double am = fabs(mu) * Em;
        if (am > 0.0) { const double t = a.c_adv * a.dxmin / am; dt = t < dt ? t : dt; }
        if (D > 0.0) { const double t = a.c_diff / 3.0 * (a.dxmin * a.dxmin) / (2.0 * D); dt = t < dt ? t : dt; }
        const double bm = a.qe * fabs(mu) * gld(a.ne, c);
        if (bm > 0.0) { const double t = a.c_diel * a.eps0 / bm; dt = t < dt ? t : dt; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double v = __shfl_xor(dt, o, 64);
        dt = v < dt ? v : dt;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dt;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kBlock / 64; w++) m = red[w] < m ? red[w] : m;
        gst(a.partial, blockIdx.x, m);
    }
}

// u* = (u0 + u)/2 (mid-point of the corrector iteration)
__global__ void __launch_bounds__(kBlock) k_mid(const double *__restrict__ u0, const double *__restrict__ u, double *__restrict__ out, long n) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) gst(out, c, 0.5 * (gld(u0, c) + gld(u, c)));
}

// Poisson guess extrapolated in time from the potentials passed in by
// earlier steps: a = phi on entry, h1 the previous step's, h2 the one
// before (held in hdst).  order 1: 2a - h1; order 2: 3a - 3h1 + h2, every
// product and sum a statement of its own (rounded separately, no fused
// multiply-add); order 0 leaves phi.  a is then kept in hdst, which becomes
// the newest history slot.
__global__ void __launch_bounds__(kBlock) k_extrap(double *__restrict__ phi, const double *__restrict__ h1,
                                                   double *__restrict__ hdst, int order, long n) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double a = gld(phi, c);
    if (order == 1) {
        const double t = 2.0 * a;
        const double g = t - gld(h1, c);
        gst(phi, c, g);
    } else if (order == 2) {
        const double t0 = 3.0 * a;
        const double t1 = 3.0 * gld(h1, c);
        const double t2 = t0 - t1;
        const double g = t2 + gld(hdst, c);
        gst(phi, c, g);
    }
    gst(hdst, c, a);
}

// Species guesses extrapolated in time, one species per blockIdx.y, with
// the history in FP32 (its rounding, ~1e-7 of n, is far below what the
// guess needs): a = n on entry, h1 the previous step's n, h2 the one before
// (held in hd).  order 1: n <- 2a - h1; order 2: n <- 3a - 3h1 + h2, every
// product and sum a statement of its own; order 0 leaves n.  hd <- (float)a.
__global__ void __launch_bounds__(kBlock) k_extrap_species(ExtrapSet e, int order, long n) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double *__restrict__ x = e.x[blockIdx.y];
    const float *__restrict__ h1 = e.h1[blockIdx.y];
    float *__restrict__ hd = e.hd[blockIdx.y];
    const double a = gld(x, c);
    if (order == 1) {
        const double t = 2.0 * a;
        const double g = t - (double)gld(h1, c);
        gst(x, c, g);
    } else if (order == 2) {
        const double t0 = 3.0 * a;
        const double t1 = 3.0 * (double)gld(h1, c);
        const double t2 = t0 - t1;
        const double g = t2 + (double)gld(hd, c);
        gst(x, c, g);
    }
    gst(hd, c, (float)a);
}

// ------------------------------------------------------ electron energy
// Central diffusive flux along +d at face fidx: -beta_f (u_R - u_L)/h with
// the harmonic-mean face coefficient; Dirichlet face: one-sided over half a
// cell with the boundary cell's coefficient; Neumann and wall: 0.
__device__ __forceinline__ double diff_face(const GridDev &G, const int *kind, const double *gval, const double *__restrict__ u,
                                            const double *__restrict__ D, double D_c, int d, int c, int pos, int fidx) {
    const int n = G.n[d];
    const long st = G.stride[d];
    const double ih = G.ih[d];
    const long c0 = c - (long)pos * st;
#define DV(q) (D ? gld(D, c0 + (long)(q) * st) : D_c)
    if (fidx > 0 && fidx < n) {
        if (G.mask) {
            // masked step: a covered-valid face is a homogeneous Dirichlet
            // face of the valid cell (one-sided over half a cell)
            const bool vl = gld(G.mask, c0 + (fidx - 1) * st) != 0, vr = gld(G.mask, c0 + fidx * st) != 0;
            if (!vl && !vr) return 0.0;
            if (!vr) return -DV(fidx - 1) * (0.0 - gld(u, c0 + (fidx - 1) * st)) * (2.0 * ih);
            if (!vl) return -DV(fidx) * (gld(u, c0 + fidx * st) - 0.0) * (2.0 * ih);
        }
        const double a = DV(fidx - 1), b = DV(fidx);
        const double hm = (a + b == 0.0) ? 0.0 : 2.0 * a * b / (a + b);
        return -hm * (gld(u, c0 + fidx * st) - gld(u, c0 + (fidx - 1) * st)) * ih;
    }
    const int f = 2 * d + (fidx == 0 ? 0 : 1);
    const int kd = kind[f];
    if (kd == VD_BC_PERIODIC) {
        const double a = DV(n - 1), b = DV(0);
        const double hm = (a + b == 0.0) ? 0.0 : 2.0 * a * b / (a + b);
        return -hm * (gld(u, c0) - gld(u, c0 + (n - 1) * st)) * ih;
    }
    if (kd == VD_BC_DIRICHLET) {
        const double g = gval[f];
        if (fidx == 0) return -DV(0) * (gld(u, c0) - g) * (2.0 * ih);
        return -DV(n - 1) * (g - gld(u, c0 + (n - 1) * st)) * (2.0 * ih);
    }
    return 0.0;
#undef DV
}

// Electron-energy right-hand side (Eqs. (5)-(8)) at u*:
//   Ee0/dt - div(5/3 mu_e Ee* E)_WENO + Joule - elastic - inelastic + extra,
// Joule = -e Gamma_e . E at the cell with Gamma_e per direction the mean of
// the two face fluxes (WENO drift + central diffusion, wall faces carrying
// the electron wall flux); elastic = 1.5 ne kB (Te - Tg)(2 me/mb) e/(me|mu_e|).
__global__ void __launch_bounds__(kBlock) k_energy_rhs(EnergyArgs a) {
    const GridDev &G = a.g;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= G.ncell) return;
    int pos[3];
    pos[2] = c / G.nxy;
    int r = c - pos[2] * G.nxy;
    pos[1] = r / G.n[0];
    pos[0] = r - pos[1] * G.n[0];
    const double divE = drift_div_cell(G, a.fE, a.phi, a.Te, a.Tg, a.kB, a.me, c, pos);
    const FieldDesc &Fe = a.fe;
    double gam[3];
    for (int d = 0; d < 3; d++) {
        const int n = G.n[d];
        double Fs[2];
        for (int side = 0; side < 2; side++) {
            const int fidx = pos[d] + side;
            const bool boundary = (fidx == 0 || fidx == n);
            const int kd = Fe.kind[2 * d + side];
            if (boundary && kd == VD_BC_NEUMANN) { Fs[side] = 0.0; continue; }
            if (boundary && kd == VD_BC_WALLFLUX) {
                const double Ef = e_face(G, a.phi, d, c, pos[d], fidx);
                const double fl = wall_flux_f(Fe, c, gld(Fe.u, c), 0.0, fidx == 0 ? -Ef : Ef, gld(a.Te, c), a.Tg, a.kB, a.me);
                Fs[side] = fidx == 0 ? -fl : fl;
                continue;
            }
            Fs[side] = face_drift(G, Fe, a.phi, d, c, pos[d], fidx) +
                       diff_face(G, Fe.kind, Fe.gval, Fe.u, a.De, a.De_c, d, c, pos[d], fidx);
        }
        gam[d] = 0.5 * (Fs[0] + Fs[1]);
    }
    double E[3];
    e_cell(G, a.phi, c, pos, E);
    const double joule = -a.qe * (gam[0] * E[0] + gam[1] * E[1] + gam[2] * E[2]);
    const double mue = Fe.mu ? gld(Fe.mu, c) : Fe.mu_c;
    const double nu = a.qe / (a.me * fabs(mue));
    const double ne = gld(Fe.u, c);
    const double elastic = 1.5 * ne * a.kB * (gld(a.Te, c) - a.Tg) * (2.0 * a.me / a.m_bg) * nu;
    double src = joule - elastic - gld(a.S_inel, c);
    if (a.extra) src += gld(a.extra, c);
    gst(a.out, c, gld(a.Ee0, c) * a.inv_dt - divE + src);
}

// ------------------------------------------------------ face fluxes
// Total flux along +d through every face of one field: the drift part of
// face_flux (upwind WENO5, the wall flux at a wall face, nothing at a
// Neumann face) plus the central diffusive part of diff_face.  One thread
// per face; face arrays x ((nx+1) ny nz), then y (nx (ny+1) nz), then z
// (nx ny (nz+1)).
__global__ void __launch_bounds__(kBlock) k_face_flux(DriftArgs a, const double *__restrict__ D, double *__restrict__ out) {
    const GridDev &G = a.g;
    const FieldDesc &F = a.f[0];
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const long nfx = (long)(nx + 1) * ny * nz, nfy = (long)nx * (ny + 1) * nz, nfz = (long)nx * ny * (nz + 1);
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nfx + nfy + nfz) return;
    const long slot = q;
    int d, i, j, k;
    if (q < nfx) {
        d = 0; i = (int)(q % (nx + 1)); q /= nx + 1; j = (int)(q % ny); k = (int)(q / ny);
    } else if ((q -= nfx) < nfy) {
        d = 1; i = (int)(q % nx); q /= nx; j = (int)(q % (ny + 1)); k = (int)(q / (ny + 1));
    } else {
        q -= nfy;
        d = 2; i = (int)(q % nx); q /= nx; j = (int)(q % ny); k = (int)(q / ny);
    }
    const int fidx = d == 0 ? i : (d == 1 ? j : k);
    // start of the row through the face along d
    const long c0 = (d == 0 ? 0 : i) + (long)nx * (d == 1 ? 0 : j) + (long)G.nxy * (d == 2 ? 0 : k);
    const double drift = face_flux(G, F, a.phi, a.Te, a.Tg, a.kB, a.me, d, c0, fidx);
    const double diff = diff_face(G, F.kind, F.gval, F.u, D, 0.0, d, (int)c0, 0, fidx);
    gst(out, slot, drift + diff);
}

// ----------------------------------------------------- host launchers
void launch_transport(vd_ctx *ctx, const TransportArgs &a) {
    // phi read, Te written (table or energy mode), mu and D written per field-dependent species
    double bytes = (double)a.g.ncell * (8.0 + (a.te_mode != VD_TE_FIXED ? 8.0 : 8.0) + 16.0 * a.nvar + (a.beta_e ? 8.0 : 0.0) +
                                        (a.te_mode == VD_TE_ENERGY ? 16.0 : 0.0));
    timed(ctx, "transport", bytes, [&] {
        k_transport<<<ceil_div(a.g.ncell, kBlock), kBlock, 0, ctx->stream>>>(a);
    });
}

// the grids whose unmasked drift runs in k_drift25, with the wall-face
// fluxes added by k_wall_div (the other kernels fold them into each cell's
// divergence)
bool drift25_path(const GridDev &g) {
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    return !g.mask && nx % kDX == 0 && ny % kDY == 0 && nz % 8 == 0 && nx >= 3 && ny >= 3 && nz >= 3;
}

void launch_drift(vd_ctx *ctx, DriftArgs a, const FieldDesc *fields, int nfields, const char *tag) {
    if (nfields == 0) return;
    if (a.g.mask && a.near) {
        // masked step: the unmasked kernels over every cell, then the cells
        // whose stencils reach a covered cell again with the mask
        DriftArgs au = a;
        au.g.mask = nullptr;
        au.near = nullptr;
        launch_drift(ctx, au, fields, nfields, tag);
        dim3 grid(ceil_div(a.g.ncell, kBlock), nfields);
        a.f = (const FieldDesc *)upload_blob(ctx, std::string("fields:") + tag, fields, sizeof(FieldDesc) * nfields);
        timed(ctx, "weno", 0.0, [&] { k_drift_fix<<<grid, kBlock, 0, ctx->stream>>>(a); });
        VD_HIP(hipGetLastError());
        return;
    }
    VD_CHECK(nfields <= kMaxFields, "too many fields");
    a.f = (const FieldDesc *)upload_blob(ctx, std::string("fields:") + tag, fields, sizeof(FieldDesc) * nfields);
    dim3 grid(ceil_div(a.g.ncell, kBlock), nfields);
    // per field: u read, mobility read when per cell, output written, and in
    // right-hand-side mode the chemical source (and extra source, and u0 when
    // it is not u) read; phi read once for all fields
    double bytes = 8.0 * a.g.ncell;
    for (int f = 0; f < nfields; f++) {
        const FieldDesc &F = fields[f];
        if (F.rhs_done) continue;
        double per = 16.0 + (F.mu ? 8.0 : 0.0);
        if (a.mode == 1) per += (F.src ? 8.0 : 0.0) + (F.extra ? 8.0 : 0.0) + (F.u0 != F.u ? 8.0 : 0.0);
        bytes += per * a.g.ncell;
    }
    const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
    // planes per workgroup: the deepest of 32, 16, 8 that divides nz and
    // still gives 2048 workgroups (else the shallowest that divides nz)
    int kz = 0;
    for (int cand : {32, 16, 8}) {
        if (nz % cand) continue;
        kz = cand;
        if ((long)(nx / kDX) * (ny / kDY) * (nz / cand) * nfields >= 2048) break;
    }
    if (a.g.mask) {
        // masked step: the per-cell kernel (its face fluxes close the valid runs)
        timed(ctx, "weno", bytes, [&] { k_drift<<<grid, kBlock, 0, ctx->stream>>>(a); });
    } else if (nx % kDX == 0 && ny % kDY == 0 && kz > 0 && nx >= 3 && ny >= 3 && nz >= 3) {
        dim3 tg((nx / kDX) * (ny / kDY) * (nz / kz), nfields);
        timed(ctx, "weno", bytes, [&] {
            k_drift25<<<tg, kBlock, 0, ctx->stream>>>(a, kz);
            // wall fluxes of the boundary cells, one direction per launch
            bool any[3] = {false, false, false};
            for (int f = 0; f < nfields; f++)
                for (int s2 = 0; s2 < 6; s2++) any[s2 / 2] = any[s2 / 2] || fields[f].kind[s2] == VD_BC_WALLFLUX;
            for (int d = 0; d < 3; d++) {
                if (!any[d]) continue;
                const long nl = (long)a.g.ncell / a.g.n[d];
                k_wall_div<<<dim3(ceil_div(nl, kBlock), nfields), kBlock, 0, ctx->stream>>>(a, d);
            }
        });
    } else if (nx % kTX == 0 && ny % kTY == 0 && kz > 0) {
        dim3 tg((nx / kTX) * (ny / kTY) * (nz / kz), nfields);
        timed(ctx, "weno", bytes, [&] { k_drift_tiled<<<tg, kBlock, 0, ctx->stream>>>(a, kz); });
    } else {
        timed(ctx, "weno", bytes, [&] { k_drift<<<grid, kBlock, 0, ctx->stream>>>(a); });
    }
}

// masked step, Poisson: each covered neighbour of a valid cell is a
// Dirichlet face with the covered cell's potential g; rho gains
// 2 beta_f g / h^2 with beta_f the operator's face coefficient (the harmonic
// mean of the two cells' permittivities, or eps0), faces in the order x-,
// x+, y-, y+, z-, z+
__device__ __forceinline__ double hmean(double a, double b) { return (a + b == 0.0) ? 0.0 : 2.0 * a * b / (a + b); }

__global__ void __launch_bounds__(kBlock) k_mask_lift(GridDev G, const double *__restrict__ phi_cov,
                                                      const double *__restrict__ eps, double eps0, double *__restrict__ rho) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= G.ncell || !gld(G.mask, (long)c)) return;
    int pos[3];
    pos[2] = c / G.nxy;
    const int r = c - pos[2] * G.nxy;
    pos[1] = r / G.n[0];
    pos[0] = r - pos[1] * G.n[0];
    double lift = 0.0;
#pragma unroll
    for (int f = 0; f < 6; f++) {
        const int d = f >> 1;
        const int p = pos[d] + ((f & 1) ? 1 : -1);
        if (p < 0 || p >= G.n[d]) continue;
        const long nb = c + ((f & 1) ? G.stride[d] : -G.stride[d]);
        if (gld(G.mask, nb)) continue;
        const double bf = eps ? hmean(gld(eps, (long)c), gld(eps, nb)) : eps0;
        lift += 2.0 * bf * gld(phi_cov, nb) * (G.ih[d] * G.ih[d]);
    }
    gst(rho, (long)c, gld(rho, (long)c) + lift);
}

__global__ void __launch_bounds__(kBlock) k_mask_restore(GridDev G, const double *__restrict__ phi_cov, double *__restrict__ phi) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= G.ncell || gld(G.mask, (long)c)) return;
    gst(phi, (long)c, gld(phi_cov, (long)c));
}

void launch_mask_lift(vd_ctx *ctx, const GridDev &G, const double *phi_cov, const double *eps, double eps0, double *rho) {
    k_mask_lift<<<ceil_div(G.ncell, kBlock), kBlock, 0, ctx->stream>>>(G, phi_cov, eps, eps0, rho);
    VD_HIP(hipGetLastError());
}

void launch_mask_restore(vd_ctx *ctx, const GridDev &G, const double *phi_cov, double *phi) {
    k_mask_restore<<<ceil_div(G.ncell, kBlock), kBlock, 0, ctx->stream>>>(G, phi_cov, phi);
    VD_HIP(hipGetLastError());
}

void launch_react(vd_ctx *ctx, const ReactArgs &a) {
    timed(ctx, "react", (double)a.ncell * 8.0 * (2.0 * a.S + 1.0 + (a.S_inel ? 1.0 : 0.0)), [&] {
        k_react<<<ceil_div(a.ncell, kBlock), kBlock, 0, ctx->stream>>>(a);
    });
}

void launch_rho(vd_ctx *ctx, const RhoArgs &a) {
    timed(ctx, "rho", (double)a.ncell * 8.0 * (a.S + 1.0), [&] { k_rho<<<ceil_div(a.ncell, kBlock), kBlock, 0, ctx->stream>>>(a); });
}

void launch_energy(vd_ctx *ctx, const EnergyArgs &a) {
    timed(ctx, "energy", (double)a.g.ncell, [&] { k_energy_rhs<<<ceil_div(a.g.ncell, kBlock), kBlock, 0, ctx->stream>>>(a); });
}

void launch_photo_rhs(vd_ctx *ctx, const PhotoArgs &a) {
    timed(ctx, "photo", (double)a.ncell * 8.0 * (1 + a.nterm), [&] {
        k_photo_rhs<<<ceil_div(a.ncell, kBlock), kBlock, 0, ctx->stream>>>(a);
    });
}

int launch_photo_max(vd_ctx *ctx, const double *ion, long ncell, double *partial) {
    const int nb = ceil_div(ncell, kBlock);
    k_photo_max<<<nb, kBlock, 0, ctx->stream>>>(ion, ncell, partial);
    VD_HIP(hipGetLastError());
    return nb;
}

void launch_photo_unscale(vd_ctx *ctx, const PhotoArgs &a, double *out) {
    k_photo_unscale<<<ceil_div(a.ncell, kBlock), kBlock, 0, ctx->stream>>>(a, out);
    VD_HIP(hipGetLastError());
}

void launch_photo_add(vd_ctx *ctx, const PhotoArgs &a) {
    timed(ctx, "photo", (double)a.ncell * 8.0 * (a.nterm + 4), [&] {
        k_photo_add<<<ceil_div(a.ncell, kBlock), kBlock, 0, ctx->stream>>>(a);
    });
}

void launch_sigma(vd_ctx *ctx, const SigmaArgs &a, int update) {
    const long n = (long)a.na * a.nb;
    timed(ctx, "sigma", 0.0, [&] { k_sigma<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(a, update); });
}

int launch_dt_limit(vd_ctx *ctx, const DtArgs &a) {
    const int nb = (int)ceil_div(a.g.ncell, kBlock);
    timed(ctx, "dt", (double)a.g.ncell * 24.0, [&] { k_dt_limit<<<nb, kBlock, 0, ctx->stream>>>(a); });
    return nb;
}

void launch_extrap(vd_ctx *ctx, double *phi, const double *h1, double *hdst, int order, long n) {
    const double bytes = (double)n * (order == 0 ? 16.0 : (order == 1 ? 32.0 : 40.0));
    timed(ctx, "guess", bytes, [&] { k_extrap<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(phi, h1, hdst, order, n); });
}

void launch_extrap_species(vd_ctx *ctx, const ExtrapSet &e, int count, int order, long n) {
    if (count == 0) return;
    const double bytes = (double)n * count * (order == 0 ? 12.0 : (order == 1 ? 24.0 : 28.0));
    timed(ctx, "guess", bytes, [&] {
        k_extrap_species<<<dim3(ceil_div(n, kBlock), count), kBlock, 0, ctx->stream>>>(e, order, n);
    });
}

void launch_mid(vd_ctx *ctx, const double *u0, const double *u, double *out, long n) {
    timed(ctx, "mid", (double)n * 24.0, [&] { k_mid<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(u0, u, out, n); });
}

void launch_face_flux(vd_ctx *ctx, DriftArgs a, const FieldDesc &field, const double *D, double *out) {
    a.f = (const FieldDesc *)upload_blob(ctx, "fields:faces", &field, sizeof(FieldDesc));
    const long nf = (long)(a.g.n[0] + 1) * a.g.n[1] * a.g.n[2] + (long)a.g.n[0] * (a.g.n[1] + 1) * a.g.n[2] +
                    (long)a.g.n[0] * a.g.n[1] * (a.g.n[2] + 1);
    timed(ctx, "faces", 8.0 * (4.0 * a.g.ncell + nf), [&] {
        k_face_flux<<<ceil_div(nf, kBlock), kBlock, 0, ctx->stream>>>(a, D, out);
    });
}

GridDev make_grid(const vd_grid &g, const vd_bc &phi_bc) {
    GridDev G;
    memset(&G, 0, sizeof(G));
    G.n[0] = g.nx; G.n[1] = g.ny; G.n[2] = g.nz;
    G.nxy = g.nx * g.ny;
    G.ncell = g.nx * g.ny * g.nz;
    G.stride[0] = 1; G.stride[1] = g.nx; G.stride[2] = (long)g.nx * g.ny;
    G.ih[0] = 1.0 / g.dx; G.ih[1] = 1.0 / g.dy; G.ih[2] = 1.0 / g.dz;
    G.ihl[0] = 1.0 / g.dx; G.ihl[1] = 1.0 / g.dy; G.ihl[2] = 1.0 / g.dz;
    for (int f = 0; f < 6; f++) { G.phi_kind[f] = phi_bc.kind[f]; G.phi_val[f] = phi_bc.value[f]; }
    return G;
}

}  // namespace vd
