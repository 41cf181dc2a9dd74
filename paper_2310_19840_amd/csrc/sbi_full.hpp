// sbi_full.hpp -- operands and launchers of the fully nonlinear W solve
// (sbi_full.hip), kept apart from the iteration's kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "sbi_internal.hpp"

namespace sbi {

// Fully nonlinear W solve of one-dimensional grids (sbi_full.hip): the
// operands of its kernels.  Physical fields are [batch][n] with member
// stride s_phys; FP64 tables: c0 [batch][n] (S0^-1 circulant per member), d1,
// d2, s2, s2a, rs2 [n]; FP64 part [slices][batch][n] holds the slices of a pair pass (then of the apply) and
// rhs [batch][n] the right-hand side.  Members whose bed is kept as a boundary
// of its own (bed[m] = 1: a variable bed not too deep to matter) use the
// two-boundary form: bed geometry bz, bx, bxx, the circulant cm of
// S0^-1 (S0 - S_flat), the bed right-hand side rb = -D_BS[phi_s] and the bed
// potential phi_b of the sweeps in pbuf (all FP64 [batch][n]).
struct FullParams {
    int n, batch, nsplit;
    double lx;
    long long s_phys;
    const double* href;   // [batch] depth of each member's flat bed
    const void* eta;      // physical eta
    const void* phi;      // physical phi_s
    void* ex;             // eta_x
    void* exx;            // eta_xx
    void* rhs;            // pi phi_s + D[phi_s] (FP64, [batch][n])
    void* part;           // pair-pass slices, then the apply's source slices
    void* c0;
    void* d1;
    void* d2;
    void* s2;
    void* s2a;            // [n] sin(2 pi j / n) of each index distance
    void* rs2;            // [n] 1 / sin^2(pi j / n) (0 at j = 0)
    void* lfl;            // [batch][n] the flat image's single-layer term per member
    void* w;              // FP64 [batch][n]: rhs - (S - S0)[V_n]
    const void* vin;      // V_n (null: V_0 = 0)
    void* vout;           // V_(n+1)
    const void* vbuf[2];  // the two iterate buffers (V_s is in vbuf[s & 1])
    void* vfinal;         // the decided iterate of each member
    Ctl* ctl;
    int sweep, max_sweeps;
    double tol;
    const int* bed;       // [batch] 1: two-boundary form (null: no member)
    void* bz;
    void* bx;
    void* bxx;
    void* cm;
    void* rb;
    const void* pbin;     // phi_b of this sweep (null: phi_b = 0)
    void* pbout;          // phi_b of the next sweep
    int nsym;             // slices of the symmetric single-layer pass (FULL_SYM; 0: FULL_SINGLE ran)
};
enum {
    FULL_TABLES = 0, FULL_GEOM, FULL_DOUBLE, FULL_RHS, FULL_SINGLE, FULL_COMBINE, FULL_APPLY, FULL_SELECT,
    FULL_BEDGEOM, FULL_RHSB, FULL_RB, FULL_BED, FULL_PB, FULL_SURF, FULL_SYM
};
constexpr int kFullSymTile = 128;  // tile edge of FULL_SYM (n / kFullSymTile slices)

template <typename R> hipError_t launch_full_t(const FullParams&, int what, hipStream_t);
hipError_t launch_full(int fp64, const FullParams& p, int what, hipStream_t s);

}  // namespace sbi
