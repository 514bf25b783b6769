// Internal interface between the C ABI and the templated gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_tables.h"

namespace dgmhd {

// Device-resident scalars of a step: written by reductions and the
// finalisation kernel, read by every stage kernel (no host round trip).
struct Scal {
  double dt, ch, kappa, t;
  double last_maxsig;                    // max_K sum_a(|v_a|+c)/D of the last reduction
  unsigned long long maxrate_bits;       // max_K s_K / h_K (bit pattern of a non-negative double)
  unsigned long long maxsig_bits;        // max_K s_K
  unsigned long long powell_rate_bits;   // max_K |divB|_K |v.B| / E (Powell cap)
  unsigned long long n_ch_violation;     // fixed c_h below twice the max signal
  unsigned long long nonfinite;          // non-finite values met by a reduction
  // limiter statistics (accumulated, reset by the host)
  unsigned long long n_tvb, n_pos, n_floor, n_mlp, n_fallback;
  double inj_mass, inj_energy;
  unsigned int tally_flag;               // some cell's floor slots hold a value (k_tally_reduce)
  unsigned long long n_record_stage;     // stages recorded for the learned indicator
  // the next step's max signal and rate, folded into the last stage's
  // positivity limiter (bit patterns of non-negative doubles)
  unsigned long long next_maxsig_bits, next_maxrate_bits;
  // workgroups of a time-step reduction that finalises the step itself
  // (the last one computes dt, c_h and kappa); 0 between launches
  unsigned int blocks_done;
};

// What the time-step finalisation needs besides the scheme parameters.
struct DtFinalize {
  int D, d, divb;
  double hmin;
};

struct Grid {
  int n0, n1, n2;   // cells per axis (n2 = 1 in 2-D)
  int64_t C;        // number of cells
  int64_t ld;       // leading dimension of state arrays
  double h;         // cell size (uniform grids)
  // octree meshes (level == nullptr on uniform grids)
  const int8_t* level;     // [C] refinement level of each leaf
  double hbase;            // level-0 cell size
  const int32_t* faceL;    // [NF] left cell of each face (faces sorted by axis)
  const int32_t* faceR;    // [NF] right cell
  const int8_t* subL;      // [NF] quarter of the left cell's +a face (-1: full face)
  const int8_t* subR;      // [NF] quarter of the right cell's -a face (-1: full face)
  const int32_t* slots;    // [C][D][2][4] faces touching each cell side (side 1: +a), -1 = none
  int64_t NF, ldf;         // number of faces, leading dimension of face arrays
  int64_t face0[4];        // first face of each axis; face0[D] = NF
  // faces grouped by class (axis, left sub-face, right sub-face) into tiles of
  // 16 for the matrix-core face kernel: ftile[2t] = class, ftile[2t+1] =
  // offset of the tile's 16 entries in fperm (face indices, -1 = padding)
  const int32_t* ftile;
  const int32_t* fperm;
  int64_t nftile;
};

struct SchemeParams {
  double gamma, cfl, cfl_glm, glm_cr, glm_ch_fixed, powell_eta;
  double tvb_Mtilde, tvb_beta, tvb_eps, eps_rho, eps_p;
  int limiter;
  int powell_q;  // Powell q-dagger: 0 cell mean (eq. powellq-average), 1 interpolated (eq. powellq-interp)
  // learned indicator (device pointers, null until installed)
  double mlp_lo, mlp_hi;
  const uint16_t* mlp_Pb;
  const float* mlp_P;
  const double* mlp_sigma;
};

// Per-configuration launcher; one instance per handle.
struct Launcher {
  virtual ~Launcher() {}
  virtual hipError_t upload_tables(const Tables& t) = 0;
  virtual void free_tables() = 0;
  virtual size_t face_buffer_elems(const Grid& g) const = 0;
  virtual size_t jump_buffer_elems(const Grid& g, int powell_q) const = 0;
  // face fluxes of state w into ff (and Powell jumps into jp).  cap false:
  // the caller does not take the Powell cap from this launch's jumps, so a
  // face kernel that hands the cell kernels jump moments in ff may skip the
  // jump points
  virtual void face(const void* w, void* ff, void* jp, const Grid& g, const Scal* sc, const SchemeParams& sp,
                    hipStream_t s, bool cap = true) = 0;
  // mode 0: out = M^-1 R;  mode 1: out = a0 w0 + b0 (w + cdt dt M^-1 R)
  virtual void cell(const void* w, const void* w0, void* out, const void* ff, const void* jp, const Grid& g,
                    const Scal* sc, const SchemeParams& sp, double a0, double b0, double cdt, int mode,
                    hipStream_t s) = 0;
  // tile-shape variants of the cell kernel (autotuner)
  virtual int cell_variant_count() const = 0;
  virtual bool cell_variant_valid(int v) const = 0;
  virtual void set_cell_variant(int v) = 0;
  virtual int get_cell_variant() const = 0;
  // cell variant cv and face variant fv exchange the same face-flux layout on g
  virtual bool layout_compatible(int cv, int fv, const Grid& g) const = 0;
  virtual int face_variant_count() const = 0;
  virtual void set_face_variant(int v) = 0;
  virtual int get_face_variant() const = 0;
  // per-cell signal speeds -> atomic maxima in sc.  With fin, a launch that
  // can also finalises the step (dt, c_h, kappa from the maxima, which it
  // then clears) and returns true; the caller launches the finalisation
  // otherwise.
  virtual bool maxsig(const void* w, const Grid& g, Scal* sc, const SchemeParams& sp, hipStream_t s,
                      const DtFinalize* fin = nullptr) = 0;
  // maxsig(..., fin) finalises on g (so the maxima are clear after it)
  virtual bool maxsig_finalizes(const Grid& g) const = 0;
  // Powell dt cap: per-face normal-field jumps then per-cell rate
  // Powell cap from the normal-field jumps the face kernel wrote for w
  virtual void powell_cap_jp(const void* w, const void* jp, void* jsum, const Grid& g, Scal* sc, hipStream_t s) = 0;
  virtual void powell_cap(const void* w, void* jsum, const Grid& g, Scal* sc, const SchemeParams& sp,
                          hipStream_t s) = 0;
  // dynamic refinement (Sec. 4.4), Legendre bases: largest smoothness
  // indicator over the fields in the bit mask and the directions, per leaf
  // (S) or per sibling group restricted to its parent (groups[g][2^D] leaf
  // indices in octant order); transfer of the weights to a new leaf set
  // (map[i] = kind (0 copy, 1 prolongation, 2 restriction), source (leaf, or
  // group row of kids), depth, octant path 3 bits per level from the top)
  virtual void amr_smooth(const void* w, const Grid& g, uint32_t fields, double* S, hipStream_t s) = 0;
  virtual void amr_parent_smooth(const void* w, const Grid& g, uint32_t fields, const int32_t* groups,
                                 int64_t ngroups, double* Sp, hipStream_t s) = 0;
  virtual void amr_transfer(const void* w_old, int64_t ld_old, void* w_new, int64_t ld_new, const int32_t* map,
                            const int32_t* kids, int64_t nnew, hipStream_t s) = 0;
  // conserved state at the points of the projection rule: out[var][point][cell - cell0]
  virtual void nodal(const void* w, int64_t cell0, int64_t ncell, double* out, const Grid& g, hipStream_t s) = 0;
  virtual void project(const double* prim, int64_t cell0, int64_t ncell, void* w, const Grid& g,
                       const SchemeParams& sp, hipStream_t s) = 0;
  // limiters in place
  // next_sig: also reduce the max signal speed of the limited state into the
  // next step's slots (only where fused_signal() is true)
  virtual void limit(void* w, void* scratch, const Grid& g, Scal* sc, const SchemeParams& sp, hipStream_t s,
                     bool next_sig = false) = 0;
  virtual bool fused_signal(const Grid& g, const SchemeParams& sp) const = 0;
  virtual size_t limit_scratch_bytes(const Grid& g) const = 0;
  // learned indicator helpers (GLM only; return false when not built)
  virtual bool mlp_features(const void* w, uint16_t* X, const double* sigma, const Grid& g, hipStream_t s) = 0;
  virtual bool mlp_labels(const void* w, float* y, const Grid& g, Scal* sc, const SchemeParams& sp,
                          hipStream_t s) = 0;
  virtual bool mlp_scale(const void* w, double* part, double* sigma, const Grid& g, hipStream_t s) = 0;
  virtual bool mlp_record(const void* w, uint16_t* X, float* y, unsigned long long* counter, int64_t cap, double qpos,
                          double qneg, unsigned long long seed, const Grid& g, Scal* sc, const SchemeParams& sp,
                          hipStream_t s) = 0;
  virtual int nmodes() const = 0;
};

Launcher* make_launcher(int precision, int D, int d, int divb);

// scalar kernels
void launch_reset_step(Scal* sc, hipStream_t s);
void launch_reset_next(Scal* sc, hipStream_t s);  // clears the next step's signal slots
void launch_take_next(Scal* sc, hipStream_t s);   // moves them into this step's reduction
void launch_finalize_dt(Scal* sc, const SchemeParams& sp, int D, int d, int divb, double hmin, hipStream_t s);
void launch_set_scalars(Scal* sc, double ch, double kappa, double dt, hipStream_t s);
// out = c[0] x[0] + c[1] x[1] + c[2] x[2] + c[3] x[3] (FP64 arithmetic) over
// nmodes rows of ld elements, C columns used; x[k] may be null when c[k] = 0
// and out may alias any x[k]
void launch_lincomb(void* out, const void* const x[4], const double c[4], size_t elem, int64_t nmodes, int64_t ld,
                    int64_t C, hipStream_t s);
void launch_set_time(Scal* sc, double t, hipStream_t s);
void launch_reset_stats(Scal* sc, hipStream_t s);  // limiter tallies, non-finite and c_h-violation counts
// flags any non-finite weight of w (nmodes rows of ld, C columns used)
void launch_scan_nonfinite(const void* w, size_t elem, int64_t nmodes, int64_t ld, int64_t C, Scal* sc,
                           hipStream_t s);

}  // namespace dgmhd
