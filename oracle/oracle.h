/*
 * oracle.h -- FP64 CPU oracle of the second-order explicit ("A3") photoionisation
 * source-term step of Mackey, "Accuracy and efficiency of raytracing
 * photoionisation algorithms" (A&A 2012).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the bench's
 * CPU-baseline leg may load or call this library.  It shares no code, header,
 * table or constant generator with the HIP library; the two are independent
 * implementations of the same readings of the paper.
 *
 * Units are CGS throughout.  All arithmetic is IEEE double.
 */
#ifndef PI_ORACLE_H
#define PI_ORACLE_H

#include <stdint.h>

#define ORC_NTAB 64
#define ORC_MAX_SRC 4

/* ORC_GEOM_PLANE_3D: a 3D grid lit by a plane-parallel source at x = -infinity
 * (the slab test of Sect. 3.1 extended to three dimensions): every row of
 * cells along x is traced from the x = 0 face and Q is the photon flux. */
enum { ORC_GEOM_3D = 0, ORC_GEOM_SPHERICAL_1D = 1, ORC_GEOM_PLANAR_1D = 2, ORC_GEOM_PLANE_3D = 3 };
enum { ORC_SPEC_MONO = 0, ORC_SPEC_TABLE = 1 };
enum { ORC_T_FIXED = 0, ORC_T_EVOLVE = 1 };
enum { ORC_ALPHA_CONST = 0, ORC_ALPHA_POWER = 1 };
enum { ORC_W_GEOMETRIC = 0, ORC_W_MELLEMA = 1 };

typedef struct {
    int32_t geometry;        /* ORC_GEOM_*                                        */
    int32_t n[3];            /* cells per axis (1D modes use n[0] only)           */
    int32_t src[3];          /* source vertex, 0..n[d] (3D point source only)     */
    double  dx;              /* cell size [cm]                                    */
    double  Q;               /* photons/s into 4 pi (3D, spherical); flux (planar, plane 3D) */
    double  sigma0;          /* cross-section at threshold [cm^2]                 */
    int32_t spectrum;        /* ORC_SPEC_*                                        */
    double  e_excess;        /* heating per photoionisation [erg] (mono only)     */
    const double* table;     /* 5*ORC_NTAB: tau, P, P1, H, H1 (table mode only)   */
    int32_t thermal;         /* ORC_T_*                                           */
    double  T_fixed;         /* [K] when thermal == ORC_T_FIXED                   */
    int32_t recomb;          /* ORC_ALPHA_*                                       */
    double  alpha_B;         /* case-B coefficient (const) or its value at 1e4 K  */
    int32_t collisional;     /* 1: collisional ionisation (rate and cooling) on   */
    int32_t cooling;         /* 1: radiative cooling on (T evolving only)         */
    int32_t weights;         /* ORC_W_*                                           */
    int32_t source_cell_rule;/* 1: octant-corner cell takes Q/8 over mean chord   */
    int32_t n_sub;           /* SDIRK substeps per micro-integration              */
    double  K[4];            /* eq.(4) factors; +inf = criterion unused           */
    /* Further point sources (ORC_GEOM_3D only).  nsrc 0 or 1: the source at
     * src alone.  nsrc = m > 1: source 0 at src with Q, sources 1..m-1 at
     * src_more[s-1] with Q_more[s-1]; all share the spectrum (table mode: the
     * table is written for Q > 0 and scaled by Q_s / Q).  Every column array
     * (tau, tau_in) then holds m consecutive grids of N cells, source s at
     * offset s N, each traced on its own; the photoionisation and heating
     * rates of the sources add in every cell. */
    int32_t nsrc;
    int32_t src_more[ORC_MAX_SRC - 1][3];
    double  Q_more[ORC_MAX_SRC - 1];
} orc_desc;

/* per-step diagnostics (FP64 sums) */
typedef struct {
    double n_ion;        /* sum n_H (1-x) V                                 */
    double v_ion;        /* sum (1-x) V                                     */
    double r_ion;        /* volume-equivalent ionised radius; plane-parallel:
                            ionised depth, v_ion over the lit face's area     */
    double photo_rate;   /* sum V * photoionisations per volume per second  */
    double recomb_rate;  /* sum V * alpha n_H^2 (1-x)^2                     */
    int64_t newton_fail; /* stage solves that did not converge              */
} orc_diag;

int    orc_table_build(double T_bb, double Q, double* out /* 5*ORC_NTAB */);
double orc_table_eval(const double* table, int which /*0:P 1:H*/, double tau, double* dvdtau);

int    orc_raytrace_sc(const orc_desc* g, const double* nH, const double* x, double* tau_in);
int    orc_raytrace_lc(const orc_desc* g, const double* nH, const double* x, double* tau_in);

int    orc_cell_env(const orc_desc* g, int64_t cell, double* geo, double* ell);
int    orc_micro_cell(const orc_desc* g, double nH, double geo, double ell, double tau_in,
                      double x0, double E0, double h, double* x1, double* E1);
/* orc_micro_cell plus the cell's time-averaged optical depth over h (A1) */
int    orc_micro_cell_avg(const orc_desc* g, double nH, double geo, double ell, double tau_in,
                          double x0, double E0, double h, double* x1, double* E1, double* tau_avg);
int    orc_rhs_cell(const orc_desc* g, double nH, double geo, double ell, double tau_in,
                    double x, double E, double* fx, double* fE);
double orc_cell_dt(const orc_desc* g, double nH, double geo, double ell, double tau_in,
                   double x, double E);

int    orc_timestep(const orc_desc* g, const double* nH, const double* x, const double* E,
                    const double* tau, double* dt_out);
int    orc_chem(const orc_desc* g, const double* nH, const double* x0, const double* E0,
                const double* tau, double h, double* x1, double* E1);
int    orc_step(const orc_desc* g, const double* nH, double* x, double* E, double* tau,
                double* t, double t_end, int algo, double* dt_out);
int    orc_step_tc(const orc_desc* g, const double* nH, const double* nH_half, double* x,
                   double* E, double* tau, double* t, double t_end, int algo, double* dt_out);
/* Algorithm 1's combined raytrace and micro-physics pass over dt (Sect. 2.1);
 * orc_step with algo = 1 is the timestep, this pass and a raytrace of the new
 * state. */
int    orc_a1_pass(const orc_desc* g, const double* nH, double* x, double* E, double dt,
                   double* tau_avg, double* kbar);
int    orc_diagnostics(const orc_desc* g, const double* nH, const double* x, const double* E,
                       const double* tau, orc_diag* out);
int64_t orc_newton_failures(void);
void   orc_reset_newton_failures(void);
int    orc_front_index_1d(int n, const double* x);
double orc_mean_chord_source_cell(void);

#endif
