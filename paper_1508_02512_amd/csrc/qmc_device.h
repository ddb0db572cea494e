// Device-resident tables of a plan and a bound job.
//
// Every sector is stored with its variables permuted so that the ks
// variables carrying a subtracted pole (a_j = -1, Eq. 11) come first.  The
// terms of U and F are sorted by which of those ks variables they contain
// (a bit mask m < 2^ks); term ranges per mask let the kernel evaluate the
// polynomial once and obtain its value at every subtraction corner (the
// points with some of the first ks variables set to zero) by a subset-sum
// transform.  Exponents are packed 4 bits per variable into one uint32.
#pragma once

#include <stdint.h>

#define QMC_DMAX 8
#define QMC_KSMAX 4
#define QMC_NMASK (1 << QMC_KSMAX)
#define QMC_BLOCK 256
#define QMC_PROG_SLOTS 17    // power table slots: t_j, t_j^2 (j < 8) and 1
#define QMC_NO_INT (-1000000)
#define QMC_NFMAX 4          // numerator factors per sector (QMC_MAX_FACTORS)
#define QMC_NCOEF 8          // length of a sector's coefficient series (QMC_MAX_ORDERS)

struct qmc_sec_dev {
    int32_t dim;             // number of variables
    int32_t ks;              // variables with a pole, stored first
    int32_t K;               // Laurent orders carried: -ks .. K-1-ks
    int32_t deform;          // 1: contour deformation (complex kernel)
    int32_t perm[QMC_DMAX];  // original index of permuted variable j
    double a[QMC_DMAX];      // exponents a_j (permuted)
    double b[QMC_DMAX];      // exponents b_j (permuted)
    double inv_b[QMC_DMAX];  // 1/b_j for the pole variables
    int32_t aint[QMC_DMAX];  // a_j if a small non-negative integer, else QMC_NO_INT
    int32_t um[QMC_NMASK + 1];   // U terms of mask m: [um[m], um[m+1])
    int32_t fm[QMC_NMASK + 1];   // F terms of mask m: [fm[m], fm[m+1])
    // within each mask: terms of at most four power-table factors first,
    // then five to eight ([um1[m], um2[m])), then the exp form ([um2[m], um[m+1]))
    int32_t um1[QMC_NMASK], um2[QMC_NMASK];
    int32_t fm1[QMC_NMASK], fm2[QMC_NMASK];
    int32_t d1[QMC_DMAX + 1];    // dF/dt_j terms: [d1[j], d1[j+1]) in the derivative table
    int32_t d2[QMC_DMAX * (QMC_DMAX + 1) / 2 + 1];  // d2F/dt_j dt_k, j <= k, row-major
    double u0, u1, f0, f1;
    int32_t u0i, f0i;        // u0, f0 as integers, or QMC_NO_INT
    double lambda;
    int32_t lnmask;          // bit j: the real kernel needs ln t_j
    int32_t nf;              // numerator factors from integration by parts (Eq. 13)
    // terms of numerator factor i and mask m: [pm[i][m], pm[i][m+1]), split
    // by kind at pm1 and pm2 like the terms of U
    int32_t pm[QMC_NFMAX][QMC_NMASK + 1];
    int32_t pm1[QMC_NFMAX][QMC_NMASK], pm2[QMC_NFMAX][QMC_NMASK];
    int32_t pad;
};

struct qmc_lat_dev {         // lattice of one sector, components permuted
    uint32_t n;
    uint32_t z[QMC_DMAX];
    uint32_t pad;
    double inv_n;
};

// One work item: a tile of lattice indices start, start + stride, ... of
// one (kinematic point, sector, shift) group.
struct qmc_item {
    int32_t sector;          // sector header
    int32_t point;           // row of the contracted coefficients (and of lam)
    int32_t shift;           // row of the shift table
    int32_t group;           // output group (point, sector, shift)
    int32_t lat;             // lattice (n, z) of this item
    uint32_t start;          // first lattice index
    uint32_t count;          // number of indices; each lane takes ceil(count / 256)
    uint32_t stride;         // 1, or 2 for the odd indices of a doubled lattice
};

struct qmc_launch_args {
    const qmc_sec_dev *sec;
    const qmc_lat_dev *lat;  // [n_sectors]
    const uint32_t *texp;    // [n_terms] packed exponents of U and F terms
    const double *texpd;     // [n_terms][QMC_DMAX] the same exponents as doubles
    const uint32_t *tprog;   // [n_terms][2] each term as two 4-factor words
    const uint32_t *toff;    // [2][n_terms][4] LDS byte offsets of the terms' factors 1-4, 5-8
    const uint32_t *dprog;   // [n_dterms][2] the same for the derivative terms
    const double *tcoef;     // [n_points][n_terms] coefficients at each point
    const uint32_t *dexp;    // [n_dterms] packed exponents of derivative terms
    const double *dcoef;     // [n_points][n_dterms]
    const double *shifts;    // [m][QMC_DMAX]
    const double *lam;       // [points][n_sec] deformation parameter per sector
    const qmc_item *items;
    double *partial;         // [n_items][kstride][4]: (s_re, c_re, s_im, c_im)
    int32_t *viol;           // [n_items] deformation / sign violations
    int32_t n_terms, n_dterms;
    int32_t item_begin, item_end;
    int32_t kstride;         // order slots per item in `partial`
    int32_t pad0;
    int32_t korobov_r;
    int32_t n_sec;
};
