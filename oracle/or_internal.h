/* Internal layout of the oracle's code object.  Test infrastructure only. */
#ifndef TS_OR_INTERNAL_H
#define TS_OR_INTERNAL_H

#include <stdint.h>
#include "oracle.h"

struct or_code {
    int n, m;
    int64_t e;
    int64_t *row_ptr;  /* [m+1] check -> edges */
    int32_t *col;      /* [e]   variable of each edge, sorted within a row */
    int64_t *vptr;     /* [n+1] variable -> its checks */
    int32_t *vchk;     /* [e]   checks of each variable, sorted */
    int64_t *vedge;    /* [e]   edge index (in row order) of each (variable, check) */
    int z, mb, nb;     /* QC description, z = 0 for a plain CSR code */
    int girth;         /* 0 = cycle-free */
    int dv_max, dc_max;
};

/* Sorts ints ascending (qsort). */
void or_sort_i32(int32_t *a, int k);

#endif
