/*
 * cgmi_io.h -- reading a sparse matrix from a Matrix Market file into the
 * CSR layout that cg_create takes.
 *
 * The paper reads its matrices in Matrix Market format, converts them to
 * CSR and expands symmetric inputs (one stored triangle) to the full matrix
 * before the row split (Section 3.2).  This reader does the same on host
 * threads.
 *
 * Accepted files: a first line "%%MatrixMarket matrix coordinate <field>
 * <symmetry>" (case-insensitive) with field real, integer or pattern
 * (pattern entries read as 1.0) and symmetry general or symmetric; then
 * comment lines starting with '%'; a size line "M N L" with M == N; then L
 * entry lines "i j [value]" with 1-based indices.  In a symmetric file every
 * off-diagonal entry (i, j) also stands for (j, i).  Entries at the same
 * position are summed in file order (a mirrored entry directly after its
 * original) and columns are sorted within each row, so the result meets the
 * CSR conventions of cg_create (strictly increasing columns per row).
 *
 * Ownership: cg_mm_read allocates row_ptr, col and val; the caller releases
 * them with cg_mm_free (which also accepts a zero-filled struct).
 *
 * Errors (cg_last_error() names the file line): CG_EINVAL for a file that
 * cannot be opened, a missing or unsupported header (array format, complex,
 * hermitian or skew-symmetric, a non-square size), a malformed line, an
 * index outside 1..N, an entry count different from L, or more than
 * INT32_MAX stored entries after expansion; CG_ENOMEM when an allocation
 * fails.  On error *out is left zero-filled.
 */
#ifndef CGMI_IO_H
#define CGMI_IO_H

#include <stdint.h>

#include "cgmi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cg_mm_matrix {
    int32_t n;              /* rows = columns                                   */
    int64_t nnz;            /* stored entries after expansion and summing        */
    int32_t *row_ptr;       /* n + 1 entries, row_ptr[0] = 0 (library-owned)     */
    int32_t *col;           /* nnz 0-based columns, increasing within each row    */
    double *val;            /* nnz values                                        */
    int32_t symmetric;      /* 1: the file stored one triangle                   */
    int64_t file_entries;   /* entry lines in the file (L)                       */
} cg_mm_matrix;

/* Read path into *out (host memory).  threads: parsing threads (0: all
 * available).  Blocking; no GPU work. */
int cg_mm_read(const char *path, int32_t threads, cg_mm_matrix *out);
void cg_mm_free(cg_mm_matrix *m);

#ifdef __cplusplus
}
#endif
#endif /* CGMI_IO_H */
