/*
 * lnv.h -- C ABI of the MI355X (gfx950) LNV density-matrix hot path.
 *
 * The method (Sec. II.C.2 of the paper, "Density matrix: linear scaling"):
 * the density matrix in the support-function basis (Sec. II.B, rho = sum
 * phi K phi) is written through an auxiliary matrix L of restricted range
 * with the McWeeny form K = 3LSL - 2LSLSL; the band energy E = 2 Tr[KH] is
 * minimised with respect to the elements of L using dE/dL, under the
 * electron-number constraint N = 2 Tr[KS] = N_e.  All matrices are
 * atom-blocked (rows and columns indexed by atom i and function alpha) and
 * range truncated: a block (i, j) exists only when atoms i and j are closer
 * than the matrix's cutoff, so every product is a block-sparse multiply and
 * every cost is linear in the number of atoms.
 *
 * Conventions shared by every call
 *  - Device pointers are HIP device memory owned by the caller; host
 *    pointers are marked "host".  The library frees nothing.  Calls marked
 *    "hot path" allocate nothing; set-up calls may allocate and free
 *    temporaries with the stream-ordered allocator.
 *  - Calls are enqueued on the given stream.  Set-up calls that report a
 *    size to the host (nnz_out, n_items_out) synchronise that stream.
 *  - Every call returns an lnv_status.  Argument and pattern errors are
 *    detected on the host before anything is launched and leave every output
 *    untouched.  A failing HIP call returns LNV_EHIP; lnv_last_hip_error()
 *    gives its hipError_t.  Errors of already enqueued kernels surface at
 *    the next synchronising call or at lnv_sync_check().
 *  - Blocks are stored row-major, one after another in pattern order
 *    (row by row, ascending column), blk*blk values per block, blk == 4
 *    (other block edges return LNV_EUNSUPPORTED).  An atom with n_i
 *    support functions (Sec. II.B: 4 for the SZ silicon basis, 9 or 13 for
 *    larger ones) spans ceil(n_i / 4) consecutive stored rows, the layout of
 *    lnv_atoms_layout; callers that hold atom blocks of n_i x n_j values
 *    (lnv_vbsm) convert with lnv_vbsm_pack and lnv_vbsm_unpack.
 *  - Reductions (traces, dot products) are computed in FP64 with a fixed
 *    order that does not depend on timing: results are bitwise
 *    reproducible run to run on the same device and grid.
 */
#ifndef LNV_H
#define LNV_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lnv_status {
  LNV_OK = 0,
  LNV_EINVAL = 1,       /* bad argument (null pointer, negative size, ...) */
  LNV_ECAPACITY = 2,    /* output buffer too small; *nnz_out = needed size */
  LNV_EPATTERN = 3,     /* incompatible patterns or a missing index table */
  LNV_EHIP = 4,         /* a HIP runtime call failed */
  LNV_ENUMERIC = 5,     /* non-finite value or no admissible root */
  LNV_EUNSUPPORTED = 6  /* valid request this build does not implement */
} lnv_status;

/* Value types of lnv_bsm.  FP32 matrices are accepted by the multiply, the
 * transpose and the conversion calls and by the mixed-precision evaluation's
 * workspace; every other call takes FP64. */
enum { LNV_F64 = 0, LNV_F32 = 1 };

/* Largest block-row count accepted by the set-up kernels (LDS bitmaps). */
#define LNV_MAX_ATOMS 262144

/*
 * Spatial index of a pattern: where block (i, j) is stored, found in O(1)
 * with memory linear in the number of rows.  The paper's linear-scaling
 * multiplies rest on locality: a block exists only for atoms within the
 * matrix's range (Sec. II.C.2), so the columns of a row lie in the cells of
 * space near the row's own cell.  The periodic box is cut into g[0] x g[1] x
 * g[2] cells (lnv_cells); every unit (a row, or with qs = 2 an atom of four
 * rows, see below) gets its cell (packed x | y << 10 | z << 20) and its slot,
 * the rank of the unit among the units of its cell (at most occ per cell).
 * A pattern's window is the box of cells within r[a] of a row's cell along
 * each axis (r the largest offset any block of the pattern has; w[a] =
 * min(2 r[a] + 1, g[a]) cells), and its table holds, per row unit, one entry
 * per (window cell, slot):
 *   d_a  = (cell_a(j) - cell_a(i) + r_a) mod g_a     (valid iff d_a < w_a),
 *          or cell_a(j) itself on an axis the window spans (w_a = g_a)
 *   pos(i, j) = tab[unit(i) * stride + ((d_0 w_1 + d_1) w_2 + d_2) occ + slot(j)]
 * (-1: no block), stride = w_0 w_1 w_2 occ.  With qs = 2 the units are the
 * atoms of a tile4 pattern (4 rows with the same columns, in aligned runs
 * 4b..4b+3, see lnv_pattern_tile4): the table holds the position of block
 * (4a, 4b), and block (4a + s, 4b + t) is at that + s * len + t, len the
 * length of the atom's rows.  One cell (g = 1, 1, 1) makes the table the
 * dense n x n one; cells of about the shortest range keep it a few times
 * the pattern's own size.
 */
typedef struct lnv_index {
  const int32_t* tab;      /* device [n_units * stride + 1] (last entry -1) or NULL */
  const int32_t* cell;     /* device [n_units]: packed cell of each unit */
  const int32_t* slot;     /* device [n_units]: rank of each unit in its cell */
  int32_t g[3];            /* cells along each axis (each <= 1024) */
  int32_t r[3];            /* window half widths, cells */
  int32_t w[3];            /* window widths, min(2 r + 1, g) */
  int32_t occ;             /* largest number of units in one cell */
  int32_t qs;              /* log2 of rows per unit: 0 (rows) or 2 (atoms of 4 rows) */
  int64_t stride;          /* table entries per unit, w0 w1 w2 occ */
} lnv_index;

/*
 * Atom-block sparsity pattern.  row_ptr/col is CSR over atoms with columns
 * ascending in each row.  The optional index ix (lnv_pattern_index) finds a
 * block in O(1).  items lists the work pieces of the row-parallel kernels:
 * item q covers row items[2q] from position items[2q+1] for up to 64 blocks
 * (never past the end of the row).
 *
 * Cluster plan (optional; used by the multiply when both A and C carry one
 * with the same cl_m): rows are grouped into clusters of cl_m consecutive
 * atoms (consecutive atoms are spatial neighbours when atoms are numbered
 * cell by cell), and for each cluster c the sorted union of its rows'
 * columns is cl_col[cl_ptr[c] .. cl_ptr[c+1]); cl_pos[t*cl_m + r] is the
 * position of block (c*cl_m + r, cl_col[t]) or -1, and cl_cell[2t],
 * cl_cell[2t+1] the packed cell and the slot of column cl_col[t]'s unit in
 * the pattern's index (the contraction's k when P is the left operand).  As
 * the left operand A this is the contraction list of a cluster; as the
 * output C its columns are split into work pieces of 64/cl_g columns,
 * cl_items[2q] = cluster, cl_items[2q+1] = first position in cl_col.
 *
 * Atom tiles: atoms with 13 support functions are stored as 4 consecutive
 * 4x4-blocked rows (see lnv_synth_blocks), so an atom pair is a dense 16x16
 * tile.  With 16-row cluster plans (cl_m = 16: 4 such atoms) on A and C and
 * tile4 = 1 on A, B and C, the multiply forms whole 16x16x16 atom products
 * on the matrix cores (lnv_pattern_cluster, lnv_pattern_tile4).
 */
typedef struct lnv_pattern {
  int32_t n;               /* atoms (block rows = block columns) */
  int32_t n_items;         /* entries of items */
  int64_t nnzb;            /* stored blocks */
  const int32_t* row_ptr;  /* device [n+1] */
  const int32_t* col;      /* device [nnzb] */
  lnv_index ix;            /* spatial index (ix.tab == NULL: none) */
  const int32_t* items;    /* device [2*n_items] or NULL */
  int32_t cl_m;            /* rows per cluster (0: no cluster plan) */
  int32_t cl_g;            /* lanes sharing one output column (1, or 4 and 8 for tiles) */
  int32_t n_cl_items;      /* entries of cl_items */
  int32_t tile4;           /* grade from lnv_pattern_tile4 (1 tile4, 0 not) */
  const int32_t* cl_ptr;   /* device [ceil(n/cl_m)+1] */
  const int32_t* cl_col;   /* device [cl_ptr[last]] */
  const int32_t* cl_pos;   /* device [cl_ptr[last]*cl_m] */
  const int32_t* cl_items; /* device [2*n_cl_items] */
  const int32_t* cl_cell;  /* device [2*cl_ptr[last]] */
} lnv_pattern;

/* Block-sparse matrix: a pattern (host descriptor) plus block values. */
typedef struct lnv_bsm {
  const lnv_pattern* pat;  /* host pointer */
  int32_t blk;             /* block edge (stored values per block: blk*blk) */
  int32_t dtype;           /* LNV_F64 or LNV_F32 */
  void* val;               /* device [pat->nnzb * blk * blk] */
} lnv_bsm;

/* ------------------------------------------------------------ atoms
 * Atoms and their support functions (Sec. II.B: the density matrix and the
 * Hamiltonian are written in the support functions of the atoms, element
 * (i alpha, j beta), atom i carrying n_i functions).  lnv_atoms is the
 * library's map from atoms to stored rows: atom a spans rows row_start[a] ..
 * row_start[a+1]-1 (ceil(nfun[a]/4) rows); row r holds functions off_of[r]
 * .. off_of[r]+3 of atom atom_of[r] (those past nfun[a] are zero padding).
 * Atoms may be stored in any order (order in lnv_atoms_layout), e.g.
 * spatially sorted so that neighbouring rows are neighbouring atoms.
 */
typedef struct lnv_atoms {
  int32_t n_atoms;
  int32_t n_rows;             /* stored rows, sum of ceil(nfun[a] / 4) */
  const int32_t* nfun;        /* device [n_atoms]: support functions n_a (1..64) */
  const int32_t* row_start;   /* device [n_atoms+1]: first stored row of each atom */
  const int32_t* atom_of;     /* device [n_rows] */
  const int32_t* off_of;      /* device [n_rows] */
} lnv_atoms;

/* Atom-blocked matrix with blocks of each atom pair's own size: the form in
 * which the paper states the matrices (Sec. II.B).  row_ptr/col is CSR over
 * atoms (columns ascending); block p (atoms i, j) holds n_i x n_j values,
 * row-major, at val[val_off[p] ..] (lnv_vbsm_offsets). */
typedef struct lnv_vbsm {
  const lnv_atoms* atoms;     /* host pointer */
  const int32_t* row_ptr;     /* device [n_atoms+1] */
  const int32_t* col;         /* device [nnz] */
  const int64_t* val_off;     /* device [nnz+1] */
  int64_t nnz;                /* atom blocks */
  int32_t dtype;              /* LNV_F64 or LNV_F32 */
  void* val;                  /* device [val_off[nnz]] */
} lnv_vbsm;

/* lnv_atoms_layout -- the stored-row layout of atoms with nfun[a] support
 * functions (device [n_atoms], each 1..64; Sec. II.B), atoms stored in the
 * order order[0], order[1], ... (device [n_atoms], a permutation; NULL: atom
 * order).  Two-phase: always writes row_start (device [n_atoms+1]) and
 * *n_rows_out (host); with atom_of != NULL also atom_of and off_of (device
 * [cap] each; LNV_ECAPACITY when cap < *n_rows_out).  LNV_EINVAL for an
 * order that is not a permutation, LNV_EUNSUPPORTED for a function count
 * outside 1..64 or more than LNV_MAX_ATOMS rows.  Set-up call: synchronises
 * s. */
int lnv_atoms_layout(const int32_t* nfun, int32_t n_atoms, const int32_t* order,
                     int32_t* row_start, int32_t* atom_of, int32_t* off_of, int64_t cap,
                     int32_t* n_rows_out, hipStream_t s);

/* lnv_atoms_rows -- row_pos (device [n_rows][3]) = the position of each
 * stored row's atom (atom_pos: device [n_atoms][3]), the positions that
 * lnv_neighbours, lnv_cells and lnv_synth_blocks take for split atoms (the
 * ranges of Sec. II.C.2 are atom distances, so every row of an atom shares
 * its neighbours). */
int lnv_atoms_rows(const lnv_atoms* A, const double* atom_pos, double* row_pos, hipStream_t s);

/* lnv_vbsm_offsets -- val_off (device [nnz+1]) of an atom pattern (row_ptr,
 * col: device, atom CSR with nnz blocks): block p of atoms (i, j) starts at
 * the sum of n_i' n_j' over the blocks before it; *len_out (host, may be
 * NULL) = val_off[nnz], the values to allocate.  Set-up call: synchronises
 * s; LNV_EPATTERN for a malformed pattern.  Storage of the atom blocks of
 * Sec. II.B (n_i x n_j per atom pair). */
int lnv_vbsm_offsets(const lnv_atoms* A, const int32_t* row_ptr, const int32_t* col,
                     int64_t nnz, int64_t* val_off, int64_t* len_out, hipStream_t s);

/* lnv_vbsm_pack -- B = A in the stored-row layout (Sec. II.B blocks to 4x4
 * storage): element (s, t) of B's block (r, c) is element (off_of[r] + s,
 * off_of[c] + t) of A's block (atom_of[r], atom_of[c]); zero past either
 * atom's functions or where A has no block.  B's pattern is over the rows of
 * A.atoms (n = n_rows), blk 4, same dtype as A.  Every block of B is
 * written. */
int lnv_vbsm_pack(const lnv_vbsm* A, lnv_bsm* B, hipStream_t s);

/* lnv_vbsm_unpack -- A = B back in atom blocks: element (x, y) of A's block
 * (i, j) is element (x mod 4, y mod 4) of B's block (row_start[i] + x/4,
 * row_start[j] + y/4), zero where B has no block.  B's pattern needs its
 * index; same dtype.  Every value of A is written.  Back to the atom blocks
 * of Sec. II.B. */
int lnv_vbsm_unpack(const lnv_bsm* B, lnv_vbsm* A, hipStream_t s);

/* ------------------------------------------------------------ errors
 * Library infrastructure (error reporting); the paper has no counterpart.
 */
const char* lnv_strerror(int status);
int lnv_last_hip_error(void);
/* Synchronise s and report any asynchronous kernel error as LNV_EHIP
 * (library infrastructure). */
int lnv_sync_check(hipStream_t s);

/* ------------------------------------------------------------ a0: ranges
 * lnv_neighbours -- range pattern of one matrix (Sec. II.C.2: an element
 * between atoms i and j is zero when their distance exceeds the cutoff R).
 * Periodic orthorhombic cell (Sec. II.C.1 applies periodic boundary
 * conditions): the distance is to the nearest image, per axis
 *   dx = (x_j - x_i) - box * rint((x_j - x_i)/box),
 *   d2 = (dx*dx + dy*dy) + dz*dz  (no fused multiply-add),
 * and (i, j) is kept iff d2 <= R*R.  The self pair is always kept; columns
 * are ascending.
 *  pos      device [n][3] FP64 positions, each coordinate in [0, box)
 *  box      host [3] cell edges
 *  row_ptr  device [n+1], always written
 *  col      device [cap] or NULL (count only)
 *  nnz_out  host: number of pairs.  LNV_ECAPACITY if col != NULL and
 *           cap < *nnz_out (col is then not written).
 * Synchronises s.
 */
int lnv_neighbours(const double* pos, int32_t n, const double* box, double R,
                   int32_t* row_ptr, int32_t* col, int64_t cap, int64_t* nnz_out,
                   hipStream_t s);

/* ------------------------------------------------------------ a2: products
 * lnv_pattern_product -- pattern of a block-sparse product (the symbolic
 * half of the linear-scaling multiplies of Sec. II.C.2).  Output row i holds
 * every j with some k such that (i,k) in A and (k,j) in B (the natural range
 * of A.B); with mask != NULL only the j in mask's row i are kept.
 *  row_ptr      device [n+1], always written
 *  col          device [cap] or NULL (count only)
 *  nnz_out      host: output blocks (LNV_ECAPACITY as above)
 *  row_triples  device [n+1] or NULL: exclusive prefix sums of the number of
 *               (i,k,j) triples feeding each row's kept blocks (row i has
 *               row_triples[i+1] - row_triples[i]; row_triples[n] = total)
 *  triples_out  host or NULL: total triples (2*blk^3 flops each)
 * A and B need row_ptr/col; mask (if given) too.  Synchronises s.
 */
int lnv_pattern_product(const lnv_pattern* A, const lnv_pattern* B,
                        const lnv_pattern* mask, int32_t* row_ptr, int32_t* col,
                        int64_t cap, int64_t* nnz_out, int64_t* row_triples,
                        int64_t* triples_out, hipStream_t s);

/* lnv_pattern_flops -- algorithmic flops of the product A.B on its natural
 * pattern (mask == NULL) or on mask: sum over the kept triples (i,k,j) of
 * 2 f_i f_k f_j, f = row_fun (device [n]: support functions present in each
 * stored row, so padded rows count only what they hold).  Host result in
 * *flops_out.  Set-up call: allocates temporaries, synchronises s.
 * Cost of the range-truncated products of Sec. II.C.2.
 */
int lnv_pattern_flops(const lnv_pattern* A, const lnv_pattern* B, const lnv_pattern* mask,
                      const int32_t* row_fun, int64_t* flops_out, hipStream_t s);

/* lnv_pattern_half -- the half of a symmetric pattern P that holds each pair
 * {i, j} of different row groups once, balanced over the rows: rows are
 * grouped in fours (singly when n is not a multiple of 4); block (i, j) is
 * kept when i and j fall in one group (both orders: a symmetric product
 * formed on the half then has both (i, j) and (j, i) of a group, which its
 * mirror averages), or, for groups A != B of m groups, when the cyclic
 * offset D = (B - A) mod m has 2D < m (ties 2D = m: A < B).  Every row keeps
 * about half of its columns (the upper triangle j >= i of a periodic cell
 * keeps nearly all of an early row's columns and few of a late one's, which
 * leaves the multiply's last wave of work pieces nearly empty), and atoms
 * stored as 4 rows keep or drop whole 16x16 tiles, so the half of a tile4
 * pattern is tile4.  Columns ascending; two-phase like lnv_neighbours
 * (col == NULL counts).  Synchronises s.
 * Uses the symmetry of L, S and H (Sec. II.C.2); a work-saving layout, not a step of the paper.
 */
int lnv_pattern_half(const lnv_pattern* P, int32_t* row_ptr, int32_t* col, int64_t cap,
                     int64_t* nnz_out, hipStream_t s);

/* lnv_cells -- the cells of the spatial index (see lnv_index): n_units
 * positions (device [n_units][3], FP64, in the periodic box, host [3]), the
 * grid g (host [3], each 1..1024) and the grid's origin (host [3]); unit u
 * lies in cell floor(frac(((x - origin) / box)) * g) per axis, and its slot
 * is its rank among the units of that cell in unit order.  Writes cell and
 * slot (device [n_units]) and *occ_out (host: the fullest cell's count).
 * Set-up call: copies the positions to the host, synchronises s.
 * Rests on the locality of the ranges of Sec. II.C.2 (a block exists only within its cutoff).
 */
int lnv_cells(const double* pos, int32_t n_units, const double* box, const int32_t* g,
              const double* origin, int32_t* cell, int32_t* slot, int32_t* occ_out,
              hipStream_t s);

/* lnv_pattern_index -- the spatial index of P (see lnv_index) on the cells
 * (cell, slot: device [n >> qs], from lnv_cells over P's units; g, occ as
 * lnv_cells gave them).  qs = 2 needs a tile4 pattern (lnv_pattern_tile4).
 * Two-phase: with tab == NULL only the window is measured -- P->ix is filled
 * (r, w, stride, cell, slot, g, occ, qs; tab NULL) and *len_out (host) is
 * the table's length, n_units * stride + 1 (a trailing -1 that lookups
 * outside the window may read); then with tab (device [cap]) the
 * table is written and P->ix.tab set (LNV_ECAPACITY if cap < *len_out).
 * Synchronises s.
 * Rests on the locality of the ranges of Sec. II.C.2.
 */
int lnv_pattern_index(lnv_pattern* P, const int32_t* cell, const int32_t* slot,
                      const int32_t* g, int32_t occ, int32_t qs, int32_t* tab, int64_t cap,
                      int64_t* len_out, hipStream_t s);

/* lnv_pattern_transpose_map -- perm[p] = position in PT of the transpose of
 * block p of P (PT must hold the transposed pattern and have its index);
 * LNV_EPATTERN when a block has no transpose in PT.
 * Transposes needed by G of Sec. II.C.2 (X + X^T).
 */
int lnv_pattern_transpose_map(const lnv_pattern* P, const lnv_pattern* PT, int32_t* perm,
                              hipStream_t s);

/* lnv_pattern_cluster -- cluster plan of P (see lnv_pattern) for clusters of
 * m rows with g lanes per output column: (m, g) = (4, 1), one lane per
 * column accumulating the cluster's 4 rows; or atom-tile plans, m = 16 (4
 * atoms of 4 rows) with pieces of 64/g = 16 or 8 union columns (4 or 2
 * column atoms per wavefront), (m, g) = (16, 4) or (16, 8), whose unions
 * come in aligned runs of 4 columns (tile4 patterns).  P needs its index
 * (the positions and cells come from it).  Two-phase like lnv_neighbours:
 * with cl_col == NULL only *len_out (union length) and *n_items_out are
 * reported; cl_ptr is always written (device [ceil(n/m)+1]); cl_cell (device
 * [2*cap]) receives the packed cell and slot of each union column.
 * Synchronises s.
 * Work decomposition of the products of Sec. II.C.2 on the GPU (the paper's partitions and processes are not reproduced).
 */
int lnv_pattern_cluster(const lnv_pattern* P, int32_t m, int32_t g, int32_t* cl_ptr,
                        int32_t* cl_col, int32_t* cl_pos, int32_t* cl_cell, int64_t cap,
                        int32_t* cl_items, int64_t items_cap, int64_t* len_out,
                        int32_t* n_items_out, hipStream_t s);

/* lnv_pattern_tile4 -- grade of P for the atom-tile multiply and the atom
 * index (qs = 2), in *ok_out (host): 1 when P is a tile4 pattern: n is a
 * multiple of 4, rows 4a..4a+3 hold the same columns, and every row's
 * columns come in aligned runs 4b, 4b+1, 4b+2, 4b+3 -- the layout of atoms
 * stored as 4 rows each with patterns built from atom distances, their
 * products and the halves of symmetric ones (lnv_pattern_half); then the 16
 * blocks of an atom tile are found from the position p of its first one as
 * p + s*len + t (sub-row s, sub-column t, len the row length).  0 otherwise
 * (4-function atoms, mixed atom sizes).  The value belongs in
 * lnv_pattern.tile4.  Set-up call: allocates flags, synchronises s.
 * Atom tiles of 13-function atoms (Sec. II.B); layout for the products of Sec. II.C.2.
 */
int lnv_pattern_tile4(const lnv_pattern* P, int32_t* ok_out, hipStream_t s);

/* lnv_pattern_items -- work list of P: with items == NULL only counts.
 *  n_items_out  host: number of items (LNV_ECAPACITY if cap is smaller).
 * Synchronises s.
 * Work decomposition of the products of Sec. II.C.2 on the GPU.
 */
int lnv_pattern_items(const lnv_pattern* P, int32_t* items, int64_t cap,
                      int32_t* n_items_out, hipStream_t s);

/* ------------------------------------------------------------ a1: values
 * lnv_synth_blocks -- synthetic overlap (kind 0) or Hamiltonian (kind 1)
 * blocks on M's pattern, standing in for the grid integrals of Eq. (2):
 *   S_ij = w(i,j) M_ij + 2 I delta_ij,   H_ij = -(w(i,j) M_ij),
 *   w(i,j) = sum over images T of j with d_T^2 <= R^2 of exp(-(d_T/decay)),
 * images enumerated with integer offsets t in [-m, m]^3 (tx outermost,
 * m = ceil(R/box) + 1) and d_T^2 formed as in lnv_neighbours.  M_ij is a
 * seeded random block: for i <= j element e = r*nj + c is
 * scale*(u - 0.5), u = (SplitMix64 output number ctr of seed >> 11) * 2^-53,
 * ctr = stream<<56 | i<<32 | j<<8 | e (stream 1 for S, 2 for H); M_ji = M_ij^T
 * and diagonal blocks are (R + R^T) * 0.5.  Support functions per atom come
 * from nfun (device, indexed by atom; NULL: every atom has M->blk); entries
 * of a block beyond nfun are zero.
 * Atoms with more support functions than blk (9 or 13 with blk 4) span
 * several stored rows: with atom_of / off_of (device [n], both or neither)
 * stored row i holds rows off_of[i] .. off_of[i]+blk-1 of atom atom_of[i]'s
 * functions, pos is then per stored row (the atom's position repeated), and
 * the counters above use the atom pair and the element's index in the atom
 * block, so the values do not depend on the split.  Such padded rows and
 * columns are zero in S and H; the CG's identity and Hotelling start leave
 * them at zero (see lnv_cg_init).
 * Stands in for H and S of Sec. II.B (no real integrals here).
 */
int lnv_synth_blocks(const double* pos, const double* box, const int32_t* nfun,
                     const int32_t* atom_of, const int32_t* off_of, const lnv_bsm* M,
                     int32_t kind, double R, double decay, uint64_t seed, double scale,
                     hipStream_t s);

/* ------------------------------------------------------------ a3: multiply
 * lnv_bsm_multiply -- C = alpha * A * op(B) + beta * C on C's pattern only
 * (blocks of the product outside C's pattern are not formed: a range
 * truncated product).  op(B) = B (transB = 0) or B^T (transB = 1); with
 * transB = 2, B is symmetric and B.val holds only the blocks of its half
 * (B on a pattern from lnv_pattern_half, with its index): blocks outside the
 * half are read as the transposes of their mirror blocks.  transB = 2 runs on
 * the atom-tile path only (16-row cluster plans on A and C, tile4 patterns,
 * FP64 or all-FP32 storage); elsewhere, and for lnv_bsm_multiply_dot, it
 * returns LNV_EUNSUPPORTED.  These
 * are the sparse matrix products of Sec. II.C.2: with every matrix range
 * truncated, each product costs a bounded number of block triples per row,
 * so its cost is linear in the number of atoms.
 * Needs A.row_ptr/col, B's spatial index (either orientation) and C.items.
 * dtypes: all FP64; all FP32 (FP32 products and accumulation, or as set by
 * lnv_set_f32_accumulation); or FP32 A and B with an FP64 C (FP64
 * multiply-add: the products of FP32 values are exact in FP64, the sums
 * round in FP64; beta scales the FP64 C).  Other mixes: LNV_EUNSUPPORTED.
 * Hot path: allocates nothing and needs no workspace
 * (lnv_multiply_ws_bytes).
 */
int lnv_bsm_multiply(double alpha, const lnv_bsm* A, const lnv_bsm* B, int32_t transB,
                     double beta, lnv_bsm* C, hipStream_t s);

/* lnv_multiply_ws_bytes -- device workspace in bytes of the product C =
 * A op(B) (Sec. II.C.2): 0 for lnv_bsm_multiply (with_dot = 0); with
 * with_dot != 0 the partials buffer of lnv_bsm_multiply_dot (two doubles per
 * work piece: the cluster pieces when the product runs on cluster plans,
 * else C's row items).  Host result in *bytes_out; no device work. */
int lnv_multiply_ws_bytes(const lnv_bsm* A, const lnv_bsm* B, int32_t transB,
                          const lnv_bsm* C, int32_t with_dot, int64_t* bytes_out);

/* lnv_bsm_multiply_dot -- as lnv_bsm_multiply, and in the same pass
 * out[d] = <M_d, C> for the given partners M_1, M_2 (NULL to skip; both on
 * C's pattern); with store == 0 the finished product is not written back
 * (only the traces are wanted; C.val is not touched).  partials: device
 * [2 * max(C.n_items, C.n_cl_items)] scratch; out: device.
 * The products and traces of Sec. II.C.2 (E = 2 Tr[KH] and N = 2 Tr[KS] are sums of such traces).
 */
int lnv_bsm_multiply_dot(double alpha, const lnv_bsm* A, const lnv_bsm* B, int32_t transB,
                         double beta, lnv_bsm* C, int32_t store, const lnv_bsm* M1,
                         const lnv_bsm* M2, double* partials, double* out, hipStream_t s);

/* lnv_bsm_multiply_dot_noalloc -- lnv_bsm_multiply_dot for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the trace partials live in a fixed
 * scratch array of LNV_NOALLOC_PARTIALS doubles (4 MiB) that the library
 * holds on each GPU it runs on until the process ends, instead of the
 * caller's partials buffer.  Same arguments and results otherwise; M1 and
 * out are required (the call exists for the traces).  The call allocates
 * nothing (no hipMalloc, no library allocation; the device address of the
 * scratch is looked up once per device on the first call made with that
 * device current).  Errors: LNV_ECAPACITY when the product has more than
 * LNV_NOALLOC_PARTIALS / 2 work pieces (lnv_pattern n_cl_items, or n_items
 * without a cluster plan); LNV_EUNSUPPORTED while the multiply timing is on
 * (it creates events).  Every call on one GPU shares that GPU's scratch:
 * calls that overlap on one device (concurrent streams, or host threads)
 * race, and must be serialised by the caller.  Every work piece writes its
 * partials before they are reduced, so the scratch needs no clearing.
 * Same operation as lnv_bsm_multiply_dot (Sec. II.C.2).
 */
#define LNV_NOALLOC_PARTIALS (1 << 19)
int lnv_bsm_multiply_dot_noalloc(double alpha, const lnv_bsm* A, const lnv_bsm* B,
                                 int32_t transB, double beta, lnv_bsm* C, int32_t store,
                                 const lnv_bsm* M1, const lnv_bsm* M2, double* out,
                                 hipStream_t s);

/* lnv_bsm_transpose -- AT = A^T: block p of A, transposed, goes to position
 * perm[p] of AT (perm from lnv_pattern_transpose_map).  Needs A.items.
 * A and AT of one dtype.  Hot path (HBM-bound copy).
 * Transposes needed by G of Sec. II.C.2 (X + X^T, A^T X).
 */
int lnv_bsm_transpose(const lnv_bsm* A, const int32_t* perm, lnv_bsm* AT, hipStream_t s);

/* lnv_bsm_convert -- B = A converted elementwise to B's dtype (FP64 <-> FP32,
 * round to nearest), A and B on the same pattern (or patterns with the same
 * number of blocks).  Hot path (HBM-bound).
 * Feeds the mixed-precision products (not in the paper, which works in FP64).
 */
int lnv_bsm_convert(const lnv_bsm* A, lnv_bsm* B, hipStream_t s);

/* lnv_bsm_lincomb -- out = a X + b Y + c Z elementwise on one pattern (Y, Z
 * may be NULL; out may alias any input).  FP64.  Hot path (HBM-bound).
 * Updates of L and of the search vectors in the minimisation of Sec. II.C.2.
 */
int lnv_bsm_lincomb(double a, const lnv_bsm* X, double b, const lnv_bsm* Y, double c,
                    const lnv_bsm* Z, lnv_bsm* out, hipStream_t s);

/* lnv_bsm_remap -- B = A carried over to B's pattern (same atoms, e.g. the
 * range pattern of a new geometry): blocks of B present in A's pattern are
 * copied, the others are zero.  A's pattern needs its index.  FP64, blk 4.
 * Carries L to a new geometry (molecular dynamics, Sec. III.C).
 */
int lnv_bsm_remap(const lnv_bsm* A, lnv_bsm* B, hipStream_t s);

/* lnv_bsm_norm_inf -- out[0] = max_a sum_b |A_ab| (the matrix infinity norm,
 * over orbital rows).  partials: device [A.pat->n] scratch; out: device.
 * FP64, blk 4.
 * Gershgorin bound of the start of Hotelling's iteration (Sec. II.C.2).
 */
int lnv_bsm_norm_inf(const lnv_bsm* A, double* partials, double* out, hipStream_t s);

/* lnv_set_f32_accumulation -- arithmetic of the FP32 products (process-wide):
 * LNV_ACC_F32 (the default): FP32 multiply-add into FP32 accumulators (the
 * atom-tile multiply: v_mfma_f32_16x16x4_f32);
 * LNV_ACC_F64: FP64 multiply-add into FP64 accumulators (the product of two
 * FP32 values is exact in FP64, so only the sums round, in FP64), the result
 * rounded once to FP32 at the store;
 * LNV_ACC_F16X3: atom-tile multiplies split each operand as x*2^8 = hi + lo
 * in FP16 and form Ah.Bh + Ah.Bl + Al.Bh on v_mfma_f32_16x16x16_f16 with
 * FP32 accumulation (about FP32 accuracy for |x| >= 5e-4; entries must stay
 * below 255 in magnitude); the 4x4 multiplies run as LNV_ACC_F32.
 * Either way the operands and the result are stored in FP32.
 * Not in the paper (which works in FP64): arithmetic of this library's FP32 products.
 */
enum { LNV_ACC_F32 = 0, LNV_ACC_F64 = 1, LNV_ACC_F16X3 = 2 };
int lnv_set_f32_accumulation(int32_t acc);

/* lnv_bsm_dot -- <A, B> = sum over A's blocks of A_ij . B_ij (Frobenius),
 * with B_ij taken at the same position when B shares A's pattern object,
 * otherwise through B's spatial index (absent blocks count as zero).
 * partials: device [LNV_DOT_PARTIALS] scratch; out: device [1].  Hot path.
 * The traces of Sec. II.C.2: for symmetric matrices Tr[AB] = <A, B>.
 */
#define LNV_DOT_PARTIALS 1024
int lnv_bsm_dot(const lnv_bsm* A, const lnv_bsm* B, double* partials, double* out,
                hipStream_t s);

/* ------------------------------------------------------------ a4: evaluation
 * Intermediates of one evaluation.  With A = LS (stored in both orientations,
 * SL and LS), X = HLS (stored with its transpose XT) and Z = SLS on patterns
 * that hold every entry the projections below read (X_kj and Z_kj with some
 * i for which (i, k) is in pat(S.L) and (i, j) in L's pattern: the natural
 * ranges, or those cut to atoms within R_S + 2 R_L of each other):
 *   E = 2 (3 <L, X> - 2 <L, P_L(X A)>)
 *   N = 2 (3 <L, Z> - 2 <L, P_L(A^T Z)>)
 *   G = dE/dL = 2 P_L[3 (X + X^T) - 2 (Y + Y^T + A^T X)],   Y = P_L(X A)
 *   F = dN/dL = 12 P_L[Z - A^T Z]
 * which follow from K = 3LSL - 2LSLSL and E = 2 Tr[KH] (Sec. II.C.2) by
 * differentiating each stored entry of L.
 *  SL  values on pat(S.L)   (pattern needs items; its index for the metric)
 *  LS  values on pat(L.S)   (pattern needs its index)
 *  X   values on pat(H.L.S) (pattern needs its index and items)
 *  XT  values on X's pattern transposed (pattern needs its index)
 *  Z   values on pat(S.L.S) (pattern needs its index and items)
 *  (pat(.) above: either range, the same cut for X, XT and Z)
 *  perm_SL, perm_X  transpose maps SL -> LS and X -> XT
 * Every operand B of the products is read in its stored orientation: a
 * transposed read would gather 64 blocks from 64 distant rows per step.
 * LS and XT may be left out together (both val NULL; their patterns and
 * perm_SL, perm_X are then not used): the products read S.L and X
 * transposed instead, which the atom-tile multiply does at full speed (a
 * tile is read as 16 rows either way) -- for cells of 13-function atoms
 * too large to hold both orientations of the intermediates.
 * lnv_cg_step needs them (scratch of the line search).
 *  YT, W, V  device [nnzb_L * 16]: P_L(SLSLH), P_L(SLHLS), P_L(SLSLS)
 *  partials  device [partials_len] scratch, partials_len >=
 *            lnv_partials_len(max(n_items, n_cl_items) of L's pattern)
 *  scalars   device [LNV_NSCALARS] FP64 (see LNV_SC_*)
 * Symmetric products (optional, val == NULL: not used): Z = SLS, W = P_L(SLHLS)
 * and V = P_L(SLSLS) are symmetric for symmetric L, S, H, so only their
 * blocks in one half of their pattern need forming; the rest is their
 * transpose.
 *  Zu  values on the half of Z's pattern (lnv_pattern_half; needs its index,
 *      items, and the cluster plan of the other outputs), dtype of Z
 *  Lu  values on the half of L's pattern (same needs): W's blocks there;
 *      Vu (device [nnzb of Lu * 16], dtype of W) V's
 * Z, W, V are then filled by a transposing copy (Z's and L's patterns need
 * items and must be symmetric; a block whose transpose is missing comes out
 * NaN).  Exception: in a lean workspace (LS and XT left out) whose products
 * run on the atom tiles, Z stays on its half -- V and the assembly read it
 * there (lnv_bsm_multiply's transB = 2) -- and Z.val is not written.  lnv_cg_step uses the same buffers for the electron-number
 * check (Z, V at the new L) and Lu for the metric products P_L(T G T); in
 * the line search and the electron-number correction Lu and Vu hold L and
 * the direction on the half (weight 2 off the diagonal), the partners of
 * the traces of the symmetric product S P M P S formed on that half (the
 * CG step's cubics, Sec. II.C.2).  Without them these products are formed
 * in full.
 */
typedef struct lnv_eval_ws {
  lnv_bsm SL;
  lnv_bsm LS;
  lnv_bsm X;
  lnv_bsm XT;
  lnv_bsm Z;
  const int32_t* perm_SL;
  const int32_t* perm_X;
  double* YT;
  double* W;
  double* V;
  double* partials;
  int64_t partials_len;
  double* scalars;
  lnv_bsm Zu;
  lnv_bsm Lu;
  void* Vu;
  /* Host flag, owned by the library: nonzero while SL2 of the enclosing
   * lnv_cg_ws and Z hold S.L and S.L.S of the L that the last lnv_cg_step
   * on this workspace left (see lnv_cg_step).  lnv_cg_step sets it;
   * lnv_eval, lnv_hotelling and lnv_cg_init on this workspace clear it.  A
   * caller that changes L or S (or the buffers) itself between steps must
   * clear it, or restart with k = 0.  Initialise to 0.
 * Sizing helper (library infrastructure).
 */
  int32_t carry;
} lnv_eval_ws;

#define LNV_NSLOTS 12
int64_t lnv_partials_len(int32_t n_items_L);

/* Device scalar block (doubles). */
enum {
  LNV_SC_E = 0, LNV_SC_N = 1, LNV_SC_MU = 2, LNV_SC_BETA = 3, LNV_SC_ALPHA = 4,
  LNV_SC_DELTA = 5, LNV_SC_FF = 6, LNV_SC_GG = 7, LNV_SC_C1 = 8, LNV_SC_C2 = 9,
  LNV_SC_C3 = 10, LNV_SC_N0 = 11, LNV_SC_N1 = 12, LNV_SC_N2 = 13, LNV_SC_N3 = 14,
  LNV_SC_FORCE_RESET = 15, LNV_SC_SKIP_NCORR = 16, LNV_SC_GNORM = 17,
  LNV_SC_N_AFTER = 18, LNV_SC_LAMBDA = 19, LNV_SC_STATUS = 20, LNV_SC_LL = 21,
  LNV_SC_GF = 22, LNV_SC_DF = 23, LNV_SC_T0 = 24, LNV_SC_T1 = 25, LNV_SC_T2 = 26,
  LNV_SC_T3 = 27, LNV_SC_T4 = 28, LNV_SC_T5 = 29, LNV_SC_GG_PREV = 30,
  LNV_SC_GGP = 31, LNV_SC_FCFC = 32, LNV_SC_SIGMA = 33, LNV_SC_GGN = 34,
  LNV_SC_NCORR = 35,  /* electron-number corrections computed (never reset by the library) */
  LNV_SC_E_PREV = 36,   /* runaway guard: E of the previous iteration (NaN after a start) */
  LNV_SC_RISES = 37,    /* consecutive rises of E */
  LNV_SC_GUARD_K = 38,  /* iteration of the last guard trip */
  LNV_SC_OCC_MIN = 39,  /* occupation bounds of L S from the last check */
  LNV_SC_OCC_MAX = 40,
  LNV_NSCALARS = 48
};
/* LNV_SC_STATUS bits set by the device (sticky until cleared by the caller).
 * LNV_ST_GUARD: the runaway guard restarted the direction at least once;
 * LNV_ST_RUNAWAY: it tripped twice within one reset period -- the
 * minimisation is running away and should be stopped (lnv_cg_check). */
enum {
  LNV_ST_NONFINITE = 1, LNV_ST_NO_ALPHA = 2, LNV_ST_NO_DELTA = 4, LNV_ST_DELTA_CAPPED = 8,
  LNV_ST_GUARD = 16, LNV_ST_RUNAWAY = 32
};

/*
 * lnv_eval -- E, N (written to EN[0], EN[1], device, and to
 * scalars[LNV_SC_E/N]), G = dE/dL and F = dN/dL on L's pattern.  L, S, H,
 * G, F are FP64 with blk 4; L's pattern needs its index and items, S's needs its index.
 * Hot path: allocates nothing, no host synchronisation.
 * Sec. II.C.2, Eq. (4).
 */
int lnv_eval(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, lnv_bsm* G,
             lnv_bsm* F, double* EN, lnv_eval_ws* ws, hipStream_t s);

/* ------------------------------------------------------------ batches of cells
 * A batch of independent periodic cells is one block-diagonal system: the
 * rows of cell c are cell_start[c] .. cell_start[c+1]-1 (cell_of[row] = c),
 * its box is boxes[3c .. 3c+2] and its master seed seeds[c].  Every kernel of
 * the evaluation then serves all cells in one launch per product; only the
 * range patterns, the synthetic matrices and the traces need the cells.
 *
 * lnv_neighbours_cells -- lnv_neighbours with each row tested only against
 * the rows of its own cell, in its cell's box (device arrays: cell_start
 * [n_cells+1], cell_of [n], boxes [n_cells*3]).  Same two-phase protocol.
 * Ranges of Sec. II.C.2 applied per cell; batching itself is not in the paper.
 */
int lnv_neighbours_cells(const double* pos, int32_t n, int32_t n_cells,
                         const int32_t* cell_start, const int32_t* cell_of, const double* boxes,
                         double R, int32_t* row_ptr, int32_t* col, int64_t cap,
                         int64_t* nnz_out, hipStream_t s);

/* lnv_synth_blocks_cells -- lnv_synth_blocks for a batch: row i uses its
 * cell's box and seed (cell_of, boxes, seeds: device), atom_of[i] is the
 * row's atom index within its cell (the counter key), fun_of[i] that atom's
 * function count and off_of[i] the row's first function (all device [n]).
 * As lnv_synth_blocks (Sec. II.B stand-ins), per cell.
 */
int lnv_synth_blocks_cells(const double* pos, const int32_t* cell_of, const double* boxes,
                           const uint64_t* seeds, const int32_t* atom_of, const int32_t* fun_of,
                           const int32_t* off_of, const lnv_bsm* M, int32_t kind, double R,
                           double decay, double scale, hipStream_t s);

/* lnv_cell_traces -- per-cell E and N (EN_cells[2c], EN_cells[2c+1], device)
 * from the trace partials that lnv_eval or lnv_eval_mixed left in
 * ws->partials; call it right after that evaluation, on the same stream and
 * workspace.  cell_item_ptr (device [n_cells+1]): the work items of L's
 * pattern that belong to each cell (items are in row order, so each cell's
 * items are one range).  Fixed reduction order.
 * Per-cell E = 2 Tr[KH] and N = 2 Tr[KS] (Sec. II.C.2).
 */
int lnv_cell_traces(const lnv_pattern* PL, const lnv_eval_ws* ws, int32_t n_cells,
                    const int32_t* cell_item_ptr, double* EN_cells, hipStream_t s);

/* ------------------------------------------------------------ a3/a4 mixed precision
 * lnv_eval_mixed -- lnv_eval with the six block products in FP32 (FP32
 * multiply-add, FP32 accumulation) and everything else in FP64: L, S and H
 * are FP64 and are rounded to FP32 copies by the call; the assembly of G and
 * F reads the FP32 intermediates and forms G, F, E, N and every trace in
 * FP64, with the FP64 L on the left of each trace.  The workspace mirrors
 * lnv_eval_ws with FP32 values (same patterns and tables):
 *  L, S, H   FP32 copies on L's, S's and H's pattern objects (written)
 *  SL .. Z   FP32 intermediates, patterns as in lnv_eval_ws
 *  YT, W, V  device [nnzb_L * 16] FP32
 * G, F FP64 on L's pattern.  Hot path: allocates nothing.
 */
typedef struct lnv_eval32_ws {
  lnv_bsm L;
  lnv_bsm S;
  lnv_bsm H;
  lnv_bsm SL;
  lnv_bsm LS;
  lnv_bsm X;
  lnv_bsm XT;
  lnv_bsm Z;
  const int32_t* perm_SL;
  const int32_t* perm_X;
  float* YT;
  float* W;
  float* V;
  double* partials;
  int64_t partials_len;
  double* scalars;
  lnv_bsm Zu;   /* optional half products, as in lnv_eval_ws (FP32)
 * Sec. II.C.2, Eq. (4), with FP32 products (not in the paper).
 */
  lnv_bsm Lu;
  void* Vu;
} lnv_eval32_ws;

int lnv_eval_mixed(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, lnv_bsm* G,
                   lnv_bsm* F, double* EN, const lnv_eval32_ws* ws, hipStream_t s);

/* ------------------------------------------------------------ adjoint
 * lnv_adjoint -- derivatives of E = 2 Tr[KH], K = 3LSL - 2LSLSL (Sec. II.C.2,
 * Eq. 4), with respect to each stored entry of H and of S at fixed L:
 *   dH = dE/dH = 2 K on H's pattern          = P_H(6 L.SL - 4 LSL.SL)
 *   dS = dE/dS = 2 [3 LHL - 2 (LSLHL + LHLSL)] on S's pattern
 *              = P_S(6 L.HL) - 4 (Y + Y^T),  Y = P_S(LSL.HL)
 * (dE/dL is lnv_eval's G).  L, S and H must be symmetric and stored in both
 * triangles, as for lnv_eval.  The natural-range intermediates are formed
 * anew on every call (nothing is carried over from lnv_eval):
 *  SL   values on pat(S.L)   (pattern needs its index and items)
 *  LSL  values on pat(L.S.L) (pattern needs items)
 *  HL   values on pat(H.L)   (pattern needs its index and items; used only for dS)
 *  YS   device [nnzb_S * 16] scratch (used only for dS)
 * dS is on S's pattern (needs its index and items), dH on H's pattern (needs
 * items); dNS = dN/dS = 12 P_S(LSL - LSLSL) on S's pattern (N = 2 Tr[KS],
 * for forces under the electron-number constraint).  Any of the three may be
 * NULL, not all.  FP64, blk 4.  Hot path: allocates nothing, no host
 * synchronisation.
 * Symmetric products (optional, val == NULL: formed in full): LSL, the
 * symmetric parts 6 LSL - 4 LSLSL of dH and 12 (LSL - LSLSL) of dN/dS, and
 * 6 LHL of dS are formed from the blocks of their halves (lnv_pattern_half)
 * and mirrored, as in lnv_eval_ws:
 *  LSLu  values on the half of pat(L.S.L)
 *  Hu    values on the half of H's pattern
 *  Su    values on the half of S's pattern
 * (each half pattern with its index, items and the cluster plan of the other
 * outputs).
 */
typedef struct lnv_adj_ws {
  lnv_bsm SL;
  lnv_bsm LSL;
  lnv_bsm HL;
  double* YS;
  lnv_bsm LSLu;
  lnv_bsm Hu;
  lnv_bsm Su;
  /* Optional (val NULL: not used): S.L transposed (values on pat(L.S), with
   * perm_SL from lnv_pattern_transpose_map(pat(S.L), pat(L.S))) and H.L
   * transposed (pat(L.H), perm_HL likewise).  With them the restricted
   * products put the shorter range on the left: P_H(LS.LSL) for P_H(LSL.SL)
   * (the same matrix L S L S L) and P_S(LH.LSL) = Y^T for Y = P_S(LSL.HL)
   * (dS takes Y + Y^T), so the contraction runs over LS's or LH's rows with
   * the natural-range L.S.L on the right, whose pattern then needs its index; the
   * left patterns need items (and the cluster plans of the other left
   * operands).
 * Forces need dE/dS and dE/dH (Sec. III.A).
 */
  lnv_bsm LS;
  const int32_t* perm_SL;
  lnv_bsm LH;
  const int32_t* perm_HL;
} lnv_adj_ws;

int lnv_adjoint(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, lnv_bsm* dS,
                lnv_bsm* dH, lnv_bsm* dNS, const lnv_adj_ws* ws, hipStream_t s);

/*
 * lnv_forces -- forces on the atoms from the synthetic matrices' dependence
 * on the positions (the paper's forces are the exact derivative of the
 * energy, Sec. III.A; here S and H depend on the positions through the image
 * weights of lnv_synth_blocks, S_ab = w_S M^S_ab + 2I, H_ab = -w_H M^H_ab):
 *   F_a = -sum over stored blocks of <GS - mu GNS, dS/dx_a> + <GH, dH/dx_a>
 * with dw/dx_a = sum_T exp(-d_T/decay)/decay (x_b - x_a + T)/d_T over the
 * in-range images.  GS = dE/dS and GH = dE/dH (lnv_adjoint) give -dE/dx at
 * fixed L; with GNS = dN/dS and mu the chemical potential of a minimum under
 * N = N_e, the force of that constrained minimum.  GNS may be NULL.
 *  pos, box, nfun, atom_of, off_of, seed, scale: as given to lnv_synth_blocks
 *  GS, GNS on S's pattern, GH on H's pattern (FP64; patterns need index)
 *  seg_ptr, seg_atom (device [n_seg+1], [n_seg]): atom seg_atom[s] owns the
 *      stored rows seg_ptr[s] .. seg_ptr[s+1]-1
 *  acc: device [3 n] scratch;  F: device [3 n_atoms] output (Hartree/bohr)
 * Fixed summation order.  Hot path for molecular dynamics: allocates nothing.
 */
int lnv_forces(const double* pos, const double* box, const int32_t* nfun,
               const int32_t* atom_of, const int32_t* off_of, uint64_t seed, double scale,
               const lnv_bsm* GS, const lnv_bsm* GNS, double mu, double R_S, double decay_S,
               const lnv_bsm* GH, double R_H, double decay_H, int32_t n_seg,
               const int32_t* seg_ptr, const int32_t* seg_atom, double* acc, double* F,
               hipStream_t s);

/* lnv_occupation_bounds -- bounds of the occupation numbers, the
 * eigenvalues of L S (K = 3LSL - 2LSLSL of Sec. II.C.2 is idempotent when
 * they are 0 or 1; the McWeeny form runs away outside [0, 1]): the extreme
 * eigenvalues of the tridiagonal matrix of `steps` (1..64) Lanczos steps on
 * L S in the inner product x^T S y, from a fixed pseudo-random start.  They
 * lie inside the spectrum and approach its ends as steps grow.  out: device
 * [2] (smallest, largest; NaN for a zero start in the S norm); work: device
 * [lnv_lanczos_len(n)].  FP64, blk 4.  Hot path: allocates nothing, no host
 * synchronisation. */
int64_t lnv_lanczos_len(int32_t n_rows);
int lnv_occupation_bounds(const lnv_bsm* L, const lnv_bsm* S, int32_t steps, double* work,
                          double* out, hipStream_t s);

/* lnv_cg_check -- synchronise s and report the sticky status of a
 * minimisation (scalars: device [LNV_NSCALARS]): LNV_ENUMERIC when
 * LNV_ST_NONFINITE or LNV_ST_RUNAWAY is set, else LNV_OK; *status_out
 * (host, may be NULL) receives the bits.
 * Guards the minimisation of Sec. II.C.2 (weak idempotency: occupations in [0, 1]).
 */
int lnv_cg_check(const double* scalars, int32_t* status_out, hipStream_t s);

/* ------------------------------------------------------------ a5-a7: CG
 * Buffers of the conjugate-gradient minimisation (all on L's pattern unless
 * stated).  gc/gc_prev (metric runs) or g/gc_prev (identity metric) and
 * D/D_prev are swapped by lnv_cg_step after each step.
 *  LL  values on pat(L.L) (pattern needs items): G T and F T of the metric
 *      products P_L(T (G T)), P_L(T (F T)) when the pattern has its index (T G and
 *      T F of P_L((T G) T) otherwise: the same triples, but the restricted
 *      product then contracts over the long rows of T G).  May share memory
 *      with ev.XT (dead at that point) when pat(L.L) has no more blocks than
 *      pat(S.L.H).  Unused without a metric.
 */
typedef struct lnv_cg_ws {
  lnv_eval_ws ev;
  lnv_bsm LL;
  double* SL2;     /* second value buffer on pat(S.L) */
  double* Hp;      /* [nnzb_H * 16]: H - mu S */
  double* G;
  double* F;
  double* Gc;      /* P_L(T G T) (metric runs) */
  double* Fc;      /* P_L(T F T) (metric runs) */
  double* g;
  double* gc;      /* metric runs */
  double* gc_prev;
  double* D;
  double* D_prev;
  double* lanczos; /* device [lnv_lanczos_len(n)] or NULL (no occupation checks) */
} lnv_cg_ws;

typedef struct lnv_opts {
  int32_t reset_period;  /* search direction reset period (40) */
  double n_tol;          /* relative electron-number tolerance (1e-11) */
  double step_cap;       /* max |delta| ||F_c|| / ||L|| of the N correction (0.1) */
  /* NULL: the step's evaluation (E, N, G, F) in FP64.  Otherwise it runs as
   * lnv_eval_mixed on this workspace (FP32 block products under the FP32
   * accumulation mode, FP64 assembly and traces; its partials and scalars
   * are not used: the step's own are), and S.L is widened to FP64 from the
   * FP32 product for the line search.  With a metric, P_L(T G T) and
   * P_L(T F T) (the preconditioner) are formed in FP32 as well, in the
   * workspace's buffers after the evaluation has used them (its pattern of
   * X must hold pat(L.L), which then needs its index, and Lu, Vu must be set;
   * otherwise they stay FP64).  The line search, the electron-number check
   * and correction stay FP64. */
  const struct lnv_eval32_ws* eval32;
  /* Runaway guard (always on): two consecutive rises of E by more than
   * 1e-11 |E|, or occupation bounds of L S outside [-0.5, 1.5], restart the
   * direction (beta = 0, LNV_ST_GUARD); a second trip within reset_period
   * iterations sets LNV_ST_RUNAWAY.  Occupation bounds (lnv_occupation_bounds,
   * occ_iter Lanczos steps, 1..64) are taken every occ_every-th iteration
   * (0: never) when the workspace has lanczos, into LNV_SC_OCC_MIN/MAX. */
  int32_t occ_every;
  int32_t occ_iter;
} lnv_opts;

/*
 * lnv_hotelling -- sparse approximate inverse of the overlap on T's pattern,
 * (identity of the orbitals present, as in lnv_cg_init; S's pattern needs its index),
 * the metric of the minimisation (Sec. II.C.2 uses an approximate sparse
 * S^-1 from Hotelling's iteration):  T0 = sigma I with
 * sigma = 1 / max_a sum_b |S_ab| (a Gershgorin bound, so ||I - T0 S|| < 1),
 * T_{n+1} = P_T(2 T_n - T_n S T_n), n_iter steps.  T's pattern (L's in the
 * CG) needs its index and items; scratch: ws->ev.SL (pattern pat(S.T) with its index and
 * items), ws->Gc, ws->ev.partials, ws->ev.scalars (sigma in LNV_SC_SIGMA).
 */
int lnv_hotelling(const lnv_bsm* S, lnv_bsm* T, int32_t n_iter, lnv_cg_ws* ws, hipStream_t s);

/* ------------------------------------------------------------ canonical purification
 * The start of the minimisation (Sec. II.C.2 generates the initial density
 * matrix from H by a generalisation of the McWeeny transform: canonical
 * purification with the approximate inverse overlap T).  With rho = K S,
 * theta = n_elec/2 occupied states of n_orb orbitals (functions present):
 *   start  K0 = (lambda/n)(mu T - P_L(T H T)) + (theta/n) T,  mu = <T, H>/n,
 *          lambda = min(theta/(b - mu), (n - theta)/(mu + b)), b = ||T||inf ||H||inf
 *   step   t_p = Tr[rho^p] = <K (S K)^(p-1), S>,  c = (t2 - t3)/(t1 - t2),
 *          K <- ((1 + c) KSK - KSKSK)/c (c >= 1/2),
 *          ((1 - 2c) K + (1 + c) KSK - KSKSK)/(1 - c) (c < 1/2),
 *          KSK = P_L(K.SK), KSKSK = P_L(KSK.SK), then K <- (K + K^T)/2
 *   stop   (K kept) when t1 - t2 <= tol theta, c is undefined or outside
 *          [0, 1], or t1 - t2 grew (truncation pushes the spectrum out of
 *          [0, 1]); later steps do nothing.
 * Every scalar decision is taken on the device: a caller runs as many steps
 * as it allows without synchronising and reads the history afterwards.
 * Workspace (device memory, caller-owned):
 *  SK         values on pat(S.L) (pattern with its items and cluster plan)
 *  K2, K3, KT [nnzb_L * 16] FP64 on L's pattern
 *  perm_L     L's transpose map onto itself (lnv_pattern_transpose_map)
 *  partials   [lnv_partials_len(L's work items)] FP64
 *  scalars    [LNV_PM_NSCALARS] FP64 (LNV_PM_*)
 *  hist       [4 * hist_len] FP64: per step (c, t1, t2, t3), c = NaN for the
 *             step that stopped; LNV_PM_STEPS entries are written
 * L's pattern needs its index, items and cluster plan; S's and H's their
 * indices; FP64, blk 4.
 */
enum {
  LNV_PM_MU = 0, LNV_PM_B = 1, LNV_PM_LAMBDA = 2, LNV_PM_DOT = 3, LNV_PM_NT = 4, LNV_PM_NH = 5,
  LNV_PM_T1 = 6, LNV_PM_T2 = 7, LNV_PM_T3 = 8, LNV_PM_C = 9, LNV_PM_PREV = 10,
  LNV_PM_STOPPED = 11, LNV_PM_STEPS = 12, LNV_PM_A0 = 13, LNV_PM_A1 = 14, LNV_PM_A2 = 15,
  LNV_PM_HALF = 16, LNV_PM_NSCALARS = 32
};
typedef struct lnv_pm_ws {
  lnv_bsm SK;
  double* K2;
  double* K3;
  double* KT;
  const int32_t* perm_L;
  double* partials;
  int64_t partials_len;
  double* scalars;
  double* hist;
  int32_t hist_len;
} lnv_pm_ws;

/* lnv_pm_start -- K0 into K (on L's pattern) from T (on L's pattern) and H;
 * HT: scratch values on pat(H.L) (pattern with its index, items and cluster
 * plan), H.T.  Resets the step counter and history.  First iterate of the
 * canonical purification that starts the minimisation (Sec. II.C.2). */
int lnv_pm_start(lnv_bsm* K, const lnv_bsm* T, const lnv_bsm* H, lnv_bsm* HT, double n_orb,
                 double n_elec, lnv_pm_ws* ws, hipStream_t s);

/* lnv_pm_step -- one purification step of K (no-op once stopped or after
 * hist_len steps).  n_elec and tol as for the start and stop rule.  The
 * generalised McWeeny step of the canonical purification (Sec. II.C.2). */
int lnv_pm_step(lnv_bsm* K, const lnv_bsm* S, double n_elec, double tol, lnv_pm_ws* ws,
                hipStream_t s);

/*
 * lnv_cg_init -- L0 = lambda * T on L's pattern (T = NULL: the identity),
 * lambda the smallest positive real root of N(lambda T) = n_elec, a cubic in
 * lambda (6 Tr[TSTS] l^2 - 4 Tr[TSTSTS] l^3 = n_elec).  The paper starts
 * from a generalised McWeeny purification of H; the scaled metric is the
 * start used here.  Writes L and scalars[LNV_SC_LAMBDA].  The identity is
 * that of the orbitals present: diagonal entries whose S_aa is zero (padded
 * rows, see lnv_synth_blocks) are left at zero, and so stay zero through the
 * CG (their gradient vanishes).  S's pattern needs its index.
 * Start of the minimisation of Sec. II.C.2.
 */
int lnv_cg_init(lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* T, double n_elec, lnv_cg_ws* ws,
                hipStream_t s);

/*
 * lnv_cg_step -- one conjugate-gradient iteration k (0-based) at the current L,
 * with metric T (NULL: identity; otherwise on L's pattern, e.g. from
 * lnv_hotelling):
 *  1. E, N, G, F = eval(L);  G_c = P_L(T G T), F_c = P_L(T F T)
 *  2. mu = <G,F_c>/<F,F_c>;  g = G - mu F;  g_c = G_c - mu F_c
 *  3. beta = 0 if k % reset_period == 0 or the previous line search failed,
 *     else max(0, <g, g_c - g_c_prev> / <g_prev, g_c_prev>)  (Polak-Ribiere)
 *  4. D = -g_c + beta D_prev;  D <- D - (<D,F>/<F,F_c>) F_c
 *  5. alpha = local minimiser of the exact cubic (E - mu N)(L + alpha D)
 *     (none: alpha = 0 and a reset at the next step);  L += alpha D
 *  6. if |N(L) - N_e| > n_tol N_e: delta = smallest-|delta| real root of
 *     N(L + delta F_c) = N_e, applied when |delta| ||F_c|| <= step_cap ||L||
 * Sec. V.C (density-matrix minimisation of gramicidin A) resets the search
 * direction every 40 iterations; the other choices are readings of the
 * method's electron-number constraint (Sec. II.C.2).  Every decision is
 * taken on the device: the call never synchronises.  Diagnostics are in
 * scalars (E, N at the start of the step, mu, beta, alpha, delta, ...).
 * For k > 0, L must be the previous call's result (as the direction
 * history already assumes; restart with k = 0 after changing L), and S and
 * the workspace must be unchanged since that call: the step leaves S.L of
 * its final L in ws->SL2 (S.L_new = S.L + alpha S.D from the line search's
 * S.D, plus delta S.F_c from the correction's, by linearity) and S.L.S in
 * ws->ev.Z (the check's S.L_new.S plus delta S.F_c.S) and sets
 * ws->ev.carry.  A step with k > 0 not divisible by reset_period and
 * ws->ev.carry set starts from them: an FP64 step's evaluation forms
 * neither S.L nor S.L.S, and a mixed step (opts->eval32) takes the carried
 * FP64 S.L for its line search and electron-number check.  Otherwise (a
 * reset step, or the flag cleared by another call on the workspace) both
 * are formed afresh.
 */
int lnv_cg_step(lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, const lnv_bsm* T,
                double n_elec, int64_t k, const lnv_opts* opts, lnv_cg_ws* ws, hipStream_t s);

/* ------------------------------------------------------------ batches of cells
 * lnv_batch -- many independent cells minimised together: the cells are one
 * block-diagonal system (lnv_neighbours_cells, lnv_synth_blocks_cells), every
 * block product one launch for all of them, and every scalar of the
 * minimisation (E, N, mu, beta, alpha, delta, the guard's state) taken per
 * cell.  The rows of a cell are consecutive, so its work items of L's
 * pattern and its values are ranges.  All pointers are device memory owned
 * by the caller:
 *  item_ptr  int32 [n_cells+1]: first work item of L's pattern (items are in
 *            row order) of each cell, item_ptr[n_cells] = L's n_items
 *  val_ptr   int64 [n_cells+1]: first value of each cell in L's values
 *            (16 x the first block of its first row), val_ptr[n_cells] = 16 nnzb
 *  row_cell  int32 [n_rows]: the cell of each block row
 *  n_elec    FP64 [n_cells]: electron count of each cell
 *  scalars   FP64 [n_cells * LNV_NSCALARS]: cell c's scalar block (LNV_SC_*,
 *            status bits included) at c * LNV_NSCALARS; lnv_cg_check takes
 *            one cell's block
 *  row_off   int32 [n_cells+1]: first block row of each cell
 *  n_orb     FP64 [n_cells]: orbitals (support functions present) of each cell
 * 1 <= n_cells <= 1024 (LNV_EUNSUPPORTED beyond).  The minimisation of
 * Sec. II.C.2, per cell; the paper runs one system at a time (running many
 * small systems in one launch is this library's addition).
 */
typedef struct lnv_batch {
  int32_t n_cells;
  const int32_t* item_ptr;
  const int64_t* val_ptr;
  const int32_t* row_cell;
  const double* n_elec;
  double* scalars;
  const int32_t* row_off;
  const double* n_orb;
} lnv_batch;

/* lnv_hotelling_batch -- lnv_hotelling per cell: each cell's sigma from its
 * own rows (LNV_SC_SIGMA of its scalar block), T0 = sigma_c I on its rows,
 * then the products of the iteration for all cells at once (T's pattern is
 * block diagonal).  Workspace as for lnv_hotelling.  The metric of
 * Sec. II.C.2, per cell. */
int lnv_hotelling_batch(const lnv_bsm* S, lnv_bsm* T, int32_t n_iter, const lnv_batch* b,
                        lnv_cg_ws* ws, hipStream_t s);

/* lnv_pm_start_batch, lnv_pm_step_batch -- canonical purification per cell
 * (lnv_pm_start, lnv_pm_step) with each cell's n_orb, n_elec, mu, b, lambda,
 * c and stopping test; ws->scalars holds n_cells blocks of LNV_PM_NSCALARS
 * and ws->hist n_cells blocks of 4 hist_len (cell c's at c times the block).
 * Every launch runs for all cells: a cell that has stopped takes the update
 * coefficients (1, 0, 0), which leave its K unchanged.  The start of
 * Sec. II.C.2, per cell. */
int lnv_pm_start_batch(lnv_bsm* K, const lnv_bsm* T, const lnv_bsm* H, lnv_bsm* HT,
                       const lnv_batch* b, lnv_pm_ws* ws, hipStream_t s);
int lnv_pm_step_batch(lnv_bsm* K, const lnv_bsm* S, const lnv_batch* b, double tol,
                      lnv_pm_ws* ws, hipStream_t s);

/* lnv_cg_init_batch -- lnv_cg_init per cell: L0 = lambda_c T (T = NULL: the
 * identity) on each cell's rows, lambda_c the smallest positive root of that
 * cell's N(lambda T) = n_elec[c].  Clears every cell's scalar block but its
 * sigma (the correction counter too) and the direction history; writes L
 * and LNV_SC_LAMBDA per cell.  Workspace as for lnv_cg_init (S's pattern
 * needs its index).  Start of the minimisation of Sec. II.C.2, per cell.
 */
int lnv_cg_init_batch(lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* T, const lnv_batch* b,
                      lnv_cg_ws* ws, hipStream_t s);

/* lnv_cg_step_batch -- lnv_cg_step (FP64, metric T or the identity) for every
 * cell of a batch at once: the six products of the evaluation, the metric's,
 * the line search's and the electron-number check's and correction's
 * products are one launch each for all cells; the traces are reduced per
 * cell (fixed order) and mu, beta, alpha, the check and delta are taken per
 * cell (a cell within the electron-number tolerance keeps delta = 0 while
 * others are corrected).  Differences from lnv_cg_step: no mixed-precision
 * evaluation (opts->eval32 must be NULL: LNV_EUNSUPPORTED), no occupation
 * bounds (the E-rise guard stays), S.L and S.L.S formed afresh every step,
 * and the traces of the line search taken from stored products (a
 * product's fused trace partials cover row clusters that may straddle two
 * cells).  The workspace is lnv_cg_step's (ev.YT and ev.W serve as product
 * scratch).  For k > 0, L and the workspace must be those the previous step
 * left.  Sec. II.C.2 / Sec. V.C as lnv_cg_step, per cell.
 */
int lnv_cg_step_batch(lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, const lnv_bsm* T,
                      const lnv_batch* b, int64_t k, const lnv_opts* opts, lnv_cg_ws* ws,
                      hipStream_t s);

/* ------------------------------------------------------------ timing
 * Optional HIP-event timing of the block multiply kernel: while enabled,
 * every multiply launch is bracketed by events on its stream.
 * lnv_timing_read synchronises the recorded events and returns the summed
 * kernel time (ms) and launch count since the last reset.
 * Library infrastructure (measurement).
 */
int lnv_timing_enable(int32_t on);
int lnv_timing_read(double* ms_total, int64_t* launches);
int lnv_timing_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* LNV_H */
