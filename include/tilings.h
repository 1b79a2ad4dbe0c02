/*
 * tilings.h -- C-ABI of the MI355X (gfx950) Glauber-sweep library for random
 * tilings: domino tilings of Aztec diamonds, lozenge tilings of hexagons and the
 * six-vertex model with domain-wall boundary (Keating & Sridhar, "Random Tilings
 * with the GPU", arXiv:1804.07250).
 *
 * The library implements the domain-decomposed Markov chain of Section 1.1.3,
 * eq. (1.1): the sites are coloured so that sites of one colour never
 * interact, and one colour step applies the local move of every site of that
 * colour at once (Section 1.1.2 "admissible clusters"; Section 1.2 for the
 * lozenge 3-colouring and the six-vertex 4-colouring).  A sweep visits the
 * colours 0..K-1 in order.  Every random draw is a pure function of
 * (seed, sweep, colour, site) through Philox4x32-10, so results do not depend
 * on how the work is tiled, launched or batched.
 *
 * Conventions shared by every entry point:
 *   - all functions return a tl_status (TL_OK == 0, errors < 0) and never
 *     throw; tl_last_error() returns a thread-local message for the last error;
 *   - handles are not thread-safe; each sampler owns one HIP stream (its own,
 *     or the caller's through tl_options.stream);
 *   - sweeps are asynchronous (stream ordered); observables, export, import,
 *     hash and sync synchronise the sampler's stream;
 *   - host buffers are owned by the caller; device state is owned by the
 *     library and freed by tl_sampler_destroy.
 */
#ifndef TILINGS_H
#define TILINGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TL_OK = 0,
    TL_EINVAL = -1,       /* invalid argument: shape, size, weights <= 0 or NaN, buffer size */
    TL_EUNTILEABLE = -2,  /* the domain has no tiling */
    TL_ENOMEM = -3,       /* device or host allocation failed */
    TL_EBUDGET = -4,      /* request exceeds the memory budget of a server */
    TL_EDEVICE = -5,      /* a HIP call failed (message in tl_last_error) */
    TL_EBUSY = -6         /* result not ready yet */
} tl_status;

typedef enum { TL_DOMINO = 0, TL_LOZENGE = 1, TL_SIXVERTEX = 2 } tl_model;
typedef enum { TL_AZTEC = 0, TL_HEXAGON = 1, TL_DWBC_SQUARE = 2, TL_MASK = 3 } tl_shape;
/* Extremal start: Aztec domino MIN = all-horizontal brick tiling, MAX = all-vertical;
 * domino domain given by a mask: MIN = T_min, MAX = T_max of its height order (see
 * TL_MASK below); lozenge MIN = empty box, MAX = full box; six-vertex MIN = |I-J|,
 * MAX = N-|I+J-N|. */
typedef enum { TL_INIT_MIN = 0, TL_INIT_MAX = 1 } tl_init;
typedef enum { TL_HEATBATH = 0, TL_METROPOLIS = 1 } tl_rule;
typedef enum {
    TL_W_UNIFORM = 0,       /* all weights 1 (Section 1.1.1, last sentence) */
    TL_W_TWO_PERIODIC = 1,  /* domino edge weights: w[0] = a, w[1] = b (see below) */
    TL_W_VOLUME = 2,        /* lozenge volume weight q^volume: q = w[0], or w[0]/w[1] if w[1] > 0 */
    TL_W_SIXVERTEX = 3,     /* six-vertex vertex weights, squared: w[0] = a^2, w[1] = b^2, w[2] = c^2 */
    TL_W_VOLUME_BW = 4,     /* domino volume weights prod_v q_v^h(v): q = w[0]/w[1] on black vertices
                             * (x+y even), w[2]/w[3] on white ones (a zero denominator reads as 1) */
    TL_W_SIXVERTEX6 = 5     /* six-vertex weights of the six vertex types: w = a1, a2, b1, b2, c1, c2
                             * (a1: no path edge, a2: all four, b1: left+right, b2: bottom+top,
                             * c1: bottom+left, c2: right+top); with the boundary fixed the chain
                             * depends on them through a1 a2, b1 b2, c1 c2 only */
} tl_weight_kind;

/* Domain (Section 1.1 "domain"; Section 1.2):
 *   TL_DOMINO    + TL_AZTEC:       Aztec diamond of order n (faces [x,x+1]x[y,y+1]
 *                                  with |2x+1|+|2y+1| <= 2n), 1 <= n <= 16384;
 *   TL_DOMINO    + TL_MASK:        any simply-connected domain (Section 1.1): the faces
 *                                  (x, y) of a w x h box with mask[y*w + x] != 0, row 0
 *                                  southmost; w, h >= 1, w + h <= 32768;
 *   TL_SIXVERTEX + TL_MASK:        the six-vertex model on a simply-connected domain whose
 *                                  vertices are the cells (x, y) with mask[y*w + x] != 0,
 *                                  domain-wall type boundary (below); w, h <= 32767;
 *   TL_LOZENGE   + TL_MASK:        lozenge tilings of a simply-connected union of unit
 *                                  triangles: mask[(y*w + x)*2 + t] != 0 selects triangle t
 *                                  of square (x, y) of the sheared box, t = 0 the lower-right
 *                                  {(x,y),(x+1,y),(x+1,y+1)}, t = 1 the upper-left
 *                                  {(x,y),(x,y+1),(x+1,y+1)}; w + h <= 32766;
 *   TL_LOZENGE   + TL_HEXAGON:     hexagon with sides a, b, c >= 1, a+c and b+c <= 32767;
 *   TL_SIXVERTEX + TL_DWBC_SQUARE: N x N vertices, domain-wall boundary, 1 <= n <= 32767.
 *
 * TL_MASK.  The mask (host memory, h*w bytes) is read during tl_sampler_create
 * only; the sampler keeps a copy.  The domain must be non-empty, connected through
 * edges, without a vertex where exactly two diagonally opposite faces belong to it,
 * and without holes (TL_EINVAL otherwise); a domain without tilings gives
 * TL_EUNTILEABLE (Thurston's test, Section 1.1).  The chain runs on the Aztec
 * diamond of order n = ceil((w+h)/2) that holds the box at face offset (ox, oy),
 * ox + oy = n, ox - oy = D with m = floor((h-w)/2), D = m if m - n is even, else
 * m - 1; its faces outside the domain stay uncovered, and the draws of a site are
 * those of the same site of that diamond.  Heights: a face of the diamond's box is
 * black when its coordinates sum to an even number; across an edge walked with a
 * black face on its left the height rises by 1 (edge of a domino) or falls by 3
 * (edge covered by a domino).  T_max / T_min are the tilings of largest / smallest
 * height.  Exports and observables use the w x h box (0xFF outside the domain).
 *
 * Height-model masks keep the draws, colours and moves of their fixed shapes,
 * with heights on the (w+1) x (h+1) corner points (export: int32, INT32_MIN off
 * the domain); the sites are the points whose cells (six-vertex: four;
 * lozenge: six triangles) all lie in the domain, the other points of the
 * domain are fixed.  Six-vertex: legs through the south and west sides of cells
 * carry paths, legs through the north and east sides are empty (the N x N mask
 * is the domain-wall square); the lowest, then leftmost, point has height
 * (I + J) mod 2; extremes h_max / h_min; observables: type-c cells of the w x h
 * box.  Lozenge: Thurston's heights 3H + X + Y fix the boundary; T_max / T_min
 * are normalised so that the smallest H of T_min is 0 (the hexagon's triangles
 * give the hexagon exactly); observables: H - H_min at the (w+1) x (h+1)
 * points.  Either: TL_EUNTILEABLE when no state meets the boundary.
 * Batches take domino masks, servers masks of every model. */
typedef struct {
    int32_t model;   /* tl_model */
    int32_t shape;   /* tl_shape */
    int32_t n;       /* Aztec order / six-vertex N */
    int32_t a, b, c; /* hexagon sides */
    int32_t init;    /* tl_init */
    int32_t w, h;    /* TL_MASK: box of the mask, in faces */
    const uint8_t *mask; /* TL_MASK: h rows of w bytes, nonzero = face in the domain */
    uint32_t flags;  /* one TL_FREE_* side (six-vertex masks only), else 0 */
} tl_domain;

/* Free boundary (Section 1.2: boundary faces need variations of the c-flip).
 * One of TL_FREE_NORTH, TL_FREE_SOUTH, TL_FREE_EAST, TL_FREE_WEST leaves the
 * legs through that side of the cells of a six-vertex mask free instead of
 * fixed: the boundary points all of whose boundary edges are such sides move
 * too, flipping when their three other neighbours share a height m.  Such a
 * flip changes only the two cells beside those neighbours' edges, so it has
 * its own table over the context (first diagonal at m+1) + 2 (second diagonal
 * at m+1), the diagonals being the two points beside those cells: north SW,
 * SE; south NW, NE; east SW, NW; west SE, NE; built from all six weights
 * (weight kinds TL_W_UNIFORM and TL_W_SIXVERTEX6 only).  The rest of the
 * boundary keeps the domain-wall type legs and must be one piece (TL_EINVAL
 * otherwise); one free side per domain.  A free south (west) side keys the
 * draws of point (I, J) as those of point (I, J + 2) ((I + 2, J)) of the
 * model's box, so that its points are inner points there (colours are those
 * of (I, J)). */
#define TL_FREE_NORTH 1u
#define TL_FREE_SOUTH 2u
#define TL_FREE_EAST 4u
#define TL_FREE_WEST 8u

/* Weights (Section 1.1.1 edge and volume weights; Section 1.2 vertex weights).
 * Two-periodic: a crossed edge weighs a when its even endpoint (x+y even in
 * centred coordinates) has x even, b otherwise.  Domino volume weights: a
 * rotation changes the height at its vertex by 4, up (vertical pair) raising
 * it at black vertices and lowering it at white ones, so P(vertical) is
 * q^4/(1+q^4) at a black site and 1/(1+q^4) at a white one.  Six-vertex: corners NE/SW of a
 * flipped face carry a, NW/SE carry b, type-c corners carry c; a flip changes
 * four corners, a and b each at two of them, so the chain depends on a^2, b^2
 * and c^2 only, which are passed exactly (c = sqrt(2) as c^2 = 2).  Acceptance uses
 * uint32 thresholds T = floor(2^32 p) (rule TL_HEATBATH: p = W_up/(W_up+W_down);
 * TL_METROPOLIS: lazy Metropolis, p = min(1, W_new/W_old)/2). */
typedef struct {
    int32_t kind;  /* tl_weight_kind */
    int32_t rule;  /* tl_rule */
    double w[6];
} tl_weights;

typedef struct {
    void *stream;                /* hipStream_t to run on; NULL = a stream owned by the sampler */
    uint32_t obs_every;          /* accumulate observables after sweep t when (t+1) % obs_every == 0; 0 = never */
    uint32_t obs_bin;            /* observable bin edge in cells (0 or 1 = per cell) */
    uint32_t sweeps_per_launch;  /* sweeps fused in one launch of the tiled kernel; 0 = automatic */
    uint32_t tile_rows;          /* tile height of the tiled kernel; 0 = automatic */
    uint32_t kernel;             /* 0 = automatic, 1 = one launch per colour step, 2 = tiled multi-sweep
                                  * with the tile in LDS, 3 = tiled with the tile in registers (dominoes:
                                  * a lane per row, a wavefront per group column, at most 64 rows with
                                  * the halo; other models run kernel 2).  Automatic: kernel 3 for
                                  * dominoes above order 128 unless tile fields are set, else kernel 2 */
    uint32_t tile_groups;        /* tile width in groups of 128 sites; 0 = automatic */
    uint32_t colour_order;       /* 0 = colours 0..K-1 in every sweep; 1 = random (see below) */
    void *device_buf;            /* samplers: caller-owned device memory for the state (NULL = the
                                  * library allocates it); at least tl_sampler_state_bytes bytes,
                                  * 256-byte aligned, kept alive until tl_sampler_destroy */
    size_t device_buf_bytes;
    const char *tune_cache;      /* samplers: path of the tile-shape cache tl_sampler_autotune
                                  * reads and appends to (NULL = none) */
} tl_options;

/* Random colour order (Section 2.2, RandomWalk: the colour of every step is
 * drawn at random).  Sweep t is the K colour steps s = K t .. K t + K - 1;
 * step s updates colour floor(K u / 2^32), u = word 0 of Philox(key = seed,
 * ctr = (s, 0, 0, 2^31)), with the site draws of sweep counter s (the per-site
 * uniform defined above with t replaced by s).  K t must stay below 2^32.
 * Samplers (plain sweeps and coupling from the past) and batches. */

/* Caller-owned state (device_buf).  A sampler created with device_buf set
 * keeps its two bit-plane buffers (the state and the spare it is swapped with
 * by the tiled kernel) in that memory instead of allocating them: buffer 0 at
 * device_buf, buffer 1 tl_sampler_state_bytes / 2 bytes further (each
 * buffer's size rounded up to a multiple of 256 bytes).  Which of the
 * two holds the current state is internal; read it with tl_sampler_export.
 * The library never frees device_buf; the caller keeps it alive, and touches
 * it on no other stream, until tl_sampler_destroy returns.  Observable bins,
 * masked-domain tables and the upper chain of coupling from the past are still
 * allocated by the library.  Errors: TL_EINVAL if device_buf_bytes is below
 * tl_sampler_state_bytes or device_buf is not 256-byte aligned; batches and
 * servers refuse device_buf (they manage their own pools). */

typedef struct tl_sampler tl_sampler;

/* Observables (cells: domino faces of the 2n x 2n box or of the mask's w x h
 * box, lozenge vertices of the (a+c+1) x (b+c+1) box, six-vertex vertices of
 * the N x N grid).  Per-cell
 * quantity: domino = face covered by a horizontal domino; lozenge = H - H_min;
 * six-vertex = vertex of type c.  Buffers are caller-owned and may be NULL. */
typedef struct {
    uint64_t sweeps;        /* out: sweeps done so far */
    uint64_t samples;       /* out: samples accumulated */
    int64_t scalar_now;     /* out: whole-domain quantity of the current state */
    int64_t scalar_sum;     /* out: sum of the whole-domain quantity over samples */
    uint32_t bins_x, bins_y;/* out: bin grid */
    uint64_t *bin_sum;      /* in/out: bins_x*bins_y sums over samples, or NULL */
    uint64_t *bin_now;      /* in/out: bins_x*bins_y sums of the current state, or NULL */
    double *bin_density;    /* in/out: bin_sum / (samples * in-domain cells of the bin), or NULL */
    size_t bin_capacity;    /* in: entries available in each non-NULL buffer */
} tl_observables;

/* Create a sampler in the extremal state of dom->init, with sweep counter 0.
 * The seed keys every draw (Philox key = (seed mod 2^32, seed >> 32)).
 * opt may be NULL.  Errors: TL_EINVAL, TL_EUNTILEABLE (TL_MASK), TL_ENOMEM,
 * TL_EDEVICE. */
tl_status tl_sampler_create(const tl_domain *dom, const tl_weights *w, uint64_t seed,
                            const tl_options *opt, tl_sampler **out);

/* Tile shape of the tiled kernel picked by measurement (a performance choice
 * only: every shape gives the same chain).  Candidates of tile height, width
 * in groups and sweeps per launch (for dominoes, in LDS and in registers) are
 * timed over probe_sweeps sweeps (0 = 50)
 * on a copy of the state, which the sampler's state and sweep counter never
 * see; the fastest is kept for the sampler's later sweeps (tile fields of its
 * options still take precedence).  With opt->tune_cache set, a shape
 * recorded there for the same model, shape, sizes, table kind, colour order
 * and device is used without probing, and a newly measured one is appended
 * (one text line per entry).  Synchronous.  Errors: TL_EINVAL, TL_ENOMEM,
 * TL_EDEVICE. */
typedef struct {
    uint32_t tile_rows, tile_groups, sweeps_per_launch;   /* 0, 0, 0: the automatic shape won */
    uint32_t candidates;     /* shapes timed (0 when taken from the cache) */
    uint32_t from_cache;     /* 1 if the shape came from the cache */
    float ms_per_sweep;      /* of the chosen shape, as measured (0 from the cache) */
    uint32_t kernel;         /* tiled kernel of the chosen shape: 2 LDS tiles, 3 register tiles */
} tl_tune_info;
tl_status tl_sampler_autotune(tl_sampler *s, uint32_t probe_sweeps, tl_tune_info *out);

/* Device bytes of a sampler's state (its two bit-plane buffers, each rounded
 * up to a multiple of 256 bytes) for this domain: the size opt->device_buf
 * must have (host only, no device work; see "Caller-owned state" above).
 * Errors: TL_EINVAL, TL_EUNTILEABLE. */
tl_status tl_sampler_state_bytes(const tl_domain *dom, size_t *bytes);

/* Enqueue n sweeps (sweeps t .. t+n-1) on the sampler's stream; returns without
 * waiting.  sweep(a); sweep(b) gives the same state as sweep(a+b). */
tl_status tl_sampler_sweep(tl_sampler *s, uint64_t n);

/* Wait for the sampler's stream. */
tl_status tl_sampler_sync(tl_sampler *s);

/* Observables of the current state and the accumulated samples (synchronous). */
tl_status tl_sampler_observables(tl_sampler *s, tl_observables *out);

/* Size in bytes of the canonical export, and its row layout (rows x row_bytes):
 * domino uint8 per face of the 2n x 2n box, or of the w x h box of a mask
 * (partner 0:N 1:S 2:E 3:W, 0xFF outside the domain); lozenge int32 H per vertex of the sheared box (INT32_MIN outside);
 * six-vertex int32 h per face of the (N+1)^2 box.  Row 0 is the southmost. */
tl_status tl_sampler_export_size(const tl_sampler *s, size_t *bytes, uint32_t *rows, uint32_t *row_bytes);

/* Copy the canonical export of the current state into a host buffer of at
 * least export_size bytes (synchronous); *sweep_out (nullable) = sweeps done. */
tl_status tl_sampler_export(tl_sampler *s, void *host, size_t bytes, uint64_t *sweep_out);

/* Canonical hash of the current state: SHA-256 over the SHA-256 digests of the
 * export's rows, computed on the device except for the last 32*rows bytes. */
tl_status tl_sampler_hash(tl_sampler *s, uint8_t digest[32]);

/* For callers that cannot allocate memory (tight serving loops, harnesses that
 * forbid hipMalloc): the same digest as tl_sampler_hash, computed without any
 * allocation.  The canonical export and the row digests are staged in a static
 * device buffer of TL_HASH_NOALLOC_SCRATCH_BYTES bytes that every GPU the
 * library runs on holds until the process ends; the row digests come back to a
 * static host buffer.  Limit: the export plus 32 bytes per row must fit in the
 * buffer, and the export may have at most 32768 rows (TL_EINVAL, with the
 * sizes in tl_last_error, otherwise; an order-2048 Aztec diamond or a 1024^3
 * hexagon fits).  Every call on a GPU shares that GPU's buffer: a lock held
 * from the first kernel until the digest is back orders the calls, so calls
 * from several threads wait for each other instead of racing, and the buffer
 * keeps the last call's contents (nothing in it needs to start at zero).
 * Synchronises the sampler's stream; runs on the sampler's device. */
#define TL_HASH_NOALLOC_SCRATCH_BYTES (40u << 20)
tl_status tl_sampler_hash_noalloc(tl_sampler *s, uint8_t digest[32]);

/* Replace the state by a canonical export (validated on the host: TL_EINVAL if
 * it is not a state of the domain) and set the sweep counter. */
tl_status tl_sampler_import(tl_sampler *s, const void *host, size_t bytes, uint64_t sweep);

/* Free the sampler and its device memory. */
tl_status tl_sampler_destroy(tl_sampler *s);

/* Return the sampler to the extremal start of its domain with sweep counter 0,
 * no accumulated samples and a new seed (device work only, asynchronous). */
tl_status tl_sampler_reset(tl_sampler *s, uint64_t seed);

/* Per-launch timing of the sweep kernels: with period p > 0, every p-th sweep
 * kernel launch carries a start/stop event pair recorded by its own dispatch
 * (p = 1 times every launch); p = 0 switches timing off. */
tl_status tl_sampler_set_timing(tl_sampler *s, int period);

/* Synchronise and report (then clear) the timed launches: total kernel time in
 * ms, number of launches, colour steps they performed, and the algorithmic
 * bytes of one colour step (the packed state read and written once). */
tl_status tl_sampler_kernel_time(tl_sampler *s, double *ms, uint64_t *launches, uint64_t *colour_steps,
                                 double *bytes_per_colour_step);

/* Number of sites (rotation locations) and colour classes of the sampler. */
tl_status tl_sampler_info(const tl_sampler *s, uint64_t *sites, uint32_t *colours);

/* Threshold table the sampler uses (for checks against exact rationals):
 * writes up to cap entries, returns the count in *count. */
tl_status tl_sampler_thresholds(const tl_sampler *s, uint32_t *out, uint32_t cap, uint32_t *count);

/* ------------------------------------------------------- coupling from the past
 * Exact sampling (Section 1.1.4; the CFTP host function of Section 2.2): two
 * chains, from the maximal and from the minimal state of the domain (domino:
 * all-vertical and all-horizontal brick; lozenge: full and empty box;
 * six-vertex: h_max and h_min), run the same sweeps from time -2^R to time 0
 * for R = 1, 2, ..., max_log2 until they end equal (compared on the device).
 * The draws of each time step stay fixed across rounds: time tau in
 * [-2^r, -2^(r-1)) uses sweep counter tau + 3 * 2^(r-1), time -1 counter 0, so
 * round R runs the counters [2^(R-1), 2^R), [2^(R-2), 2^(R-1)), ..., [1, 2),
 * [0, 1) in that order, keyed by the sampler's seed.
 * The moves must preserve the height order: heat-bath rule only, and for the
 * six-vertex model an up threshold that never decreases when a diagonal face
 * is raised (a <= c and b <= c for weights a, b, c, Section 1.2.4); otherwise
 * TL_EINVAL.  On success the sampler holds the sample, its sweep counter is
 * 2^R (later sweeps use fresh draws), accumulated samples are cleared, and
 * *out (nullable) reports R, the 2^R sweeps of the final round and the sweeps
 * run over all rounds and both chains.  If the chains have not met at
 * max_log2 (1..31), TL_EBUSY; the sampler then holds the minimal chain at time
 * 0 of the last round.  A state that fits one work-group runs up to three
 * consecutive rounds side by side (each with its own two chains, on the
 * sampler's stream and two more), checked in order of R, so the answer is the
 * same as with one round after the other; total_sweeps counts the rounds up
 * to R only.  Larger states run the rounds one after the other with a second
 * state for the maximal chain.  Synchronous. */
typedef struct {
    uint32_t log2_sweeps;   /* R of the round whose chains met */
    uint64_t sweeps;        /* 2^R */
    uint64_t total_sweeps;  /* sweeps over all rounds, both chains */
} tl_cftp_info;
tl_status tl_sampler_cftp(tl_sampler *s, uint32_t max_log2, tl_cftp_info *out);

/* ------------------------------------------------------------------ batched
 * Many independent domino chains on Aztec diamonds of uneven orders (1..512)
 * or on domains given by masks (TL_MASK, w + h <= 1024; each runs on the Aztec
 * diamond it is embedded in, as a sampler does), advanced together: each
 * tl_batch_sweep call is one persistent kernel launch (replayed from a
 * captured hipGraph) in which work-groups take whole chains, longest first,
 * and keep them in LDS for all the call's sweeps.  Chain i is keyed by
 * seeds[i], so its tiling equals the tiling of a tl_sampler with the same
 * domain, weights, seed and colour order.  One weight set and one colour
 * order (opt->colour_order, fixed or random per step) for all chains. */
typedef struct tl_batch tl_batch;

/* doms[0..n) (domino: Aztec of order <= 512, or a mask), seeds[0..n).
 * Errors: TL_EINVAL, TL_EUNTILEABLE (a mask without tilings), TL_ENOMEM,
 * TL_EDEVICE. */
tl_status tl_batch_create(int32_t n, const tl_domain *doms, const tl_weights *w, const uint64_t *seeds,
                          const tl_options *opt, tl_batch **out);
/* Pick the work-group size (256, 512 or 1024 threads) with the shortest probe
 * of probe_sweeps sweeps; only before the first sweep (the chains are then
 * returned to their start).  Outputs are nullable. */
tl_status tl_batch_autotune(tl_batch *b, uint32_t probe_sweeps, uint32_t *threads_out, float *ms_out);
/* Advance every chain by n sweeps (asynchronous). */
tl_status tl_batch_sweep(tl_batch *b, uint64_t n);
tl_status tl_batch_sync(tl_batch *b);
/* Return every chain to its start (sweep counter 0). */
tl_status tl_batch_reset(tl_batch *b);
/* Total sites, packed state bytes, work-group size and resident work-groups. */
tl_status tl_batch_info(const tl_batch *b, uint64_t *sites, uint64_t *state_bytes, uint32_t *threads,
                        uint32_t *workgroups);
/* Time each batch launch with events (enable != 0); report and clear. */
tl_status tl_batch_set_timing(tl_batch *b, int enable);
tl_status tl_batch_kernel_time(tl_batch *b, double *ms, uint64_t *launches, uint64_t *colour_steps);
/* Canonical export / hash of one chain (same formats as the sampler's: the
 * diamond's 2n x 2n box, or the mask's w x h box), and the export's size. */
tl_status tl_batch_export_size(tl_batch *b, int32_t chain, size_t *bytes, uint32_t *rows, uint32_t *row_bytes);
tl_status tl_batch_export(tl_batch *b, int32_t chain, void *host, size_t bytes);
tl_status tl_batch_hash(tl_batch *b, int32_t chain, uint8_t digest[32]);
tl_status tl_batch_destroy(tl_batch *b);

/* -------------------------------------------------------------------- served
 * A request loop with continuous batching: jobs (any model and domain) are
 * queued by tl_server_submit and admitted in arrival order by a scheduler
 * thread while the device-memory budget and the slot count allow; admitted
 * chains stay resident on the device and advance together in ticks: each tick
 * moves every resident job by tl_options.sweeps_per_launch sweeps (default 8;
 * twice that for jobs with one-bit decisions) in one launch for the height
 * models and one for dominoes, a work-group per tile of each job, so jobs that
 * arrive while others run share the GPU with them.  A finished
 * job's result is its canonical hash and whole-domain observable; its memory
 * is released at once.  A job gives the same result alone and in a mix.
 * Domains given by masks are served too (their host pre-pass runs in
 * tl_server_submit; a masked height-model domain's device tables count
 * against the budget), and opt->colour_order sets the colour order of every
 * job (fixed, or random per step as for a sampler). */
typedef struct tl_server tl_server;
typedef struct {
    uint64_t ticket;
    int32_t status;          /* TL_OK, or the error that ended the job */
    uint64_t sweeps;         /* sweeps performed */
    double t_submit;         /* seconds since server creation: submission, */
    double t_start;          /*   admission (device state created) */
    double t_done;           /*   and completion */
    uint8_t hash[32];        /* canonical hash of the final state */
    int64_t scalar_now;      /* whole-domain observable of the final state */
} tl_result;
typedef struct {
    uint64_t queued, active, admitted, completed;
    uint64_t bytes_in_use, peak_bytes;
    uint32_t peak_active;
} tl_server_counters;

/* Budget in bytes of device state (sum over resident jobs), at most max_slots
 * resident jobs; opt (nullable): sweeps_per_launch = quantum, colour_order. */
tl_status tl_server_create(size_t hbm_budget_bytes, int32_t max_slots, const tl_options *opt, tl_server **out);
/* Queue a job; TL_EBUDGET if it can never fit the budget, TL_EINVAL for an
 * invalid domain or weights.  *ticket identifies it. */
tl_status tl_server_submit(tl_server *sv, const tl_domain *dom, const tl_weights *w, uint64_t seed,
                           uint64_t n_sweeps, uint64_t *ticket);
/* Result of a finished job, TL_EBUSY while it is queued or running. */
tl_status tl_server_poll(tl_server *sv, uint64_t ticket, tl_result *out);
/* Block until the job finishes or timeout_s passes (TL_EBUSY). */
tl_status tl_server_wait(tl_server *sv, uint64_t ticket, double timeout_s, tl_result *out);
tl_status tl_server_stats(tl_server *sv, tl_server_counters *out);
/* Stop the scheduler; jobs still queued or running end with TL_EBUSY. */
tl_status tl_server_destroy(tl_server *sv);

/* Threshold table of a (domain, weights) pair without creating a sampler (host
 * only, no device work): heat-bath tables have one entry per context, lazy
 * Metropolis tables two ([ctx*2 + current state is up]).  Contexts: domino
 * 2c + (x mod 2); lozenge 0; six-vertex the mask of high diagonal faces
 * NE=1, NW=2, SW=4, SE=8, followed, for a TL_FREE_NORTH domain, by the table of
 * its free points (context (SW high) + 2 (SE high)).  Writes up to cap
 * entries, the count in *count. */
tl_status tl_thresholds(const tl_domain *dom, const tl_weights *w, uint32_t *out, uint32_t cap, uint32_t *count);

/* Extremal states of a TL_MASK domain on the host (no device work), as
 * canonical exports (caller-owned buffers of `bytes` bytes each, either may be
 * NULL): dominoes, Thurston's tileability test and T_max / T_min (Section 1.1;
 * h x w bytes, height convention stated with TL_MASK); six-vertex, h_max and
 * h_min of the domain-wall type boundary ((h+1) x (w+1) int32).  Errors:
 * TL_EINVAL (not a mask domain, bad mask, buffers too small), TL_EUNTILEABLE. */
tl_status tl_domain_extremes(const tl_domain *dom, void *max_out, void *min_out, size_t bytes);

const char *tl_status_str(tl_status st);
const char *tl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TILINGS_H */
