/*
 * pkt.h -- C ABI of libpkt, a GPU (MI355X / gfx950) truss decomposition library.
 *
 * The operation (Kabir and Madduri, "Shared-memory Graph Truss Decomposition",
 * arXiv:1707.02000, Background section): for a simple undirected graph G, the
 * support S(e) of an edge is the number of triangles containing it; the k-truss
 * is the largest subgraph in which every edge lies in at least k-2 triangles of
 * the subgraph; the trussness of an edge is the largest k whose k-truss contains
 * it.  Truss decomposition is the trussness of every edge.
 *
 * The method (PKT section, Algorithms 3-5): support by oriented triangle
 * counting with edge ids, then level-synchronous peeling -- for l = 0, 1, ...
 * the edges with support l form a frontier; every frontier edge intersects the
 * adjacency of its endpoints and lowers the support of the other two edges of
 * each triangle still present (floored at l, a triangle with two frontier edges
 * handled by the lower edge id only); edges reaching l form the next frontier,
 * until no edge is left.  trussness = final support + 2.
 *
 * Conventions for every entry point
 *   - Pointers named "device" are HIP device pointers; all others are host.
 *   - Input CSR: offsets[0] = 0, offsets non-decreasing, offsets[n] = 2m; every
 *     row strictly ascending (sorted, no duplicates); ids in [0, n); no
 *     self-loops; symmetric ((u,v) present iff (v,u) present).  Any number of
 *     connected components and isolated vertices.  m <= 2^31 - 1.
 *   - Edge order of every output: edge e is the e-th pair (u, v), u < v, in
 *     row-major order of the input CSR (rows ascending, then columns
 *     ascending) -- the lexicographic order of the pairs.
 *   - Ownership: the caller allocates and owns every buffer (inputs, outputs,
 *     workspace).  The library allocates no device memory, frees nothing and
 *     keeps no pointer after a call returns.
 *   - Work runs on `stream` (a hipStream_t; NULL = the default stream).  Calls
 *     return when the result is complete on that stream.  Calls with distinct
 *     workspaces may run concurrently.
 *   - Errors are returned as truss_status codes, never raised or aborted.  On
 *     error the output contents are unspecified but nothing outside the given
 *     buffers is written.  truss_last_error() gives a message for the calling
 *     thread's last error.
 */
#ifndef PKT_H_
#define PKT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TRUSS_OK = 0,
  TRUSS_E_ARG = 1,           /* bad argument: NULL pointer, negative size, bad option */
  TRUSS_E_NOT_SIMPLE = 2,    /* a row is not strictly ascending, or has a self-loop */
  TRUSS_E_NOT_SYMMETRIC = 3, /* (u, v) present without (v, u) */
  TRUSS_E_RANGE = 4,         /* vertex id outside [0, n), bad offsets, m too large, or (with more
                                than 2^28 - 1 edges) a vertex of degree above 2^28, whose edge
                                supports would not fit the 29-bit support field */
  TRUSS_E_WORKSPACE = 5,     /* workspace too small or misaligned (needs 256-byte alignment) */
  TRUSS_E_DEVICE = 6,        /* a HIP call failed; see truss_last_error() */
  TRUSS_E_INTERNAL = 7       /* iteration bound exceeded (a level or sub-level watchdog) */
} truss_status;

/* How each frontier round (sub-level) of the peeling is launched.  Every choice
 * gives the same trussness; only the running time differs. */
typedef enum {
  TRUSS_CHOICE_FUSED = 0,        /* one launch, 512 blocks: work prefix in LDS, items, finalize
                                    (frontiers of at most 2048 edges) */
  TRUSS_CHOICE_FUSED_NARROW = 1, /* the same with 32 blocks */
  TRUSS_CHOICE_WIDE = 2,         /* device scan of per-edge work, then 2048 blocks of items
                                    (one binary search per shorter-row entry), then finalize */
  TRUSS_CHOICE_WIDE_NARROW = 3,  /* the same with 256 blocks */
  TRUSS_CHOICE_WIDE_GALLOP = 4,  /* wide, 8 shorter-row entries per item, galloping search */
  TRUSS_CHOICE_WAVE = 5,         /* one wave per frontier edge, no work scan: the two rows merged
                                    in 64-entry chunks (binary search in the longer row when it is
                                    over 8 times the shorter), then finalize */
  TRUSS_CHOICE_HASH = 6,         /* one wave per frontier edge, no work scan: the longer row (up to
                                    256 entries) hashed into LDS and probed by the shorter row's
                                    entries (longer rows as TRUSS_CHOICE_WAVE), then finalize */
  TRUSS_NUM_CHOICES = 7
} truss_choice;

/* Launch choices the cost model scores (TRUSS_VARIANT_LEARNED): the first six.  The LDS-hash
 * round stays outside its choice space: it is slower than the merge round on every traced
 * workload, and scoring it made the model's held-out choices worse. */
#define TRUSS_MODEL_CHOICES 6

/* Policy that picks the launch of every round. */
typedef enum {
  TRUSS_VARIANT_AUTO = 0,    /* built-in heuristic: FUSED up to 2048 frontier edges, else WIDE */
  TRUSS_VARIANT_BSEARCH = 1, /* same as AUTO (binary search everywhere) */
  TRUSS_VARIANT_MERGE = 2,   /* galloping search in every round (FUSED rounds gallop too) */
  TRUSS_VARIANT_FIXED = 3,   /* every round uses truss_options.force_choice (where valid) */
  TRUSS_VARIANT_LEARNED = 4  /* the MLP cost model (truss_options.mlp_weights) predicts the time
                                of every valid choice from the frontier's features (frontiers of
                                more than 32768 edges); the cheapest is launched when it is predicted
                                at least 10 % faster than the heuristic's launch, which stands
                                otherwise and for smaller frontiers */
} truss_variant;

/* Features of a frontier, in the order the cost model and the trace use them:
 * log2(1 + frontier edges), log2(1 + mean endpoint degree), log2(1 + max endpoint
 * degree), log2(1 + p99 endpoint degree) (from a log2 histogram), log2(1 + level),
 * log2(1 + mean shorter-row length).  Degrees are of the working adjacency. */
#define TRUSS_NUM_FEATURES 6

/* One record per launch sequence of the peeling loop (when tracing). */
typedef struct {
  int32_t level;             /* support level at the start */
  int32_t kind;              /* 0 level scan, 1 fused launch, 2 wide launch sequence, 3 one wave
                                per edge (merge), 4 one wave per edge (LDS hash) */
  int32_t choice;            /* truss_choice launched (kinds 1 and 2) */
  int32_t rounds;            /* frontier rounds completed by the sequence */
  int64_t frontier;          /* frontier size at the start */
  int64_t items;             /* intersection items of the first round (kind 2), else -1 */
  float ms;                  /* device time of the sequence */
  float features[8];         /* the frontier's features (first TRUSS_NUM_FEATURES used) */
  int32_t round_index;       /* index of the sequence's first frontier round in the run */
} truss_trace_record;

/* Host-side trace buffer: the library appends up to `capacity` records and
 * sets `count`.  Tracing runs the host-driven loop with one sync per sequence. */
typedef struct {
  int64_t capacity;
  int64_t count;
  truss_trace_record* records;
} truss_trace;

/* truss_options.relabel = 1 (auto) relabels graphs of at least this many edges ... */
#define TRUSS_RELABEL_MIN_EDGES (1 << 20)
/* ... whose maximum degree is at least this many times the mean degree 2m / n. */
#define TRUSS_RELABEL_MIN_SKEW 16

typedef struct {
  int32_t variant;           /* truss_variant; default AUTO */
  int32_t device_loop;       /* 0 = host-driven: the host reads the loop state after every launch
                                sequence; 1 = device-driven: batches of gated steps between host
                                checks; 2 = as 1, the steps replayed from a captured hipGraph;
                                3 = pipelined host loop: launch sequences guessed from the last
                                published loop state stay in flight (two by default), the loop
                                state is published to host-mapped memory and polled (default 3;
                                a trace forces 0, profile turns 2 into 1) */
  int32_t validate;          /* 1 = check the input CSR before any other work (default 1) */
  int32_t owner_rule;        /* 0 = the lower edge id owns a two-frontier-edge triangle (the
                                paper's rule, default); 1 = the higher id (the paper's stated
                                alternative); for tests, the output does not change */
  int32_t compact;           /* 1 = periodically drop peeled edges from the working adjacency
                                (default 1); 0 = intersect the full rows every time */
  int32_t steps_per_sync;    /* device_loop 1, 2: steps per host check; 3: sequences in flight
                                (at most 5); 0 = auto */
  const float* mlp_weights;  /* device: weights for TRUSS_VARIANT_LEARNED (truss_mlp_weights_floats
                                floats), or NULL */
  truss_trace* trace;        /* host: per-sequence trace of the peeling loop, or NULL */
  int32_t profile;           /* 1 = time every launch of the wide sub-level kernel with events
                                (truss_stats.wide_ms) */
  int32_t batch_mode;        /* truss_decompose_batched: 0 = all graphs at once as one disjoint
                                union through one level loop (default); 1 = one graph after
                                another through the single-graph path (a comparison point);
                                2 = one persistent launch, one workgroup per graph from a queue
                                ordered by decreasing edge count */
  int32_t force_choice;      /* truss_choice for TRUSS_VARIANT_FIXED */
  int32_t single_round;      /* 1 = every launch sequence runs exactly one frontier round (no
                                continuation of tiny rounds inside the fused launch); for
                                collecting per-round timing traces */
  int32_t* peel_round;       /* device, int32[m], or NULL: receives for every edge the index of the
                                frontier round that processed it (a peeling order: rounds run in
                                level order, so a lower trussness never gets a later round) */
  int32_t multi_round;       /* 1 = with device_loop 0 or 3, consecutive fused rounds run in one
                                cooperative launch of 64 workgroups that meet at a grid barrier
                                between rounds (measured slower than one launch per round on
                                this GPU; default 0) */
  int32_t relabel;           /* truss_decompose and truss_decompose32 only: 0 = decompose the graph
                                as given; 2 = relabel the vertices by increasing (degree, id) on the
                                device, decompose the relabelled graph and map its trussness (and
                                peel_round) back to the input's edge order -- the output does not
                                change, and on graphs with hubs the level loop runs faster because
                                the high-degree rows it searches most sit together; 1 = auto
                                (default): relabel when the graph has at least
                                TRUSS_RELABEL_MIN_EDGES edges and a maximum degree at least
                                TRUSS_RELABEL_MIN_SKEW times the mean degree (where it was measured
                                to gain; small or evenly spread graphs lose its cost).  1 and 2
                                need the larger workspace truss_workspace_bytes gives for them; the
                                relabelling's time is counted in ms_build.  Not used by
                                truss_support, truss_decompose32_static or the batched entry
                                point */
  int32_t reserved[6];       /* zero (room for later options without a layout change) */
} truss_options;

typedef struct {
  int64_t m;             /* edges */
  int64_t levels;        /* levels scanned (non-empty and skipped-to) */
  int64_t sublevels;     /* frontier rounds */
  int64_t triangles;     /* triangles in the input graph */
  int32_t t_max;         /* maximum trussness (0 when m = 0) */
  int32_t compactions;   /* adjacency rebuilds */
  float ms_validate;     /* phase times (ms, device events) */
  float ms_build;        /* edge ids, orientation; with relabel = 1 also the relabelling */
  float ms_support;
  float ms_peel;         /* level loop: scans, sub-levels, compactions */
  float ms_total;
  int64_t choice_count[8];  /* launch sequences run with each truss_choice (first
                               TRUSS_NUM_CHOICES used) */
  /* the wide sub-level intersection kernel (the dominant kernel) */
  int64_t wide_launches;   /* launches that found work */
  int64_t wide_items;      /* intersection items (one per shorter-row entry searched) */
  int64_t wide_frontier;   /* frontier edges */
  float wide_ms;           /* summed device time of its timed launches (opt.profile only) */
  int32_t wide_timed;      /* launches timed into wide_ms: with the host-driven loop those of
                              rounds above level 0; with the device-driven loop every launch,
                              including those that found their gate closed */
} truss_stats;

/* Fills *opt with the defaults listed above. */
void truss_default_options(truss_options* opt);

/* Workspace bytes needed by truss_decompose and truss_decompose32 for a graph with
 * n vertices and two_m adjacency slots (= offsets[n]) under the options *opt (NULL =
 * defaults).  With relabel = 1 or 2 (the default is 1) this adds, beyond the
 * decomposition's own arrays, the relabelled CSR and the permutation: about 16 bytes
 * per edge and 40 per vertex more. */
truss_status truss_workspace_bytes(int32_t n, int64_t two_m, const truss_options* opt, size_t* bytes);

/*
 * Trussness of every edge of one graph.
 *   n           vertices (>= 0)
 *   offsets     device, int64[n+1]
 *   adj         device, int32[offsets[n]]
 *   trussness   device, int32[m] output, m = offsets[n] / 2, edge order as above
 *   workspace   device, >= truss_workspace_bytes(...) bytes, 256-byte aligned;
 *               contents on entry are ignored
 *   opt         NULL = defaults
 *   stats       NULL or host struct receiving counters and phase times
 *   stream      hipStream_t (NULL = default stream)
 * Input is validated first when opt->validate is set; with validate = 0 the input
 * must satisfy the contract above (the library then reads only offsets[0..n] and
 * adj[0..offsets[n]) but its results are unspecified for a malformed CSR).
 */
truss_status truss_decompose(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* trussness,
                             void* workspace, size_t workspace_bytes, const truss_options* opt,
                             truss_stats* stats, void* stream);

/* Same as truss_decompose for int32 offsets (requires offsets[n] <= 2^31 - 1).
 * Needs truss_workspace_bytes(n, two_m, opt) bytes, which include the int64 copy of
 * the offsets the library makes. */
truss_status truss_decompose32(int32_t n, const int32_t* offsets, const int32_t* adj, int32_t* trussness,
                               void* workspace, size_t workspace_bytes, const truss_options* opt,
                               truss_stats* stats, void* stream);

/*
 * truss_decompose32 with no allocation at all, for callers that cannot allocate
 * (serving loops that must not call hipMalloc, harnesses that forbid allocation).
 * The workspace is a static device array of 64 MiB (2^26 bytes) inside the
 * library, one per GPU, held until the process ends: graphs whose
 * truss_workspace_bytes(n, offsets[n]) under relabel = 0 exceeds it are rejected
 * with TRUSS_E_WORKSPACE (about 700 000 edges for sparse graphs; this entry point
 * never relabels).  The library calls
 * no hipMalloc, hipFree, hipHostMalloc, event, stream or graph creation here: the
 * loop state is read back into pageable host memory, device_loop 2 and 3 run as 1
 * (device-driven steps), opt->trace and opt->profile are rejected (TRUSS_E_ARG)
 * and the phase times in *stats stay 0.  Every call on one GPU uses that GPU's
 * array: calls that overlap on one GPU (two host threads, or two streams) race
 * and give undefined results.  Not for stream capture: the level loop reads its
 * state back from the device.  Arguments, output and errors otherwise as
 * truss_decompose32.
 */
truss_status truss_decompose32_static(int32_t n, const int32_t* offsets, const int32_t* adj, int32_t* trussness,
                                      const truss_options* opt, truss_stats* stats, void* stream);

/*
 * Initial support of every edge (number of triangles containing it), same
 * edge order, into support (device, int32[m]).  Same workspace as
 * truss_decompose.
 */
truss_status truss_support(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* support,
                           void* workspace, size_t workspace_bytes, const truss_options* opt, void* stream);

/* Endpoints of every edge in output order: el_u[e] < el_v[e] (device, int32[m]
 * each).  Same workspace as truss_decompose. */
truss_status truss_edge_list(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* el_u,
                             int32_t* el_v, void* workspace, size_t workspace_bytes, void* stream);

/*
 * The maximal k-trusses, given the trussness (Introduction and Background
 * sections: a k-truss is a maximal connected subgraph in which every edge lies in
 * at least k - 2 triangles of the subgraph).  The edges of trussness >= k contain every k-truss
 * and have that property themselves, so the k-trusses are their connected
 * components (two such edges that share a vertex belong to the same k-truss).
 *   n, m             vertices and edges of the graph (n >= 0, 0 <= m < 2^31)
 *   el_u, el_v       device, int32[m]: edge endpoints in any order and orientation
 *                    (e.g. from truss_edge_list); edge e is (el_u[e], el_v[e])
 *   trussness        device, int32[m], e.g. from truss_decompose
 *   k                >= 2
 *   label            device, int32[m] out: for an edge of trussness >= k, the
 *                    smallest edge id of its k-truss (so the labels are unique and
 *                    equal labels mean the same k-truss); -1 for the other edges
 *   num_trusses      host, may be NULL: the number of k-trusses
 * The caller owns every buffer.  Workspace: truss_ktruss_workspace_bytes(n)
 * bytes at 256-byte alignment.  Errors: TRUSS_E_ARG (bad n, m or k, or a NULL
 * pointer with m > 0), TRUSS_E_RANGE (an endpoint of an edge of trussness >= k
 * outside [0, n); label is then undefined), TRUSS_E_WORKSPACE, TRUSS_E_DEVICE.
 */
truss_status truss_ktruss_workspace_bytes(int32_t n, size_t* bytes);
truss_status truss_ktruss(int32_t n, int64_t m, const int32_t* el_u, const int32_t* el_v,
                          const int32_t* trussness, int32_t k, int32_t* label, int32_t* num_trusses,
                          void* workspace, size_t workspace_bytes, void* stream);

/*
 * Core numbers of every vertex (k-core decomposition: the k-core is the maximal
 * subgraph of minimum degree >= k, and the core number of v the largest k whose
 * k-core holds v), by the level-synchronous vertex peeling that the PKT section
 * carries over to edges (Background section, parallel k-core decomposition).
 *   n, offsets, adj  the CSR contract of truss_decompose (device); isolated
 *                    vertices get core number 0
 *   core             device, int32[n] out
 *   max_core         host, may be NULL: the largest core number
 * The caller owns every buffer.  Workspace: truss_kcore_workspace_bytes(n)
 * bytes at 256-byte alignment.  The host copies the counters back once per
 * round and once per level (one stream synchronisation each).  Errors:
 * TRUSS_E_ARG, TRUSS_E_RANGE (offsets out of order or past offsets[n], or a
 * neighbour id outside [0, n); core is then undefined), TRUSS_E_WORKSPACE,
 * TRUSS_E_DEVICE, TRUSS_E_INTERNAL.
 */
truss_status truss_kcore_workspace_bytes(int32_t n, size_t* bytes);
truss_status truss_kcore(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* core, int32_t* max_core,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Vertex reordering by increasing core number (KCO; Performance Results section, the
 * support-computation study and Table 2): relabel the vertices so that ids grow
 * with the core number, decompose the relabelled graph, and map its trussness back
 * (the trussness of an edge does not depend on the labels).  Three calls, all on
 * `stream` and all stream-ordered; each synchronises the stream a few times to
 * check its inputs.  The caller owns every buffer.
 *
 * truss_kco_order: the new id of every vertex, sorted by (core number, old id).
 *   n                vertices (>= 0)
 *   core             device, int32[n]: core numbers (truss_kcore), each >= 0
 *   new_id           device, int32[n] out: new id of old vertex v
 *   order            device, int32[n] out: old vertex at new id i (the inverse)
 *   workspace        device, truss_kco_order_workspace_bytes(n) bytes, 256-byte aligned
 * Errors: TRUSS_E_ARG, TRUSS_E_RANGE (a negative core number), TRUSS_E_WORKSPACE,
 * TRUSS_E_DEVICE.
 *
 * truss_kco_relabel: the CSR of the relabelled graph, every row sorted.
 *   offsets, adj     device, the input: a symmetric CSR as for truss_decompose
 *                    (int64[n+1] starting at 0, int32[2m])
 *   new_id, order    device, int32[n]: a permutation and its inverse (truss_kco_order)
 *   offsets2         device, int64[n+1] out
 *   adj2             device, int32[2m] out (NULL when m = 0)
 *   workspace        device, truss_kco_relabel_workspace_bytes(n, 2m) bytes (about
 *                    18 bytes per adjacency slot), 256-byte aligned
 * Errors: TRUSS_E_ARG (NULL buffers), TRUSS_E_RANGE (2m above (2^24 - 1) * 2^11,
 * offsets not starting at 0 or out of order, a neighbour outside [0, n), or new_id
 * not a permutation with order its inverse), TRUSS_E_NOT_SYMMETRIC (some (u, v)
 * without (v, u)); the outputs are then undefined.  TRUSS_E_WORKSPACE,
 * TRUSS_E_DEVICE.
 *
 * truss_kco_map: trussness per input edge from the trussness of the relabelled graph.
 *   n, m             vertices and edges of the input
 *   el_u, el_v       device, int32[m]: the input's edges (any order; truss_edge_list
 *                    gives the canonical one, so that the output is indexed by the
 *                    input's edge ids)
 *   new_id           device, int32[n]: as given to truss_kco_relabel
 *   offsets2, adj2   device: its output
 *   trussness2       device, int32[m]: truss_decompose of the relabelled graph
 *   trussness        device, int32[m] out: trussness of edge (el_u[e], el_v[e])
 *   workspace        device, truss_kco_map_workspace_bytes(n) bytes, 256-byte aligned
 * Errors: TRUSS_E_ARG (offsets2[n] != 2m, NULL buffers), TRUSS_E_RANGE (offsets2 out
 * of order, a new id or an endpoint outside [0, n), an edge with no image in the
 * relabelled graph; its entry is then -1), TRUSS_E_WORKSPACE, TRUSS_E_DEVICE.
 */
truss_status truss_kco_order_workspace_bytes(int32_t n, size_t* bytes);
truss_status truss_kco_order(int32_t n, const int32_t* core, int32_t* new_id, int32_t* order, void* workspace,
                             size_t workspace_bytes, void* stream);
truss_status truss_kco_relabel_workspace_bytes(int32_t n, int64_t two_m, size_t* bytes);
truss_status truss_kco_relabel(int32_t n, const int64_t* offsets, const int32_t* adj, const int32_t* new_id,
                               const int32_t* order, int64_t* offsets2, int32_t* adj2, void* workspace,
                               size_t workspace_bytes, void* stream);
truss_status truss_kco_map_workspace_bytes(int32_t n, size_t* bytes);
truss_status truss_kco_map(int32_t n, int64_t m, const int32_t* el_u, const int32_t* el_v, const int32_t* new_id,
                           const int64_t* offsets2, const int32_t* adj2, const int32_t* trussness2,
                           int32_t* trussness, void* workspace, size_t workspace_bytes, void* stream);

/* Trussness by the local h-index iteration, the barrier-free alternative to the
 * level-synchronous loop that the Background section cites (Sariyuce et al.'s
 * local nucleus decomposition): sweep 0 sets every edge's estimate to its support,
 * and every sweep gives each edge, all at once, the h-index of
 * min(estimate(f1), estimate(f2)) over its triangles {e, f1, f2} under the
 * previous sweep's estimates; the estimates stop at trussness - 2.
 *   n, offsets, adj  device: a simple symmetric CSR with rows strictly increasing
 *                    (int64[n+1] starting at 0, int32[2m]), 2m < 2^31
 *   trussness        device, int32[m] out, canonical edge order (as truss_decompose):
 *                    estimate + 2 after the last sweep run
 *   max_sweeps       sweeps to run at most after sweep 0; < 0: until none changes
 *   sweeps           host, may be NULL: sweeps run that changed an estimate
 *   converged        host, may be NULL: 1 if a sweep changed nothing (the output is
 *                    then the trussness), else 0
 *   workspace        device, truss_hindex_workspace_bytes(n, 2m) bytes (about 9
 *                    bytes per adjacency slot and 16 per vertex), 256-byte aligned
 * Work per sweep is the triangle walk of every edge whose neighbourhood changed,
 * one to three times; the host synchronises once per sweep.  Errors: TRUSS_E_ARG,
 * TRUSS_E_RANGE (offsets out of order, a neighbour outside [0, n)),
 * TRUSS_E_NOT_SIMPLE (a row not strictly increasing, a self loop),
 * TRUSS_E_NOT_SYMMETRIC, TRUSS_E_WORKSPACE, TRUSS_E_DEVICE, TRUSS_E_INTERNAL.
 */
truss_status truss_hindex_workspace_bytes(int32_t n, int64_t two_m, size_t* bytes);
truss_status truss_hindex(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* trussness,
                          int32_t max_sweeps, int32_t* sweeps, int32_t* converged, void* workspace,
                          size_t workspace_bytes, void* stream);

/*
 * Batched decomposition of many independent graphs.  By default they are
 * decomposed together as one disjoint union (one level loop and one launch
 * sequence for the whole batch; trussness is per connected component and the
 * union's edge order is the packed order below).
 *   num_graphs       G >= 0
 *   graph_vtx_off    device, int64[G+1]: the offsets of graph g occupy
 *                    offsets_packed[graph_vtx_off[g] .. graph_vtx_off[g+1]), i.e.
 *                    n_g + 1 entries
 *   graph_adj_off    device, int64[G+1]: the adjacency of graph g occupies
 *                    adj_packed[graph_adj_off[g] .. graph_adj_off[g+1]), i.e. 2 m_g
 *                    entries
 *   offsets_packed   device, int32: local offsets of each graph (start at 0)
 *   adj_packed       device, int32: local vertex ids
 *   trussness_packed device, int32[sum m_g]: graph g's edges at graph_adj_off[g] / 2 + e
 * Each graph must satisfy the CSR contract with n_g <= 2^20 and m_g <= 2^24.
 * Workspace: truss_batched_workspace_bytes with the same sizes.
 */
truss_status truss_batched_workspace_bytes(int32_t num_graphs, int64_t total_vtx_entries, int64_t total_adj,
                                           const truss_options* opt, size_t* bytes);
truss_status truss_decompose_batched(int32_t num_graphs, const int64_t* graph_vtx_off,
                                     const int64_t* graph_adj_off, const int32_t* offsets_packed,
                                     const int32_t* adj_packed, int32_t* trussness_packed,
                                     int64_t total_vtx_entries, int64_t total_adj, void* workspace,
                                     size_t workspace_bytes, const truss_options* opt, truss_stats* stats,
                                     void* stream);

/*
 * The launch cost model of TRUSS_VARIANT_LEARNED: an fp32 MLP from the
 * TRUSS_NUM_FEATURES frontier features to one predicted log2(device microseconds)
 * per scored launch choice (TRUSS_MODEL_CHOICES, 3 hidden layers of 64, ReLU).  Weights are
 * truss_mlp_num_params() floats in device memory: feature mean and standard
 * deviation (for normalisation), then each layer's weights and biases.  Rows of X
 * are feature vectors, rows of T the measured log2 times, rows of M 1 where a
 * choice was measured (0 otherwise); all device, row-major.  Training minimises
 * the masked mean squared error.  The tuning workflow and its traces are in
 * paper_1707_02000_amd/tuner.py; this is not part of the decomposition itself.
 */
int32_t truss_mlp_num_params(void);

/* Device bytes of workspace for n rows (forward, gradient, training). */
size_t truss_mlp_workspace_bytes(int32_t n);

/* Normalisation from X, layers seeded uniform in +-1/sqrt(fan_in), output biases
 * the mean measured target per choice. */
truss_status truss_mlp_init(const float* X, const float* T, const float* M, int32_t n, uint64_t seed,
                            float* weights, void* stream);

/* Y[n][TRUSS_NUM_CHOICES] = model(X[n][TRUSS_NUM_FEATURES]). */
truss_status truss_mlp_forward(const float* X, int32_t n, const float* weights, float* Y, void* workspace,
                               size_t workspace_bytes, void* stream);

/* Gradient (truss_mlp_num_params floats; zero for the normalisation entries) and
 * loss (one float) of the masked mean squared error, all device. */
truss_status truss_mlp_gradient(const float* X, const float* T, const float* M, int32_t n, const float* weights,
                                float* grad, float* loss, void* workspace, size_t workspace_bytes, void* stream);

/* `steps` full-batch Adam steps (beta 0.9 / 0.999, eps 1e-8) at rate lr, in place;
 * loss_history (device, `steps` floats, or NULL) receives the loss before each step. */
truss_status truss_mlp_train(const float* X, const float* T, const float* M, int32_t n, float* weights, int32_t steps,
                             float lr, float* loss_history, void* workspace, size_t workspace_bytes, void* stream);

/* The peeling loop's decision for n frontiers: choice[i] = the valid choice of
 * least predicted time if it beats the heuristic's launch by 10 % (log2 margin
 * 0.1375), else the heuristic's launch (fused choices are valid up to 2048 frontier
 * edges, ncurr gives each frontier's size); Y (or NULL) receives the predictions.
 * Uses the same device inference and decision routines as the loop. */
truss_status truss_mlp_choose(const float* X, const int32_t* ncurr, int32_t n, const float* weights, int32_t* choice,
                              float* Y, void* stream);

/* Static message for a status code. */
const char* truss_strerror(truss_status status);

/* Message for the calling thread's most recent error (empty if none). */
const char* truss_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PKT_H_ */
