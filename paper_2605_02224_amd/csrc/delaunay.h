// Incremental 3-D Delaunay triangulation that records successor lists (host side).
//
// Successor list L_i (Sec. 3; Fig. 2 caption): when p_j is inserted, j is appended to the
// list of every Delaunay neighbour of p_j in DT(P_{1:j}), so each list is ascending in rank.
// The construction is Bowyer-Watson with exact predicates and a vertex at infinity (ghost
// tetrahedra on every convex-hull facet), so hull adjacencies are exact and no bounding box
// distorts the diagram.  Point location uses the lists already built: a 1-NN descent
// (the DP-NNS walk of Sec. 3) finds the nearest older site of p_j, and some tetrahedron
// incident to that site conflicts with p_j.
//
// Degeneracies: ties of the in-sphere test are resolved by perturbing the lifted coordinate
// |p|^2 of every site downward by an amount that grows with its rank, so the newest site is
// inside every sphere it lies exactly on (the triangulation is the unique regular
// triangulation of the perturbed lifting).  Facet adjacency (positive-area Voronoi facet) is
// never lost by this choice; exactly degenerate contacts may add weak adjacencies.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace mknn {

constexpr int32_t kInf = -1;

struct Csr {
  std::vector<int64_t> off;   // n + 1
  std::vector<int32_t> ent;   // ranks
};

enum BuildStatus { kBuildOk = 0, kBuildDuplicate = 1, kBuildDegenerateStart = 2,
                   kBuildInternal = 3 };

class DelaunayBuilder {
 public:
  // pts: n x 3 doubles by rank (must outlive the builder)
  DelaunayBuilder(const double *pts, int64_t n);

  // Inserts ranks 0..n-1 in order.  On failure, *bad_rank names the offending rank.
  BuildStatus build(int64_t *bad_rank);

  // Inserts rank j (j == number inserted so far); used by build() and by incremental use.
  BuildStatus insert_next();

  // Clouds whose first four ranks are coplanar (or collinear): the lists are defined for
  // every prefix (Sec. 3) -- while the prefix spans a line or a plane, the Voronoi cells are
  // slabs or prisms over the cells of that line or plane.  low_dim_plan picks the start:
  // A = the first rank off the line of ranks 0 and 1, B = the first rank off the plane of
  // ranks 0, 1 and A; when there is none, a spare point (ids nreal, nreal + 1 of pts, which
  // the caller reserves) is placed off the line or plane instead.  Returns kBuildDuplicate
  // (*bad = 1) if ranks 0 and 1 coincide.
  static BuildStatus low_dim_plan(double *pts, int64_t nreal, int32_t *A, int32_t *B,
                                  int64_t *bad);
  // Builds the lists of ranks 0 .. nreal-1 (the builder holds nreal + 2 points) starting from
  // the tetrahedron (0, 1, A, B).  A rank j on the line or in the plane is then inserted
  // with A and B already present; its neighbours of smaller rank are exactly its neighbours
  // in the diagram of the prefix (the cone over the line's or plane's triangulation has no
  // other edges between them), and A and B take their own list entries when their turn
  // comes: every older rank, since a point off the line (plane) of the older ones is a
  // Voronoi neighbour of each of them.  Spare points never enter a list.
  BuildStatus build_low_dim(int64_t nreal, int32_t A, int32_t B, int64_t *bad_rank);

  int64_t inserted() const { return ninserted_; }

  // Successor lists as CSR (entries ascending within each list).
  Csr successors() const;
  // Delaunay neighbours of each rank at its own insertion (the transpose of the lists).
  Csr predecessors() const;

  // Structural self-check: orientations, symmetric neighbour links, vertex incidences.
  bool validate(std::string *why) const;
  // Every finite tetrahedron has an empty circumsphere (exact); O(T * n), small inputs only.
  bool validate_empty_spheres(std::string *why) const;

  int64_t num_tets() const;
  // Tetrahedron slots (some free); tet(t, v) copies slot t's vertices and returns false
  // for a free slot.
  int64_t num_tet_slots() const { return (int64_t)stamp_.size(); }
  bool tet(int64_t t, int32_t v[4]) const;
  int64_t exact_fallbacks() const;

  // Finite Delaunay neighbours of the vertex inserted last (ascending ids).
  const std::vector<int32_t> &last_neighbors() const { return nbrs_; }

  // True when some tetrahedron (finite or ghost) incident to edge (a, b) has p strictly inside
  // its circumsphere (a ghost: p strictly beyond its hull facet, or in the facet's plane and
  // strictly inside its circumcircle).  p need not be a vertex.
  bool edge_in_conflict(int32_t a, int32_t b, const double *p);

  // Start the triangulation from four given affinely independent vertices instead of the
  // first four ids; the remaining ids are then inserted in increasing order (skipping
  // these four).  Returns false if they are coplanar.
  bool start_with(const int32_t first4[4]);

  // Insert only the given ids, in the given order (before the first insertion); ids not
  // listed are never inserted.
  bool set_order(std::vector<int32_t> order);
  // The point array now holds n points (the first ones unchanged, the array possibly
  // moved); the new ids join the end of the insertion order.
  void grow(const double *pts, int64_t n);
  // Number of ids in the insertion order (inserted or still to insert).
  int64_t order_size() const { return (int64_t)order_.size(); }
  // 1-NN of p among the inserted sites and its squared distance.
  int32_t nearest(const double *p, double *d) const { return nearest_inserted(p, d); }

  // Removes the inserted vertex v (the insertion order must be ascending in id).  Its star is replaced by the tetrahedra of the
  // triangulation of its link vertices (built here, in id order) that v would destroy if
  // inserted there, under the same perturbation as the construction; the result is the
  // triangulation the construction gives without v.  On failure (fewer than five sites
  // left, a local triangulation that cannot start, or a cavity whose boundary does not
  // match v's link) nothing is changed.  v's own list is emptied; the lists of other
  // vertices are the caller's to fix (set_list), since point location walks them.
  BuildStatus remove(int32_t v);
  // Replaces v's list (the successor list point location walks).
  void set_list(int32_t v, const int32_t *ent, int32_t len);

 private:
  const double *P_;
  int64_t n_;
  int64_t ninserted_ = 0;

  std::vector<int32_t> tv_;   // 4 vertices per tet (kInf for the vertex at infinity)
  std::vector<int32_t> tn_;   // 4 neighbours per tet, opposite the same-index vertex
  std::vector<uint32_t> stamp_;
  std::vector<int32_t> free_;
  std::vector<int32_t> vtet_; // one incident tet per vertex
  uint32_t epoch_ = 1;

  // dynamic successor lists
  std::vector<int64_t> lstart_;
  std::vector<int32_t> llen_, lcap_;
  std::vector<int32_t> pool_;

  // scratch
  std::vector<int32_t> stack_, cavity_, star_;
  struct Boundary { int32_t v[4]; int32_t h; int32_t outer; int32_t outer_face; };
  std::vector<Boundary> bnd_;
  std::vector<uint64_t> hkey_;
  std::vector<int32_t> hval_;
  std::vector<uint32_t> hstamp_;
  std::vector<uint32_t> vmark_;
  uint32_t vepoch_ = 1, hepoch_ = 1;
  std::vector<int32_t> nbrs_;

  const double *pt(int32_t v) const { return P_ + 3 * (int64_t)v; }
  int32_t alloc_tet();
  bool conflict(int32_t t, const double *p, bool strict = false) const;
  bool destroyed_by(int32_t t, const double *p, int32_t v, const int32_t *ids) const;
  std::vector<int32_t> order_;      // insertion order of ids (identity unless start_with)
  std::vector<char> gone_;          // removed vertices
  int64_t live_ = 0;                // inserted and not removed
  int64_t walk_pos_ = 0;            // order_ position of the oldest vertex not removed
  bool ascending_ = true;           // order_ ascending in id (identity, or set_order's)
  // the perturbation ranks vertices by insertion; with an ascending order that is the id
  int32_t rank_of(int32_t v) const { return v; }
  std::vector<char> done_;
  int64_t nreal_ = -1;              // build_low_dim: ids >= nreal_ are spare points
  bool quiet_start_ = false;        // init_first_tet records no list entries
  int32_t nearest_inserted(const double *p, double *dbest) const;
  int32_t locate(int32_t near, const double *p);
  void append(int32_t owner, int32_t rank);
  bool init_first_tet();
};

}  // namespace mknn
