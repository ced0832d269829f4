// Voronoi cell builder for the synthetic sweep workloads.
//
// Builds the Voronoi tessellation of seed points in the unit box [0,1)^3, either
// clipped by the box walls (vacuum boundaries) or periodic (faces towards periodic
// images carry an integer image shift).  Each cell is obtained independently by
// clipping a starting cube with the bisector planes of its nearest seeds, in
// order of increasing distance, until no farther seed can cut the cell (security
// radius: a seed at distance r can only cut the cell if r < 2 * max vertex radius).
//
// This is an input generator only: it produces face areas, unit normals
// n = (p' - p)/|p' - p| (the Voronoi normal of the paper's appendix A) and cell
// volumes.  It contains none of the transport sweep's arithmetic.
//
// C ABI (loaded through ctypes):
//   voro_build(...)  -> opaque handle (or NULL), per-cell status
//   voro_counts(h, &n_half_faces)
//   voro_fetch(h, face_ptr, nbr, shift, area, normal, volume)
//   voro_free(h)
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

// One face of the convex cell polyhedron, in coordinates relative to the seed.
// Plane: x . d <= h.  label >= 0: neighbour seed index (with periodic image
// shift code `shift`); label < 0: box wall -(1 + wall index).
struct Face {
  V3 d;
  double h;
  int32_t label;
  int8_t shift;
  std::vector<V3> poly;
};

struct CellOut {
  std::vector<int32_t> nbr;
  std::vector<int8_t> shift;
  std::vector<double> area;
  std::vector<double> normal;  // 3 per face
  double volume = 0.0;
};

inline int8_t shift_code(int sx, int sy, int sz) {
  return (int8_t)((sx + 1) * 9 + (sy + 1) * 3 + (sz + 1) - 13);
}

// Clip the polyhedron by x . d <= h.  Returns false if the cell vanished.
bool clip(std::vector<Face>& faces, V3 d, double h, int32_t label, int8_t shift) {
  // Quick test: any vertex outside?
  bool any_out = false;
  for (const Face& f : faces) {
    for (const V3& v : f.poly) {
      if (dot(v, d) - h > 0.0) { any_out = true; break; }
    }
    if (any_out) break;
  }
  if (!any_out) return true;

  std::vector<V3> cut_pts;
  std::vector<Face> kept;
  kept.reserve(faces.size() + 1);
  for (Face& f : faces) {
    const size_t m = f.poly.size();
    std::vector<V3> np;
    np.reserve(m + 2);
    for (size_t k = 0; k < m; ++k) {
      const V3 a = f.poly[k];
      const V3 b = f.poly[(k + 1) % m];
      const double sa = dot(a, d) - h;
      const double sb = dot(b, d) - h;
      const bool ina = !(sa > 0.0), inb = !(sb > 0.0);
      if (ina) np.push_back(a);
      if (ina != inb) {
        // Intersection computed from the inside endpoint towards the outside
        // one, so both faces sharing this edge produce the identical point.
        const V3 pin = ina ? a : b;
        const V3 pout = ina ? b : a;
        const double sin_ = ina ? sa : sb;
        const double sout = ina ? sb : sa;
        const double t = sin_ / (sin_ - sout);
        const V3 x = add(pin, scl(sub(pout, pin), t));
        np.push_back(x);
        cut_pts.push_back(x);
      }
    }
    if (np.size() >= 3) {
      f.poly.swap(np);
      kept.push_back(std::move(f));
    }
  }
  // New face on the cutting plane: order the cut points by angle.
  std::sort(cut_pts.begin(), cut_pts.end(), [](const V3& a, const V3& b) {
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.z < b.z;
  });
  cut_pts.erase(std::unique(cut_pts.begin(), cut_pts.end(),
                            [](const V3& a, const V3& b) {
                              return a.x == b.x && a.y == b.y && a.z == b.z;
                            }),
                cut_pts.end());
  if (cut_pts.size() >= 3) {
    V3 c{0, 0, 0};
    for (const V3& p : cut_pts) c = add(c, p);
    c = scl(c, 1.0 / (double)cut_pts.size());
    const double dn = norm(d);
    const V3 e3 = scl(d, 1.0 / dn);
    V3 tmp = std::fabs(e3.x) < 0.9 ? V3{1, 0, 0} : V3{0, 1, 0};
    V3 e1 = cross(tmp, e3);
    e1 = scl(e1, 1.0 / norm(e1));
    const V3 e2 = cross(e3, e1);
    std::vector<std::pair<double, V3>> ang;
    ang.reserve(cut_pts.size());
    for (const V3& p : cut_pts) {
      const V3 r = sub(p, c);
      ang.push_back({std::atan2(dot(r, e2), dot(r, e1)), p});
    }
    std::sort(ang.begin(), ang.end(),
              [](const std::pair<double, V3>& a, const std::pair<double, V3>& b) {
                return a.first < b.first;
              });
    Face nf;
    nf.d = d;
    nf.h = h;
    nf.label = label;
    nf.shift = shift;
    for (auto& pr : ang) nf.poly.push_back(pr.second);
    kept.push_back(std::move(nf));
  }
  faces.swap(kept);
  return faces.size() >= 4;
}

double max_radius2(const std::vector<Face>& faces) {
  double r2 = 0.0;
  for (const Face& f : faces)
    for (const V3& v : f.poly) r2 = std::max(r2, dot(v, v));
  return r2;
}

// Starting cube [lo, hi] (relative coordinates), faces labelled by `labels`.
std::vector<Face> make_cube(V3 lo, V3 hi, const int32_t labels[6],
                            const int8_t shifts[6]) {
  // corners
  V3 P[8];
  for (int k = 0; k < 8; ++k)
    P[k] = {(k & 1) ? hi.x : lo.x, (k & 2) ? hi.y : lo.y, (k & 4) ? hi.z : lo.z};
  // faces: -x, +x, -y, +y, -z, +z (vertex loops, outward CCW)
  const int loops[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4},
                           {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
  const V3 dirs[6] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                      {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
  const double hs[6] = {-lo.x, hi.x, -lo.y, hi.y, -lo.z, hi.z};
  std::vector<Face> faces(6);
  for (int f = 0; f < 6; ++f) {
    faces[f].d = dirs[f];
    faces[f].h = hs[f];
    faces[f].label = labels[f];
    faces[f].shift = shifts[f];
    for (int k = 0; k < 4; ++k) faces[f].poly.push_back(P[loops[f][k]]);
  }
  return faces;
}

struct Build {
  int32_t n = 0;
  std::vector<CellOut> cells;
  int64_t n_half_faces = 0;
};


// Cell i from its candidate neighbours cand[0..k) (sorted by increasing
// minimum-image distance; the seed itself may appear).  Returns the status:
// 0 ok, 1 candidates exhausted before the security radius, 2 degenerate cell,
// 3 periodic cell too large for minimum-image neighbours.
int build_cell(int32_t i, int32_t n, const double* pts, int32_t periodic, int32_t k,
               const int32_t* cand, CellOut& out) {
  const V3 p{pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
  std::vector<Face> faces;
  if (periodic) {
    // The periodic cell lies within half a box of its seed; the cube's faces
    // are the bisectors with the seed's own images.
    const int32_t lab[6] = {i, i, i, i, i, i};
    const int8_t sh[6] = {shift_code(-1, 0, 0), shift_code(1, 0, 0),
                          shift_code(0, -1, 0), shift_code(0, 1, 0),
                          shift_code(0, 0, -1), shift_code(0, 0, 1)};
    faces = make_cube({-0.5, -0.5, -0.5}, {0.5, 0.5, 0.5}, lab, sh);
  } else {
    const int32_t lab[6] = {-1, -2, -3, -4, -5, -6};
    const int8_t sh[6] = {0, 0, 0, 0, 0, 0};
    faces = make_cube({-p.x, -p.y, -p.z}, {1.0 - p.x, 1.0 - p.y, 1.0 - p.z}, lab, sh);
  }
  int st = 1;
  double r2max = max_radius2(faces);
  for (int32_t q = 0; q < k; ++q) {
    const int32_t j = cand[q];
    if (j == i || j < 0) continue;
    V3 dv{pts[3 * j] - p.x, pts[3 * j + 1] - p.y, pts[3 * j + 2] - p.z};
    int sx = 0, sy = 0, sz = 0;
    if (periodic) {
      if (dv.x >= 0.5) { dv.x -= 1.0; sx = -1; } else if (dv.x < -0.5) { dv.x += 1.0; sx = 1; }
      if (dv.y >= 0.5) { dv.y -= 1.0; sy = -1; } else if (dv.y < -0.5) { dv.y += 1.0; sy = 1; }
      if (dv.z >= 0.5) { dv.z -= 1.0; sz = -1; } else if (dv.z < -0.5) { dv.z += 1.0; sz = 1; }
    }
    const double r2 = dot(dv, dv);
    if (r2 >= 4.0 * r2max) { st = 0; break; }
    if (!clip(faces, dv, 0.5 * r2, j, shift_code(sx, sy, sz))) { st = 2; break; }
    r2max = max_radius2(faces);
  }
  if (st == 1 && k >= n) st = 0;  // every seed was offered
  if (st == 0 && periodic && r2max >= 0.0625) st = 3;
  out = CellOut();
  double vol = 0.0;
  for (const Face& f : faces) {
    V3 av{0, 0, 0};
    const size_t m = f.poly.size();
    for (size_t t = 1; t + 1 < m; ++t)
      av = add(av, cross(sub(f.poly[t], f.poly[0]), sub(f.poly[t + 1], f.poly[0])));
    const double dn = norm(f.d);
    const V3 nrm = scl(f.d, 1.0 / dn);
    const double a = 0.5 * std::fabs(dot(av, nrm));
    vol += a * (f.h / dn) / 3.0;
    if (!(a > 0.0)) continue;
    out.nbr.push_back(f.label >= 0 ? f.label : -1);
    out.shift.push_back(f.label >= 0 ? f.shift : (int8_t)0);
    out.area.push_back(a);
    out.normal.push_back(nrm.x);
    out.normal.push_back(nrm.y);
    out.normal.push_back(nrm.z);
  }
  out.volume = vol;
  return st;
}

void count_faces(Build* B) {
  int64_t tot = 0;
  for (const CellOut& c : B->cells) tot += (int64_t)c.nbr.size();
  B->n_half_faces = tot;
}

}  // namespace

extern "C" {

// pts: n*3 seeds in [0,1)^3.  cand: n*k candidate neighbour indices sorted by
// increasing (minimum-image) distance; the first entry may be the seed itself.
// status[i]: see build_cell.
void* voro_build(int32_t n, const double* pts, int32_t periodic, int32_t k,
                 const int32_t* cand, int32_t* status) {
  Build* B = new Build();
  B->n = n;
  B->cells.resize(n);
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i)
    status[i] = build_cell(i, n, pts, periodic, k, cand + (int64_t)i * k, B->cells[i]);
  count_faces(B);
  return B;
}

// Rebuild the m cells listed in `cells` from k candidates each (cand: m*k, in
// the order of `cells`); status: m entries.
void voro_rebuild(void* h, int32_t m, const int32_t* cells, const double* pts, int32_t periodic,
                  int32_t k, const int32_t* cand, int32_t* status) {
  Build* B = static_cast<Build*>(h);
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t t = 0; t < m; ++t)
    status[t] = build_cell(cells[t], B->n, pts, periodic, k, cand + (int64_t)t * k,
                           B->cells[cells[t]]);
  count_faces(B);
}

int64_t voro_counts(void* h) { return static_cast<Build*>(h)->n_half_faces; }

void voro_fetch(void* h, int64_t* face_ptr, int32_t* nbr, int8_t* shift,
                double* area, double* normal, double* volume) {
  Build* B = static_cast<Build*>(h);
  int64_t off = 0;
  for (int32_t i = 0; i < B->n; ++i) {
    const CellOut& c = B->cells[i];
    face_ptr[i] = off;
    const size_t m = c.nbr.size();
    if (m) {
      std::memcpy(nbr + off, c.nbr.data(), m * sizeof(int32_t));
      std::memcpy(shift + off, c.shift.data(), m * sizeof(int8_t));
      std::memcpy(area + off, c.area.data(), m * sizeof(double));
      std::memcpy(normal + 3 * off, c.normal.data(), 3 * m * sizeof(double));
    }
    volume[i] = c.volume;
    off += (int64_t)m;
  }
  face_ptr[B->n] = off;
}

void voro_free(void* h) { delete static_cast<Build*>(h); }

}  // extern "C"
