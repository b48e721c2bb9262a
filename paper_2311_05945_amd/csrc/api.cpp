// Host side of the HIP library: scene preprocessing, state, the Newton time step
// and the C interface declared in include/zema.h.
//
// Time step (Sec. III: minimise B_t + D of eq. 11, then the velocity update):
//   predictor and kinematic targets; lagged friction at y^t (eqs. 9-10);
//   warm start y^t + a h ydot^t with a the CCD bound of that move (halved while a
//   tet would invert); then Newton iterations: assemble gradient and projected
//   Hessian on the active set, PCG for p, stop when the largest vertex displacement
//   of p is <= newton_tol * h, swept candidates over [y, y + p], CCD bound, halve
//   the step until no tet inverts and the energy does not increase, accept, and
//   double the automatic barrier stiffness when the minimum distance fell below
//   1e-3 dhat and decreased.
#include <algorithm>
#include <thread>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <vector>

#include "material.hpp"
#include "scene.hpp"

using namespace zema;

namespace {


double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct D3h {
  double x, y, z;
};
D3h sub(const double* a, const double* b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
D3h crs(D3h a, D3h b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double dt3(D3h a, D3h b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// ------------------------------------------------------------------ preprocessing
// Scene k of a batch owns soft bodies [soft_off[k], soft_off[k+1]) and affine bodies
// [aff_off[k], aff_off[k+1]); one scene: offsets {0, n_soft} and {0, n_aff}.
void build_scene(zema_scene* s, const zema_soft_desc* soft, int n_soft, const zema_affine_desc* aff, int n_aff,
                 const int* soft_off, const int* aff_off, int ns, const double* mu_sc) {
  s->n_soft_bodies = n_soft;
  s->n_bodies = n_soft + n_aff;
  s->ns = ns;
  s->scn.assign(ns, SceneRange());
  for (int k = 0; k < ns; ++k) {
    if (soft_off[k + 1] < soft_off[k] || aff_off[k + 1] < aff_off[k]) throw Error(ZEMA_E_ARG, "scene offsets");
    s->scn[k].mu = mu_sc[k];
  }
  if (soft_off[0] != 0 || aff_off[0] != 0 || soft_off[ns] != n_soft || aff_off[ns] != n_aff)
    throw Error(ZEMA_E_ARG, "scene offsets");
  std::vector<int> body_scene(std::max(n_soft + n_aff, 1), 0);
  for (int k = 0; k < ns; ++k) {
    for (int b = soft_off[k]; b < soft_off[k + 1]; ++b) body_scene[b] = k;
    for (int b = aff_off[k]; b < aff_off[k + 1]; ++b) body_scene[n_soft + b] = k;
  }
  std::vector<double> X, x_init, v_init, Dmi_aos, vol, lmu, llam, mass, cl_d;
  std::vector<int4> cl_v;
  std::vector<int> tets, vbody;
  std::vector<unsigned char> tmodel;
  // ---- soft bodies
  std::vector<std::array<int, 4>> faces;  // packed (a, b, c) outward + body
  std::vector<unsigned long long> fkey;
  for (int b = 0; b < n_soft; ++b) {
    const zema_soft_desc& d = soft[b];
    SceneRange& R = s->scn[body_scene[b]];
    if (b == soft_off[body_scene[b]]) {
      R.v0 = R.v1 = (int)mass.size();
      R.t0 = R.t1 = (int)vol.size();
    }
    if (d.n_verts < 0 || d.n_tets < 0 || (d.n_verts && !d.rest_pos) || (d.n_tets && !d.tets) || d.n_tris < 0 ||
        (d.n_tris && !d.tris))
      throw Error(ZEMA_E_ARG, "bad soft body descriptor");
    if (d.model < ZEMA_NEO_HOOKEAN || d.model > ZEMA_BARAFF_WITKIN)
      throw Error(ZEMA_E_ARG, "unknown constitutive model");
    if ((d.model == ZEMA_BARAFF_WITKIN) != (d.n_tris > 0) || (d.model == ZEMA_BARAFF_WITKIN && d.n_tets))
      throw Error(ZEMA_E_ARG, "garment bodies take triangles only, solids tets only");
    if (d.model == ZEMA_BARAFF_WITKIN && ns > 1) throw Error(ZEMA_E_ARG, "garment bodies are single-scene only");
    int v0 = (int)mass.size();
    double mu = d.E / (2.0 * (1.0 + d.nu)), la = d.E * d.nu / ((1.0 + d.nu) * (1.0 - 2.0 * d.nu));
    for (int i = 0; i < d.n_verts; ++i) {
      for (int k = 0; k < 3; ++k) {
        X.push_back(d.rest_pos[3 * i + k]);
        x_init.push_back(d.pos0 ? d.pos0[3 * i + k] : d.rest_pos[3 * i + k]);
        v_init.push_back(d.vel0 ? d.vel0[3 * i + k] : 0.0);
      }
      mass.push_back(0.0);
      vbody.push_back(b);
    }
    for (int e = 0; e < d.n_tets; ++e) {
      int t[4];
      for (int a = 0; a < 4; ++a) {
        int v = d.tets[4 * e + a];
        if (v < 0 || v >= d.n_verts) throw Error(ZEMA_E_MESH, "tet index out of range");
        t[a] = v0 + v;
      }
      D3h c1 = sub(&X[3 * t[1]], &X[3 * t[0]]), c2 = sub(&X[3 * t[2]], &X[3 * t[0]]),
          c3 = sub(&X[3 * t[3]], &X[3 * t[0]]);
      double det = dt3(c1, crs(c2, c3));
      if (det < 0.0) {  // reorder so that the tet is positive
        std::swap(t[1], t[2]);
        std::swap(c1, c2);
        det = -det;
      }
      double L = std::max({std::fabs(c1.x), std::fabs(c1.y), std::fabs(c1.z), std::fabs(c2.x), std::fabs(c2.y),
                           std::fabs(c2.z), std::fabs(c3.x), std::fabs(c3.y), std::fabs(c3.z)});
      if (!(det > 1e-14 * L * L * L)) throw Error(ZEMA_E_MESH, "degenerate tet");
      // Dm = [c1 c2 c3] (columns); inverse rows = (c2 x c3, c3 x c1, c1 x c2) / det
      D3h r0 = crs(c2, c3), r1 = crs(c3, c1), r2 = crs(c1, c2);
      double id = 1.0 / det;
      double Dm[9] = {r0.x * id, r0.y * id, r0.z * id, r1.x * id, r1.y * id, r1.z * id,
                      r2.x * id, r2.y * id, r2.z * id};
      for (int k = 0; k < 9; ++k) Dmi_aos.push_back(Dm[k]);
      double V = det / 6.0;
      vol.push_back(V);
      lmu.push_back(mu);
      llam.push_back(la);
      tmodel.push_back((unsigned char)d.model);
      for (int a = 0; a < 4; ++a) {
        tets.push_back(t[a]);
        mass[t[a]] += 0.25 * d.rho * V;
      }
      // outward faces of a positive tet (local index patterns)
      const int F[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
      for (int f = 0; f < 4; ++f) {
        int a = t[F[f][0]], bb = t[F[f][1]], c = t[F[f][2]];
        int lo = std::min({a, bb, c}), hi = std::max({a, bb, c}), mid = a + bb + c - lo - hi;
        fkey.push_back(((unsigned long long)lo << 42) | ((unsigned long long)mid << 21) | (unsigned long long)hi);
        faces.push_back({a, bb, c, 0});
      }
    }
    // garment triangles: rest (u, v) = rest (x, z); inverse rest edge matrix, area,
    // stretch and shear stiffness; mass rho A / 3 per vertex; each triangle is a
    // surface triangle as given
    for (int e = 0; e < d.n_tris; ++e) {
      int t[3];
      for (int a = 0; a < 3; ++a) {
        int v = d.tris[3 * e + a];
        if (v < 0 || v >= d.n_verts) throw Error(ZEMA_E_MESH, "triangle index out of range");
        t[a] = v0 + v;
      }
      const double du1 = X[3 * t[1]] - X[3 * t[0]], du2 = X[3 * t[2]] - X[3 * t[0]];
      const double dv1 = X[3 * t[1] + 2] - X[3 * t[0] + 2], dv2 = X[3 * t[2] + 2] - X[3 * t[0] + 2];
      const double det = du1 * dv2 - du2 * dv1;
      const double L = std::max({std::fabs(du1), std::fabs(du2), std::fabs(dv1), std::fabs(dv2)});
      if (!(std::fabs(det) > 1e-12 * L * L)) throw Error(ZEMA_E_MESH, "degenerate garment triangle");
      const double A = 0.5 * std::fabs(det);
      cl_v.push_back(make_int4(t[0], t[1], t[2], 0));
      const double dd[8] = {dv2 / det, -du2 / det, -dv1 / det, du1 / det, A, d.E, d.E / (2.0 * (1.0 + d.nu)), 0.0};
      cl_d.insert(cl_d.end(), dd, dd + 8);
      for (int a = 0; a < 3; ++a) mass[t[a]] += d.rho * A / 3.0;
      int lo = std::min({t[0], t[1], t[2]}), hi = std::max({t[0], t[1], t[2]}), mid = t[0] + t[1] + t[2] - lo - hi;
      fkey.push_back(((unsigned long long)lo << 42) | ((unsigned long long)mid << 21) | (unsigned long long)hi);
      faces.push_back({t[0], t[1], t[2], 0});
    }
    R.v1 = (int)mass.size();
    R.t1 = (int)vol.size();
  }
  s->nsv = (int)mass.size();
  s->ncl = (int)cl_v.size();
  s->nt = (int)vol.size();
  for (int k = 0, v = 0, t = 0; k < ns; ++k) {  // scenes without soft bodies: empty ranges in order
    if (soft_off[k + 1] == soft_off[k]) {
      s->scn[k].v0 = s->scn[k].v1 = v;
      s->scn[k].t0 = s->scn[k].t1 = t;
    }
    v = s->scn[k].v1;
    t = s->scn[k].t1;
  }
  if (s->nsv >= (1 << 21)) throw Error(ZEMA_E_ARG, "too many soft vertices");
  // boundary faces: keys occurring once
  std::vector<int> ford(fkey.size());
  for (size_t i = 0; i < ford.size(); ++i) ford[i] = (int)i;
  std::sort(ford.begin(), ford.end(), [&](int a, int b) { return fkey[a] < fkey[b] || (fkey[a] == fkey[b] && a < b); });
  std::vector<std::array<int, 3>> soft_tris;
  for (size_t i = 0; i < ford.size();) {
    size_t j = i;
    while (j < ford.size() && fkey[ford[j]] == fkey[ford[i]]) ++j;
    if (j - i == 1) soft_tris.push_back({faces[ford[i]][0], faces[ford[i]][1], faces[ford[i]][2]});
    i = j;
  }
  // ---- affine bodies
  int dof = 3 * s->nsv, node = s->nsv;
  s->nfree = 0;
  for (int b = 0; b < n_aff; ++b) {
    const zema_affine_desc& d = aff[b];
    if (d.n_verts <= 0 || d.n_tris <= 0 || !d.rest_pos || !d.tris) throw Error(ZEMA_E_ARG, "bad affine descriptor");
    if (d.mode < 0 || d.mode > 2) throw Error(ZEMA_E_ARG, "bad affine mode");
    // closed, consistently oriented: every directed edge has its reverse exactly once
    std::vector<unsigned long long> de;
    for (int t = 0; t < d.n_tris; ++t)
      for (int k = 0; k < 3; ++k) {
        int a = d.tris[3 * t + k], c = d.tris[3 * t + (k + 1) % 3];
        if (a < 0 || a >= d.n_verts || c < 0 || c >= d.n_verts) throw Error(ZEMA_E_MESH, "triangle index");
        de.push_back(((unsigned long long)a << 32) | (unsigned)c);
      }
    std::sort(de.begin(), de.end());
    for (size_t i = 0; i < de.size(); ++i) {
      if (i + 1 < de.size() && de[i + 1] == de[i]) throw Error(ZEMA_E_MESH, "non-manifold affine surface");
      unsigned long long rev = ((de[i] & 0xffffffffull) << 32) | (de[i] >> 32);
      if (!std::binary_search(de.begin(), de.end(), rev)) throw Error(ZEMA_E_MESH, "open affine surface");
    }
    Body B;
    B.mode = d.mode;
    B.rho = d.rho;
    B.stiff = d.stiffness;
    B.kappaA = d.kappa_A;
    for (int k = 0; k < 3; ++k) B.tvel[k] = d.target_vel[k];
    B.tstop = d.target_stop;
    for (int k = 0; k < 12; ++k) B.qdot0[k] = d.qdot0[k];
    // volume, centre and second moment from signed tets (ref, a, b, c), ref = vertex mean
    double ref[3] = {0, 0, 0};
    for (int i = 0; i < d.n_verts; ++i)
      for (int k = 0; k < 3; ++k) ref[k] += d.rest_pos[3 * i + k] / d.n_verts;
    double V = 0.0, m1[3] = {0, 0, 0}, m2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int t = 0; t < d.n_tris; ++t) {
      const double* P[3] = {d.rest_pos + 3 * d.tris[3 * t], d.rest_pos + 3 * d.tris[3 * t + 1],
                            d.rest_pos + 3 * d.tris[3 * t + 2]};
      double v[3][3];
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) v[a][k] = P[a][k] - ref[k];
      D3h a0{v[0][0], v[0][1], v[0][2]}, a1{v[1][0], v[1][1], v[1][2]}, a2{v[2][0], v[2][1], v[2][2]};
      double vt = dt3(a0, crs(a1, a2)) / 6.0;
      V += vt;
      double sm[3];
      for (int k = 0; k < 3; ++k) {
        sm[k] = v[0][k] + v[1][k] + v[2][k];
        m1[k] += vt * 0.25 * sm[k];
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          m2[i][j] += vt * 0.05 * (v[0][i] * v[0][j] + v[1][i] * v[1][j] + v[2][i] * v[2][j] + sm[i] * sm[j]);
    }
    if (!(V > 0.0)) throw Error(ZEMA_E_MESH, "affine surface not outward");
    B.V = V;
    B.m = d.rho * V;
    double cr[3];
    for (int k = 0; k < 3; ++k) {
      cr[k] = m1[k] / V;
      B.c[k] = ref[k] + cr[k];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) B.S[3 * i + j] = d.rho * (m2[i][j] - V * cr[i] * cr[j]);
    for (int k = 0; k < 12; ++k) B.qrest[k] = 0.0;
    for (int k = 0; k < 3; ++k) {
      B.qrest[k] = B.c[k];
      B.qrest[3 + 4 * k] = 1.0;
    }
    B.nsv = d.n_verts;
    if (B.mode != ZEMA_FIXED) {
      B.dof0 = dof;
      B.node0 = node;
      dof += 12;
      node += 4;
      s->nfree++;
    }
    s->bodies.push_back(B);
  }
  s->ndof = dof;
  s->nnodes = node;
  // ---- surface vertices, scene by scene: the scene's soft boundary vertices
  // ascending, then every vertex of its affine bodies in body order
  std::vector<int> sv_ref, sv_body, soft_sid(s->nsv, -1);
  std::vector<double> sv_x0;
  std::vector<std::array<int, 3>> all_tris;
  {
    std::vector<char> on(s->nsv, 0);
    for (auto& t : soft_tris)
      for (int k = 0; k < 3; ++k) on[t[k]] = 1;
    for (int k = 0, f = 0; k < ns; ++k) {
      SceneRange& R = s->scn[k];
      R.s0 = (int)sv_ref.size();
      for (int i = R.v0; i < R.v1; ++i)
        if (on[i]) {
          soft_sid[i] = (int)sv_ref.size();
          sv_ref.push_back(i);
          sv_body.push_back(vbody[i]);
          sv_x0.insert(sv_x0.end(), {0.0, 0.0, 0.0});
        }
      R.b0 = aff_off[k];
      R.b1 = aff_off[k + 1];
      R.f0 = f;
      for (int b = R.b0; b < R.b1; ++b) {
        Body& B = s->bodies[b];
        const zema_affine_desc& d = aff[b];
        B.sv0 = (int)sv_ref.size();
        for (int i = 0; i < d.n_verts; ++i) {
          sv_ref.push_back(-(b + 1));
          sv_body.push_back(n_soft + b);
          for (int q = 0; q < 3; ++q) sv_x0.push_back(d.rest_pos[3 * i + q] - B.c[q]);
        }
        for (int t = 0; t < d.n_tris; ++t)
          all_tris.push_back({B.sv0 + d.tris[3 * t], B.sv0 + d.tris[3 * t + 1], B.sv0 + d.tris[3 * t + 2]});
        if (B.mode != ZEMA_FIXED) ++f;
      }
      R.f1 = f;
      R.s1 = (int)sv_ref.size();
    }
    for (auto& t : soft_tris) all_tris.push_back({soft_sid[t[0]], soft_sid[t[1]], soft_sid[t[2]]});
  }
  s->nsurf = (int)sv_ref.size();
  // ---- canonical triangles and edges
  for (auto& t : all_tris) {
    int k = 0;
    if (t[1] < t[k]) k = 1;
    if (t[2] < t[k]) k = 2;
    t = {t[k], t[(k + 1) % 3], t[(k + 2) % 3]};
  }
  std::sort(all_tris.begin(), all_tris.end());
  std::vector<unsigned long long> ek;
  for (auto& t : all_tris)
    for (int k = 0; k < 3; ++k) {
      unsigned a = (unsigned)std::min(t[k], t[(k + 1) % 3]), c = (unsigned)std::max(t[k], t[(k + 1) % 3]);
      ek.push_back(((unsigned long long)a << 32) | c);
    }
  std::sort(ek.begin(), ek.end());
  ek.erase(std::unique(ek.begin(), ek.end()), ek.end());
  s->ntri = (int)all_tris.size();
  s->nedge = (int)ek.size();
  std::vector<int> tris_h, edges_h;
  for (auto& t : all_tris) tris_h.insert(tris_h.end(), {t[0], t[1], t[2]});
  std::vector<double> elen2;
  double lsum = 0.0;
  for (auto e : ek) {
    int a = (int)(e >> 32), c = (int)(e & 0xffffffffu);
    edges_h.push_back(a);
    edges_h.push_back(c);
    double l2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      double pa = sv_ref[a] >= 0 ? X[3 * sv_ref[a] + k] : sv_x0[3 * a + k];
      double pc = sv_ref[c] >= 0 ? X[3 * sv_ref[c] + k] : sv_x0[3 * c + k];
      l2 += (pc - pa) * (pc - pa);
    }
    elen2.push_back(l2);
    lsum += std::sqrt(l2);
  }
  s->cell = s->nedge ? lsum / s->nedge : 1.0;
  if (!(s->cell > 0.0)) s->cell = 1.0;
  std::vector<int> sv_scene(std::max(s->nsurf, 1), 0);
  for (int i = 0; i < s->nsurf; ++i) sv_scene[i] = body_scene[sv_body[i]];
  {
    std::vector<double> csum(ns, 0.0);
    std::vector<int> ccnt(ns, 0);
    for (int e = 0; e < s->nedge; ++e) {
      int k = sv_scene[edges_h[2 * e]];
      csum[k] += std::sqrt(elen2[e]);
      ccnt[k]++;
    }
    for (int k = 0; k < ns; ++k) {
      double c = ccnt[k] ? csum[k] / ccnt[k] : s->cell;
      s->scn[k].cell = c > 0.0 ? c : 1.0;
    }
  }
  // ---- static block pattern: tet node pairs and the 4x4 node blocks of free bodies
  int nn = s->nnodes;
  std::vector<unsigned long long> keys;
  keys.reserve((size_t)16 * s->nt + 16 * s->nfree);
  for (int e = 0; e < s->nt; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) keys.push_back((unsigned long long)tets[4 * e + a] * nn + tets[4 * e + b]);
  for (const Body& B : s->bodies)
    if (B.node0 >= 0)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) keys.push_back((unsigned long long)(B.node0 + a) * nn + (B.node0 + b));
  for (int i = 0; i < s->nsv; ++i) keys.push_back((unsigned long long)i * nn + i);  // garment vertices: mass block
  std::vector<unsigned long long> ukeys = keys;
  std::sort(ukeys.begin(), ukeys.end());
  ukeys.erase(std::unique(ukeys.begin(), ukeys.end()), ukeys.end());
  s->nnzb = (int)ukeys.size();
  std::vector<int> bptr(nn + 1, 0), bcol(s->nnzb), brow(s->nnzb), bdiag(nn, -1);
  for (int j = 0; j < s->nnzb; ++j) {
    int r = (int)(ukeys[j] / nn), c = (int)(ukeys[j] % nn);
    brow[j] = r;
    bcol[j] = c;
    bptr[r + 1]++;
    if (r == c) bdiag[r] = j;
  }
  for (int r = 0; r < nn; ++r) bptr[r + 1] += bptr[r];
  s->bsr_row_soft_end = bptr[s->nsv];
  std::vector<int> hcnt(s->nnzb + 1, 0), hpos((size_t)16 * s->nt);
  for (int e = 0; e < s->nt; ++e)
    for (int q = 0; q < 16; ++q) {
      unsigned long long k = keys[(size_t)16 * e + q];
      int j = (int)(std::lower_bound(ukeys.begin(), ukeys.end(), k) - ukeys.begin());
      hpos[(size_t)16 * e + q] = j;
      hcnt[j + 1]++;
    }
  for (int j = 0; j < s->nnzb; ++j) hcnt[j + 1] += hcnt[j];
  std::vector<int> hlist(hcnt[s->nnzb]), hfill(hcnt.begin(), hcnt.end() - 1);
  for (int e = 0; e < s->nt; ++e)
    for (int q = 0; q < 16; ++q) hlist[hfill[hpos[(size_t)16 * e + q]]++] = 16 * e + q;
  // vertex -> (tet, slot)
  std::vector<int> vtp(s->nsv + 1, 0), vtl((size_t)4 * s->nt);
  for (int e = 0; e < s->nt; ++e)
    for (int a = 0; a < 4; ++a) vtp[tets[4 * e + a] + 1]++;
  for (int i = 0; i < s->nsv; ++i) vtp[i + 1] += vtp[i];
  {
    std::vector<int> fill(vtp.begin(), vtp.end() - 1);
    for (int e = 0; e < s->nt; ++e)
      for (int a = 0; a < 4; ++a) vtl[fill[tets[4 * e + a]]++] = 4 * e + a;
  }
  // ---- upload
  const double h2 = s->P.dt * s->P.dt;
  std::vector<int4> t4(s->nt);
  std::vector<double> Dmi_soa((size_t)9 * s->nt), h2vol(s->nt);
  for (int e = 0; e < s->nt; ++e) {
    t4[e] = make_int4(tets[4 * e], tets[4 * e + 1], tets[4 * e + 2], tets[4 * e + 3]);
    for (int k = 0; k < 9; ++k) Dmi_soa[(size_t)k * s->nt + e] = Dmi_aos[(size_t)9 * e + k];
    h2vol[e] = h2 * vol[e];
  }
  s->tets.upload(t4);
  s->Dmi.upload(Dmi_soa);
  s->h2vol.upload(h2vol);
  s->lmu.upload(lmu);
  s->llam.upload(llam);
  s->tmodel.upload(tmodel);
  s->mass.upload(mass);
  {
    std::vector<int> vr(n_soft + 1, (int)mass.size());
    for (int i = (int)vbody.size() - 1; i >= 0; --i) vr[vbody[i]] = i;
    for (int b = n_soft - 1; b >= 0; --b) vr[b] = std::min(vr[b], vr[b + 1]);  // bodies without vertices
    s->soft_vr.upload(vr);
    s->v_sbody.upload(vbody);
  }
  s->mass_h = mass;
  s->vt_ptr.upload(vtp);
  s->vt_list.upload(vtl);
  s->bsr_ptr.upload(bptr);
  s->bsr_col.upload(bcol);
  s->bsr_row.upload(brow);
  s->bsr_diag.upload(bdiag);
  s->hc_ptr.upload(hcnt);
  s->hc_list.upload(hlist);
  {  // destination slots of the element records (diagonal / gradient: position in the
     // vertex's incident list; off-diagonal: position in the upper block's tet list)
    std::vector<int> slot((size_t)10 * s->nt), optr(1, 0), oblk, omir;
    for (int k = 0; k < (int)vtl.size(); ++k) slot[(size_t)(vtl[k] & 3) * s->nt + (vtl[k] >> 2)] = k;
    for (int j = 0; j < s->bsr_row_soft_end; ++j) {
      if (!(brow[j] < bcol[j])) continue;
      for (int k = hcnt[j]; k < hcnt[j + 1]; ++k) {
        int ent = hlist[k], e = ent >> 4, a = (ent >> 2) & 3, b = ent & 3;
        int lo = std::min(a, b), hi = std::max(a, b);
        int p = lo == 0 ? hi - 1 : (lo == 1 ? 1 + hi : 5);  // pair order (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)
        slot[(size_t)(4 + p) * s->nt + e] = optr.back() + (k - hcnt[j]);
      }
      optr.push_back(optr.back() + (hcnt[j + 1] - hcnt[j]));
      oblk.push_back(j);
      unsigned long long key = (unsigned long long)bcol[j] * nn + brow[j];
      omir.push_back((int)(std::lower_bound(ukeys.begin(), ukeys.end(), key) - ukeys.begin()));
    }
    if (optr.back() != 6 * s->nt) throw Error(ZEMA_E_MESH, "tet pair blocks do not match the static pattern");
    s->tslot.upload(slot);
    s->off_ptr.upload(optr);
    s->off_blk.upload(oblk);
    s->off_mir.upload(omir);
  }
  // the mixed-precision form keeps Hessian blocks and their products in FP32; only
  // the buffers of the chosen form are allocated at full size
  s->mixed = s->P.precision == ZEMA_MIXED;
  size_t nbv = (size_t)9 * s->nnzb + 9, nht = (size_t)kTetHess * s->nt + kTetHess;
  s->bsr_val.resize(s->mixed ? 9 : nbv);
  ZCHK(hipMemset(s->bsr_val.p, 0, sizeof(double) * s->bsr_val.n));
  s->bsr_val32.resize(s->mixed ? nbv : 9);
  ZCHK(hipMemset(s->bsr_val32.p, 0, sizeof(float) * s->bsr_val32.n));
  s->e_tet.resize(s->nt + s->ncl + 1);
  s->cl_v.upload(cl_v);
  s->cl_d.upload(cl_d);
  s->g_tet.resize((size_t)12 * s->nt + 12);  // [4 nt][3] gradient records
  s->h_tet.resize(s->mixed ? kTetHess : nht);
  s->h_tet32.resize(s->mixed ? nht : kTetHess);
  s->e_in.resize(s->nsv + 1);
  int nb = (int)s->bodies.size();
  std::vector<double> bf((size_t)BF * std::max(nb, 1), 0.0);
  std::vector<int> bi((size_t)4 * std::max(nb, 1), 0);
  std::vector<unsigned char> fixed(std::max(s->n_bodies, 1), 0);
  for (int b = 0; b < nb; ++b) {
    const Body& B = s->bodies[b];
    bf[BF * b + 0] = B.m;
    bf[BF * b + 1] = B.V;
    bf[BF * b + 2] = B.stiff;
    bf[BF * b + 3] = B.kappaA;
    for (int k = 0; k < 9; ++k) bf[BF * b + 4 + k] = B.S[k];
    for (int k = 0; k < 12; ++k) bf[BF * b + BF_QF + k] = B.qrest[k];
    bi[4 * b] = B.mode;
    bi[4 * b + 1] = B.dof0;
    bi[4 * b + 2] = B.node0;
    if (B.mode == ZEMA_FIXED) fixed[n_soft + b] = 1;
  }
  s->body_f.upload(bf);
  s->body_i.upload(bi);
  s->body_fixed.upload(fixed);
  s->qtilde.resize((size_t)12 * std::max(nb, 1));
  s->e_body.resize((size_t)3 * std::max(nb, 1));
  s->sv_ref.upload(sv_ref);
  s->soft_sv.upload(soft_sid.empty() ? std::vector<int>{-1} : soft_sid);
  s->body_tv.resize((size_t)3 * std::max<size_t>(s->bodies.size(), 1));
  ZCHK(hipMemset(s->body_tv.p, 0, sizeof(double) * s->body_tv.n));
  s->sv_body.upload(sv_body);
  // ---- scene table
  s->body_scene.upload(body_scene);
  s->sv_scene.upload(sv_scene);
  {
    std::vector<int> vs(std::max(s->nsv, 1), 0), fs(std::max(s->nfree, 1), 0), rng((size_t)8 * ns);
    for (int k = 0; k < ns; ++k) {
      const SceneRange& R = s->scn[k];
      for (int i = R.v0; i < R.v1; ++i) vs[i] = k;
      for (int f = R.f0; f < R.f1; ++f) fs[f] = k;
      int r[8] = {R.v0, R.v1, R.t0, R.t1, R.b0, R.b1, R.f0, R.f1};
      for (int q = 0; q < 8; ++q) rng[(size_t)8 * k + q] = r[q];
      double m = 0.0;
      for (int i = R.v0; i < R.v1; ++i) m += mass[i];
      s->scn[k].mbar = R.v1 > R.v0 ? m / (R.v1 - R.v0) : 1.0;
    }
    s->v_scene.upload(vs);
    s->f_scene.upload(fs);
    std::vector<int> sb((size_t)4 * ns);
    for (int k = 0; k < ns; ++k) {
      sb[4 * k] = soft_off[k];
      sb[4 * k + 1] = soft_off[k + 1];
      sb[4 * k + 2] = n_soft + aff_off[k];
      sb[4 * k + 3] = n_soft + aff_off[k + 1];
    }
    s->scene_bodies.upload(sb);
    s->scn_rng.upload(rng);
    std::vector<double> ic(ns), mu(ns);
    for (int k = 0; k < ns; ++k) {
      ic[k] = 1.0 / s->scn[k].cell;
      mu[k] = s->scn[k].mu;
    }
    s->icell_sc.upload(ic);
    s->mu_sc.upload(mu);
    s->kappa_sc.resize(ns);
    s->sc_u64.resize(ns);
    s->sc_dmin.resize(ns);
    s->sc_tmin.resize(ns);
    s->sc_alpha.resize(ns);
    s->sc_sum.resize((size_t)8 * ns);
    s->sc_mask.resize(ns);
    s->sc_rng.resize((size_t)8 * ns);
    s->sc_cnt.resize(ns);
    s->sc_act.resize(ns);
  }
  s->sv_x0.upload(sv_x0);
  s->tris.upload(tris_h);
  s->edges.upload(edges_h);
  s->elen2.upload(elen2);
  size_t ns3 = (size_t)3 * std::max(s->nsurf, 1);
  s->xs.resize(ns3);
  s->xs1.resize(ns3);
  s->xs2.resize(ns3);
  s->dxs.resize(ns3);
  size_t nd = std::max(s->ndof, 1);
  for (DBuf<double>* v : {&s->y, &s->ydot, &s->yt, &s->ydt, &s->yhat, &s->ytmp, &s->grad, &s->pdir, &s->yd_prev})
    v->resize(nd);
  s->counters.resize(16);
  s->umin.resize(8);
  s->red.resize(64 + 8 * 256);
  s->c_ptr.resize(nn + 1);
  ZCHK(hipMemset(s->c_ptr.p, 0, sizeof(int) * (nn + 1)));
  // initial state (device copies)
  std::vector<double> y0(nd, 0.0), yd0(nd, 0.0);
  for (int i = 0; i < 3 * s->nsv; ++i) {
    y0[i] = x_init[i];
    yd0[i] = v_init[i];
  }
  for (const Body& B : s->bodies)
    if (B.dof0 >= 0)
      for (int k = 0; k < 12; ++k) {
        y0[B.dof0 + k] = B.qrest[k];
        yd0[B.dof0 + k] = B.qdot0[k];
      }
  s->ytmp.upload(y0);
  s->pdir.upload(yd0);
}

// Mixed precision: the FP32 Hessian can be indefinite where the FP64 one is not, and
// its solve then need not be a usable Newton direction: an ascent direction of the FP64
// energy (g.p >= 0), or a solve whose FP64-checked residual stayed above half the
// right-hand side after the refinement passes.  Such a scene steps along the
// steepest-descent minimiser of the same quadratic model instead,
// p = -(g.g / g.H g) g (or -g scaled to |p| where g.H g <= 0); the line search and the
// next Newton iteration take it from there.  FP64 solves are left alone (their
// Hessian is PSD by construction).  Both were seen at the batched configuration's
// scale (512 uneven grasp scenes).
static void mixed_descent_guard(zema_scene* s, const int* active, const double* relres) {
  if (!s->mixed) return;
  const int ns = s->ns;
  std::vector<double> d((size_t)3 * ns), h((size_t)3 * ns), coef(ns, 0.0);
  std::vector<int> bad(ns, 0);
  k_scene_dots(s, s->grad.p, s->pdir.p, d.data());
  bool any = false;
  for (int k = 0; k < ns; ++k)
    if (active[k] && (d[3 * k] > 0.0 || !(relres[k] <= 0.5))) {
      bad[k] = 1;
      any = true;
    }
  if (!any) return;
  s->res_q.reserve(s->ndof);
  k_hess_matvec64(s, s->grad.p, s->res_q.p);
  k_scene_dots(s, s->grad.p, s->res_q.p, h.data());
  for (int k = 0; k < ns; ++k) {
    if (!bad[k]) continue;
    const double gg = d[3 * k + 1], pp = d[3 * k + 2], gHg = h[3 * k];
    if (gHg > 0.0)
      coef[k] = -gg / gHg;
    else
      coef[k] = gg > 0.0 && std::isfinite(pp) ? -std::sqrt(pp / gg) : 0.0;
  }
  // p = bad ? coef g : p (a select, so that a non-finite p is replaced too)
  s->res_r.reserve(s->ndof);
  ZCHK(hipMemcpyAsync(s->res_r.p, s->grad.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
  k_scale_scene(s, coef.data(), s->res_r.p);
  k_select_scene(s, bad.data(), s->res_r.p, s->pdir.p, s->pdir.p);
}

// message of a failed line search: the scene and the energies that did not decrease
static std::string ls_failure(int k, double e0, double e1) {
  char b[160];
  std::snprintf(b, sizeof b, "line search failed (scene %d: energy %.17g at the iterate, %.17g at the smallest step)",
                k, e0, e1);
  return b;
}

double auto_kappa(const zema_scene* s, int k) {
  double g = std::sqrt(s->P.gravity[0] * s->P.gravity[0] + s->P.gravity[1] * s->P.gravity[1] +
                       s->P.gravity[2] * s->P.gravity[2]);
  if (g == 0.0) g = 9.81;
  return s->P.dt * s->P.dt * s->scn[k].mbar * g / (s->P.dhat * (std::log(2.0) + 0.5));
}

// host staging arrays of per-scene uploads live in the scene, so they outlive the copy
void upload_kappa(zema_scene* s) {
  s->kappa_h.resize(s->ns);
  for (int k = 0; k < s->ns; ++k) s->kappa_h[k] = s->scn[k].kappa;
  ZCHK(hipMemcpyAsync(s->kappa_sc.p, s->kappa_h.data(), sizeof(double) * s->ns, hipMemcpyHostToDevice, s->st));
}

// energy terms at y on the current candidate set (surface positions recomputed), per
// scene: T[8 k + 0..5] the terms, 6 the total (+inf when infeasible), 7 the minimum
// distance (+inf without pairs)
void eval_energy(zema_scene* s, const double* y, double* T) {
  k_map_surface(s, y, s->xs.p);
  k_tet_energy(s, y);
  k_cloth_energy(s, y, s->e_tet.p + s->nt);
  k_inertia_energy(s, y, s->e_in.p);
  k_body_energy(s, y);
  k_contact_energy(s);
  k_spring_energy(s);
  k_joint_energy(s, y, s->e_spr.p + s->springs.size());
  if (s->ns == 1) {
    int nb = (int)s->bodies.size();
    const double* P[8] = {s->e_in.p, s->e_tet.p, s->e_body.p, s->e_body.p + nb, s->e_body.p + 2 * nb, s->e_pair.p,
                          s->e_fric.p, s->e_spr.p};
    const int64_t ncons = (int64_t)(s->springs.size() + s->joints.size());
    int64_t L[8] = {s->nsv, s->nt + s->ncl, nb, nb, nb, s->npt + s->nee, s->nfric, ncons};
    const int nseg = ncons ? 8 : 7;
    double out[9];
    k_sums(s, nseg, P, L, out, s->sc_dmin.p);
    const double espr = nseg == 8 ? out[7] : 0.0;  // springs and joints join the constraint term
    unsigned long long du;
    std::memcpy(&du, &out[nseg], sizeof(du));
    double dmin;
    std::memcpy(&dmin, &out[nseg], sizeof(double));
    T[0] = out[0] + out[2];
    T[1] = out[1];
    T[2] = out[3];
    T[3] = out[4] + espr;
    T[4] = out[5];
    T[5] = out[6];
    T[6] = T[0] + T[1] + T[2] + T[3] + T[4] + T[5];
    T[7] = (s->npt + s->nee) && du != ~0ull ? dmin : INFINITY;
  } else {
    k_scene_sums(s, T);
  }
  for (int k = 0; k < s->ns; ++k) {
    double* t = T + 8 * k;
    if (!std::isfinite(t[1]) || !(t[7] > 0.0)) t[6] = INFINITY;
  }
}

// energies, gradient (optional) and Hessian (optional) at y on the current candidates;
// false (and nothing assembled) when a scene's state is infeasible
bool assemble(zema_scene* s, const double* y, double* grad, bool hess, unsigned mask, double* T) {
  s->y_asm = y;
  eval_energy(s, y, T);
  for (int k = 0; k < s->ns; ++k)
    if (!std::isfinite(T[8 * k + 6])) return false;
  // the elastic assembly (per-tet kernel, gradient and Hessian gathers) is timed as one
  // group when the Hessian is assembled
  const bool timed = hess && grad && s->nt;
  if (timed) kt_begin(s, KT_TET);
  if (grad || hess) k_tet_assemble(s, y, hess);
  if (grad) k_gather_grad_soft(s, y, grad, mask);
  if (hess) k_gather_hess_static(s, mask);
  if (timed) kt_end(s, KT_TET, (s->mixed ? 170.0 : 320.0) * s->nt);
  k_body_terms(s, y, grad, hess, mask);
  if (mask & 8u) k_spring_terms(s, grad, hess);
  k_contact_assemble(s, grad, hess, mask);
  s->hess_valid = hess;
  return true;
}

void static_candidates(zema_scene* s, const double* y) {
  k_map_surface(s, y, s->xs.p);
  k_candidates(s, s->xs.p, s->xs.p, s->P.dhat);
}

void swept_candidates(zema_scene* s, const double* y, const double* p) {
  k_axpy(s, s->ndof, 1.0, p, y, s->ytmp.p);
  k_map_surface(s, y, s->xs.p);
  k_map_surface(s, s->ytmp.p, s->xs1.p);
  k_candidates(s, s->xs.p, s->xs1.p, s->P.dhat);
}

// per-scene minimum distances at y on the current candidates
std::vector<double> min_distance(zema_scene* s, const double* y) {
  std::vector<double> T((size_t)8 * s->ns), d(s->ns);
  eval_energy(s, y, T.data());
  for (int k = 0; k < s->ns; ++k) d[k] = T[8 * k + 7];
  return d;
}

// predictor, kinematic targets and the lagged friction table at y^t = s->y
// kinematic targets of the bodies of the scenes flagged in which (every scene when
// null) for the step each of those scenes is starting
void body_targets(zema_scene* s, const int* which) {
  int nb = (int)s->bodies.size();
  s->qt_h.resize((size_t)12 * std::max(nb, 1), 0.0);
  s->body_tv_h.resize((size_t)3 * std::max(nb, 1), 0.0);
  for (int k = 0; k < s->ns; ++k) {
    if (which && !which[k]) continue;
    const double tnext = (s->scene_step[k] + 1) * s->P.dt;
    for (int b = s->scn[k].b0; b < s->scn[k].b1; ++b) {
      const Body& B = s->bodies[b];
      // translational target velocity of a driven body over this step (learned guess input)
      for (int q = 0; q < 3; ++q) s->body_tv_h[3 * b + q] = 0.0;
      if (B.has_target) {  // a target set by the caller (the force controller of Sec. IV-A)
        for (int q = 0; q < 12; ++q) s->qt_h[12 * b + q] = B.target[q];
        for (int q = 0; q < 3; ++q) s->body_tv_h[3 * b + q] = B.target_vel[q];
        continue;
      }
      double tt = std::min(tnext, B.tstop);
      for (int q = 0; q < 12; ++q) s->qt_h[12 * b + q] = B.qrest[q];
      for (int q = 0; q < 3; ++q) s->qt_h[12 * b + q] += tt * B.tvel[q];
      if (B.mode != ZEMA_DRIVEN) continue;
      double span = std::min(tnext, B.tstop) - std::min(tnext - s->P.dt, B.tstop);
      for (int q = 0; q < 3; ++q) s->body_tv_h[3 * b + q] = B.tvel[q] * span / s->P.dt;
    }
  }
  ZCHK(hipMemcpyAsync(s->qtilde.p, s->qt_h.data(), sizeof(double) * s->qt_h.size(), hipMemcpyHostToDevice, s->st));
  ZCHK(hipMemcpyAsync(s->body_tv.p, s->body_tv_h.data(), sizeof(double) * s->body_tv_h.size(),
                      hipMemcpyHostToDevice, s->st));
}

void begin_step(zema_scene* s) {
  k_predict(s);
  s->scene_step.assign(s->ns, s->step);
  body_targets(s, nullptr);
  for (SceneRange& R : s->scn) R.kappa_lag = R.kappa;
  upload_kappa(s);
  static_candidates(s, s->y.p);
  k_friction_build(s);
  ZCHK(hipStreamSynchronize(s->st));
}

int set_state_impl(zema_scene* s, const double* y, const double* ydot, double kappa, int step) {
  ZCHK(hipMemcpyAsync(s->y.p, y, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
  ZCHK(hipMemcpyAsync(s->ydot.p, ydot, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
  ZCHK(hipMemcpyAsync(s->yd_prev.p, ydot, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
  s->step = step;
  s->stepped = false;
  for (int k = 0; k < s->ns; ++k)
    s->scn[k].kappa = kappa > 0.0 ? kappa : (s->P.kappa > 0.0 ? s->P.kappa : auto_kappa(s, k));
  upload_kappa(s);
  {
    const double* P[2] = {s->y.p, s->ydot.p};
    int64_t L[2] = {s->ndof, s->ndof};
    double out[3];
    k_sums(s, 2, P, L, out, nullptr);
    if (!std::isfinite(out[0]) || !std::isfinite(out[1])) throw Error(ZEMA_E_NONFINITE, "non-finite state");
  }
  if (k_any_inverted(s, s->y.p)) throw Error(ZEMA_E_MESH, "inverted tet in state");
  begin_step(s);
  for (double d : min_distance(s, s->y.p))
    if (!(d > 0.0)) throw Error(ZEMA_E_INTERSECT, "intersecting state");
  return 0;
}

// y_out = y^t + a p per scene, a the ACCD bound of that scene's sweep along p, halved
// for a scene until none of its tets inverts
void filtered_start(zema_scene* s, const double* p, double* y_out, double& tb, double& tc) {
  const int ns = s->ns;
  double q = now_ms();
  swept_candidates(s, s->y.p, p);
  tb += now_ms() - q;
  std::vector<double> a0(ns);
  std::vector<int> inv(ns);
  q = now_ms();
  int rc = k_ccd(s, s->y.p, p, a0.data());
  tc += now_ms() - q;
  if (rc) throw Error(rc, "intersecting pair at warm-start CCD");
  for (;;) {
    k_axpy_scene(s, a0.data(), p, s->y.p, y_out);
    if (!k_inverted(s, y_out, inv.data())) break;
    for (int k = 0; k < ns; ++k)
      if (inv[k]) a0[k] = a0[k] * 0.5 < 1e-10 ? 0.0 : a0[k] * 0.5;
  }
}

// One time step of every scene (Sec. III: Newton on the incremental potential with
// the intersection-free line search); scenes iterate in lockstep, a converged scene
// stops moving (its right-hand side is zeroed) until every scene has converged.
// one multiplier update of every driven body when some body misses its target by more
// than al_tol; false (nothing changed) otherwise
bool kinematic_al_update(zema_scene* s) {
  std::vector<double> y((size_t)s->ndof);
  ZCHK(hipMemcpyAsync(y.data(), s->y.p, sizeof(double) * s->ndof, hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  double worst = 0.0;
  for (size_t b = 0; b < s->bodies.size(); ++b) {
    const Body& B = s->bodies[b];
    if (B.mode != ZEMA_DRIVEN || B.dof0 < 0) continue;
    for (int k = 0; k < 12; ++k) worst = std::max(worst, std::fabs(y[B.dof0 + k] - s->qt_h[12 * b + k]));
  }
  if (!(worst > s->al_tol)) return false;
  for (size_t b = 0; b < s->bodies.size(); ++b) {
    Body& B = s->bodies[b];
    if (B.mode != ZEMA_DRIVEN || B.dof0 < 0) continue;
    const double c = B.kappaA / std::sqrt(B.m);
    for (int k = 0; k < 12; ++k) B.lamA[k] -= c * (y[B.dof0 + k] - s->qt_h[12 * b + k]);
    ZCHK(hipMemcpyAsync(s->body_f.p + (size_t)BF * b + BF_LAM, B.lamA, sizeof(double) * 12, hipMemcpyHostToDevice,
                        s->st));
  }
  ZCHK(hipStreamSynchronize(s->st));
  return true;
}

int time_step(zema_scene* s, zema_step_stats* st) {
  const double h = s->P.dt;
  const int n = s->ndof, ns = s->ns;
  for (int k = 0; k < ns; ++k) {
    std::memset(&st[k], 0, sizeof(st[k]));
    st[k].alpha_ccd_min = 1.0;
  }
  double t0 = now_ms(), tb = 0, ta = 0, tp = 0, tc = 0, tl = 0, tw = 0, q;
  q = now_ms();
  begin_step(s);
  tb += now_ms() - q;
  ZCHK(hipMemcpyAsync(s->yt.p, s->y.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s->st));
  ZCHK(hipMemcpyAsync(s->ydt.p, s->ydot.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s->st));
  std::vector<double> T((size_t)8 * ns), T1((size_t)8 * ns), E0((size_t)8 * ns);
  // initial guess: y^t + a h ydot^t with a the CCD bound of that sweep; with the
  // learned form also the network's proposal, filtered the same way and kept per
  // scene only if its energy is not higher (swept_candidates uses ytmp, so the
  // learned start is formed first, into ywarm)
  k_scale(s, n, h, s->ydot.p, s->pdir.p);
  const bool learned = s->P.warm_start == ZEMA_WARM_LEARNED;
  if (learned) {
    q = now_ms();
    s->feat.reserve((size_t)16 * s->nsv + 16);
    s->mlp_out.reserve((size_t)3 * s->nsv + 3);
    s->ywarm.reserve(n);
    k_features(s, s->feat.p);
    mlp_forward(s->mlp, s->st, s->feat.p, s->nsv, s->mlp_out.p);
    k_warm_dir(s, s->mlp_out.p, s->grad.p);
    tw += now_ms() - q;
    filtered_start(s, s->grad.p, s->ywarm.p, tb, tc);
  }
  filtered_start(s, s->pdir.p, s->ytmp.p, tb, tc);
  if (learned) {
    q = now_ms();
    static_candidates(s, s->ytmp.p);
    eval_energy(s, s->ytmp.p, T.data());
    static_candidates(s, s->ywarm.p);
    eval_energy(s, s->ywarm.p, T1.data());
    s->mask_h.assign(ns, 0);
    for (int k = 0; k < ns; ++k) {
      s->mask_h[k] = std::isfinite(T1[8 * k + 6]) && T1[8 * k + 6] <= T[8 * k + 6];
      st[k].warm_learned = s->mask_h[k];
    }
    k_select_scene(s, s->mask_h.data(), s->ywarm.p, s->ytmp.p, s->grad.p);  // grad is free here
    std::swap(s->ytmp.p, s->grad.p);
    tw += now_ms() - q;
  }
  std::swap(s->y.p, s->ytmp.p);
  q = now_ms();
  static_candidates(s, s->y.p);
  tb += now_ms() - q;
  std::vector<double> dprev = min_distance(s, s->y.p);
  const bool auto_k = s->P.kappa <= 0.0;
  const double tol = s->P.newton_tol * h;
  const int pcg_max = s->P.pcg_max;
  std::vector<int> active(ns, 1), done(ns, 0), pit(ns), pst(ns), pbd(ns);
  std::vector<double> alpha(ns), disp(ns), rr(ns);
  int n_active = ns;
  for (int it = 0; it < s->P.newton_max && n_active > 0; ++it) {
    if (ns > 1) {  // assembly skips scenes that have converged
      s->mask_h.assign(active.begin(), active.end());
      ZCHK(hipMemcpyAsync(s->sc_act.p, s->mask_h.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s->st));
      s->masked = it > 0;
    }
    q = now_ms();
    bool ok = assemble(s, s->y.p, s->grad.p, true, 0x3fu, T.data());
    ta += now_ms() - q;
    if (!ok) throw Error(ZEMA_E_INTERSECT, "infeasible Newton iterate");
    for (int k = 0; k < ns; ++k)
      if (active[k]) {
        st[k].energy = T[8 * k + 6];
        st[k].newton_iters = it;
      }
    if (ns == 1) {
      st[0].n_pt_active = s->n_act;  // active barrier pairs (point-triangle and edge-edge)
      st[0].n_ee_active = s->nfric;  // lagged friction pairs
    }
    k_scale(s, n, -1.0, s->grad.p, s->ytmp.p);
    q = now_ms();
    k_pcg_solve(s, s->ytmp.p, s->pdir.p, s->P.pcg_rtol, pcg_max, active.data(), pit.data(), rr.data(), pst.data(),
                pbd.data());
    tp += now_ms() - q;
    for (int k = 0; k < ns; ++k)
      if (active[k]) {
        st[k].pcg_iters += pit[k];
        st[k].pcg_breakdowns += pbd[k];
        if (pst[k]) throw Error(pst[k], "PCG failed");
      }
    mixed_descent_guard(s, active.data(), rr.data());
    k_max_disp(s, s->pdir.p, disp.data());
    // augmented Lagrangian of the kinematic energy (eq. 13, single scenes): at
    // convergence, while a driven body misses its target by more than al_tol, update
    // lambda_A <- lambda_A - kappa_A / sqrt(m) (q - q~) and continue from the same y
    if (ns == 1 && active[0] && disp[0] <= tol && s->al_tol > 0.0 && st[0].al_updates < s->al_max &&
        kinematic_al_update(s))
    {
      st[0].al_updates++;
      continue;
    }
    for (int k = 0; k < ns; ++k)
      if (active[k] && disp[k] <= tol) {
        active[k] = 0;
        done[k] = 1;
        --n_active;
      }
    if (n_active == 0) break;
    // finished scenes take no step: their direction is zero (they were not solved)
    if (ns > 1) {
      s->scale_h.resize(ns);
      for (int k = 0; k < ns; ++k) s->scale_h[k] = active[k] ? 1.0 : 0.0;
      k_scale_scene(s, s->scale_h.data(), s->pdir.p);
    }
    q = now_ms();
    swept_candidates(s, s->y.p, s->pdir.p);
    tb += now_ms() - q;
    if (ns == 1) {
      st[0].n_pt_cand = (int)s->npt;
      st[0].n_ee_cand = (int)s->nee;
    }
    q = now_ms();
    int rc = k_ccd(s, s->y.p, s->pdir.p, alpha.data());
    tc += now_ms() - q;
    if (rc) throw Error(rc, "intersecting pair at CCD start");
    for (int k = 0; k < ns; ++k) {
      if (!active[k]) alpha[k] = 0.0;
      else st[k].alpha_ccd_min = std::min(st[k].alpha_ccd_min, alpha[k]);
    }
    q = now_ms();
    eval_energy(s, s->y.p, E0.data());
    std::vector<int> acc(ns);
    for (int k = 0; k < ns; ++k) acc[k] = !active[k];
    for (;;) {
      k_axpy_scene(s, alpha.data(), s->pdir.p, s->y.p, s->ytmp.p);
      eval_energy(s, s->ytmp.p, T1.data());
      bool all = true;
      for (int k = 0; k < ns; ++k) {
        if (acc[k]) continue;
        if (std::isfinite(T1[8 * k + 6]) && T1[8 * k + 6] <= E0[8 * k + 6]) {
          acc[k] = 1;
          continue;
        }
        all = false;
        alpha[k] *= 0.5;
        st[k].ls_backtracks++;
        if (alpha[k] < 1e-10) throw Error(ZEMA_E_LINESEARCH, ls_failure(k, E0[8 * k + 6], T1[8 * k + 6]));
      }
      if (all) break;
    }
    tl += now_ms() - q;
    std::swap(s->y.p, s->ytmp.p);
    bool kchg = false;
    for (int k = 0; k < ns; ++k) {
      if (!active[k]) continue;
      double dm = T1[8 * k + 7];
      if (auto_k && dm < 1e-3 * s->P.dhat && dm < dprev[k]) {
        s->scn[k].kappa *= 2.0;
        kchg = true;
      }
      dprev[k] = dm;
    }
    if (kchg) upload_kappa(s);
  }
  s->masked = false;
  // the last searches of a batch left finished scenes out: candidates of every scene
  if (ns > 1) static_candidates(s, s->y.p);
  std::vector<double> dfin = min_distance(s, s->y.p);
  for (int k = 0; k < ns; ++k) {
    if (active[k]) st[k].newton_iters = s->P.newton_max;
    st[k].kappa = s->scn[k].kappa;
    st[k].d_min = dfin[k];
  }
  if (n_active > 0) {
    for (int k = 0; k < ns; ++k)
      if (active[k]) st[k].status = ZEMA_E_NEWTON;
    throw Error(ZEMA_E_NEWTON, "Newton did not converge");
  }
  ZCHK(hipMemcpyAsync(s->yd_prev.p, s->ydt.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s->st));
  k_velocity(s, 1.0 / h);
  s->step += 1;
  s->scene_step.assign(ns, s->step);
  ZCHK(hipStreamSynchronize(s->st));
  kt_fold(s);
  double tt = now_ms() - t0;
  for (int k = 0; k < ns; ++k) {
    st[k].ms_total = tt;
    st[k].ms_assemble = ta;
    st[k].ms_pcg = tp;
    st[k].ms_broad = tb;
    st[k].ms_ccd = tc;
    st[k].ms_linesearch = tl;
    st[k].ms_warm = tw;
  }
  return 0;
}


// n_steps time steps of every scene of a batch, each scene starting its next step as
// soon as its Newton loop has converged (scenes are independent; only the launches
// are shared).  Every global iteration: one Newton iteration (assembly, PCG,
// convergence) of the scenes inside a step; the start of a step (predictor, targets,
// lagged friction, explicit initial guess) of the scenes between steps; one shared
// swept candidate search (the Newton direction, or h ydot^t for a starting scene),
// one CCD pass and one backtracking loop (energy and inversion for an iterate,
// inversion for an initial guess).  Per scene the arithmetic is that of time_step;
// the candidate set of an initial guess is the swept set of h ydot^t (a superset of
// the pairs within d-hat at y^t and at the guess).  stats: [n_steps][ns].
int time_steps_async(zema_scene* s, int n_steps, zema_step_stats* stats) {
  const double h = s->P.dt;
  const int n = s->ndof, ns = s->ns;
  for (int k = 0; k < n_steps * ns; ++k) {
    std::memset(&stats[k], 0, sizeof(stats[k]));
    stats[k].alpha_ccd_min = 1.0;
  }
  if (s->scene_step.size() != (size_t)ns) s->scene_step.assign(ns, s->step);
  enum { BEGIN = 0, NEWTON = 1, FINISHED = 2 };
  std::vector<int> phase(ns, n_steps > 0 ? BEGIN : FINISHED), done(ns, 0), it(ns, 0);
  std::vector<int> inN(ns), inB(ns), live(ns), fin(ns), pit(ns), pst(ns), pbd(ns), inv(ns), acc(ns);
  std::vector<double> alpha(ns), disp(ns), rr(ns), dprev(ns, INFINITY), scale(ns), t0s(ns, now_ms());
  std::vector<double> T((size_t)8 * ns), T1((size_t)8 * ns), E0((size_t)8 * ns), T2((size_t)8 * ns);
  std::vector<double> alpha2(ns, 0.0);
  std::vector<int> use2(ns, 0);
  const bool learned = s->P.warm_start == ZEMA_WARM_LEARNED;
  double tw = 0;
  auto cur = [&](int k) -> zema_step_stats& { return stats[(size_t)done[k] * ns + k]; };
  const bool auto_k = s->P.kappa <= 0.0;
  const double tol = s->P.newton_tol * h;
  double ta = 0, tp = 0, tb = 0, tc = 0, tl = 0, q;
  // phase times of a global iteration go to the step each scene was in
  auto charge = [&](int k, int step, double dt_a, double dt_p, double dt_b, double dt_c, double dt_l) {
    zema_step_stats& st = stats[(size_t)step * ns + k];
    st.ms_assemble += dt_a;
    st.ms_pcg += dt_p;
    st.ms_broad += dt_b;
    st.ms_ccd += dt_c;
    st.ms_linesearch += dt_l;
  };
  std::vector<int> wasN(ns);
  for (;;) {
    int nN = 0, nB = 0;
    for (int k = 0; k < ns; ++k) {
      inN[k] = phase[k] == NEWTON;
      inB[k] = phase[k] == BEGIN;
      nN += inN[k];
      nB += inB[k];
    }
    if (nN + nB == 0) break;
    ta = tp = tb = tc = tl = tw = 0;
    std::fill(fin.begin(), fin.end(), 0);
    wasN = inN;
    // ---- one Newton iteration of the scenes inside a step
    if (nN) {
      ZCHK(hipMemcpyAsync(s->sc_act.p, inN.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s->st));
      s->masked = true;
      q = now_ms();
      bool ok = assemble(s, s->y.p, s->grad.p, true, 0x3fu, T.data());
      ta += now_ms() - q;
      if (!ok) throw Error(ZEMA_E_INTERSECT, "infeasible Newton iterate");
      for (int k = 0; k < ns; ++k)
        if (inN[k]) {
          cur(k).energy = T[8 * k + 6];
          cur(k).newton_iters = it[k];
        }
      k_scale(s, n, -1.0, s->grad.p, s->ytmp.p);
      q = now_ms();
      k_pcg_solve(s, s->ytmp.p, s->pdir.p, s->P.pcg_rtol, s->P.pcg_max, inN.data(), pit.data(), rr.data(),
                  pst.data(), pbd.data());
      tp += now_ms() - q;
      for (int k = 0; k < ns; ++k)
        if (inN[k]) {
          cur(k).pcg_iters += pit[k];
          cur(k).pcg_breakdowns += pbd[k];
          if (pst[k]) throw Error(pst[k], "PCG failed");
        }
      mixed_descent_guard(s, inN.data(), rr.data());
      k_max_disp(s, s->pdir.p, disp.data());
      for (int k = 0; k < ns; ++k)
        if (inN[k] && disp[k] <= tol) {
          fin[k] = 1;
          inN[k] = 0;
          --nN;
        }
    }
    // ---- scenes that converged end their step: velocity, statistics
    bool any_fin = false;
    for (int k = 0; k < ns; ++k) any_fin = any_fin || fin[k];
    if (any_fin) {
      k_select_scene(s, fin.data(), s->ydt.p, s->yd_prev.p, s->yd_prev.p);
      k_velocity_to(s, 1.0 / h, s->ytmp.p);
      k_select_scene(s, fin.data(), s->ytmp.p, s->ydot.p, s->ydot.p);
      for (int k = 0; k < ns; ++k) {
        if (!fin[k]) continue;
        zema_step_stats& st = cur(k);
        st.kappa = s->scn[k].kappa;
        st.d_min = T[8 * k + 7];
        st.ms_total = now_ms() - t0s[k];
        s->scene_step[k] += 1;
        done[k] += 1;
        phase[k] = done[k] < n_steps ? BEGIN : FINISHED;
        if (phase[k] == BEGIN) {
          inB[k] = 1;
          ++nB;
        }
      }
    }
    // ---- the start of a step: y^t, ydot^t, predictor, targets, kappa_lag
    if (nB) {
      for (int k = 0; k < ns; ++k)
        if (inB[k]) t0s[k] = now_ms();
      k_select_scene(s, inB.data(), s->y.p, s->yt.p, s->yt.p);
      k_select_scene(s, inB.data(), s->ydot.p, s->ydt.p, s->ydt.p);
      k_predict_to(s, s->ytmp.p);
      k_select_scene(s, inB.data(), s->ytmp.p, s->yhat.p, s->yhat.p);
      body_targets(s, inB.data());
      for (int k = 0; k < ns; ++k)
        if (inB[k]) s->scn[k].kappa_lag = s->scn[k].kappa;
      // explicit initial-guess direction h ydot^t
      k_scale(s, n, h, s->ydot.p, s->ytmp.p);
      k_select_scene(s, inB.data(), s->ytmp.p, s->pdir.p, s->pdir.p);
      if (learned) {  // the network's direction of the starting scenes (its own search)
        q = now_ms();
        ZCHK(hipMemcpyAsync(s->sc_act.p, inB.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s->st));
        s->masked = true;
        s->feat.reserve((size_t)16 * s->nsv + 16);
        s->mlp_out.reserve((size_t)3 * s->nsv + 3);
        s->ywarm.reserve(n);
        s->pdir2.reserve(n);
        k_features(s, s->feat.p);
        mlp_forward(s->mlp, s->st, s->feat.p, s->nsv, s->mlp_out.p);
        k_warm_dir(s, s->mlp_out.p, s->pdir2.p);
        for (int k = 0; k < ns; ++k) scale[k] = inB[k] ? 1.0 : 0.0;
        k_scale_scene(s, scale.data(), s->pdir2.p);
        tw += now_ms() - q;
      }
    }
    const bool two = learned && nB > 0;  // a second proposal of the starting scenes
    // directions of scenes that take no move are zero
    for (int k = 0; k < ns; ++k) {
      live[k] = inN[k] || inB[k];
      scale[k] = live[k] ? 1.0 : 0.0;
    }
    k_scale_scene(s, scale.data(), s->pdir.p);
    // ---- shared swept search over the moving scenes, friction of the starting ones
    ZCHK(hipMemcpyAsync(s->sc_act.p, live.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s->st));
    s->masked = true;
    q = now_ms();
    if (two) {  // boxes over y, y + p and y + p2: both proposals of a starting scene
      k_axpy(s, n, 1.0, s->pdir.p, s->y.p, s->ytmp.p);
      k_map_surface(s, s->y.p, s->xs.p);
      k_map_surface(s, s->ytmp.p, s->xs1.p);
      k_axpy(s, n, 1.0, s->pdir2.p, s->y.p, s->ytmp.p);
      k_map_surface(s, s->ytmp.p, s->xs2.p);
      k_candidates(s, s->xs.p, s->xs1.p, s->P.dhat, s->xs2.p);
    } else {
      swept_candidates(s, s->y.p, s->pdir.p);
    }
    if (nB) k_friction_rebuild(s, inB.data());
    tb += now_ms() - q;
    q = now_ms();
    int rc = k_ccd(s, s->y.p, s->pdir.p, alpha.data());
    if (!rc && two) rc = k_ccd(s, s->y.p, s->pdir2.p, alpha2.data());
    tc += now_ms() - q;
    if (rc) throw Error(rc, "intersecting pair at CCD start");
    for (int k = 0; k < ns; ++k) {
      if (!live[k]) alpha[k] = 0.0;
      else if (inN[k]) cur(k).alpha_ccd_min = std::min(cur(k).alpha_ccd_min, alpha[k]);
    }
    // ---- backtracking: an iterate needs no energy increase (and no inverted tet, where
    // the energy is infinite), an initial guess no inverted tet
    q = now_ms();
    if (two) {  // the network's proposal: halved while a tet inverts, then its energy
      for (int k = 0; k < ns; ++k)
        if (!inB[k]) alpha2[k] = 0.0;
      for (;;) {
        k_axpy_scene(s, alpha2.data(), s->pdir2.p, s->y.p, s->ywarm.p);
        if (!k_inverted(s, s->ywarm.p, inv.data())) break;
        for (int k = 0; k < ns; ++k)
          if (inB[k] && inv[k]) alpha2[k] = alpha2[k] * 0.5 < 1e-10 ? 0.0 : alpha2[k] * 0.5;
      }
      eval_energy(s, s->ywarm.p, T2.data());
    }
    if (nN) eval_energy(s, s->y.p, E0.data());
    for (int k = 0; k < ns; ++k) acc[k] = !live[k];
    std::fill(use2.begin(), use2.end(), 0);
    for (;;) {
      k_axpy_scene(s, alpha.data(), s->pdir.p, s->y.p, s->ytmp.p);
      eval_energy(s, s->ytmp.p, T1.data());
      if (nB) k_inverted(s, s->ytmp.p, inv.data());
      bool all = true;
      for (int k = 0; k < ns; ++k) {
        if (acc[k]) continue;
        if (inN[k]) {
          if (std::isfinite(T1[8 * k + 6]) && T1[8 * k + 6] <= E0[8 * k + 6]) {
            acc[k] = 1;
            double dm = T1[8 * k + 7];
            if (auto_k && dm < 1e-3 * s->P.dhat && dm < dprev[k]) s->scn[k].kappa *= 2.0;
            dprev[k] = dm;
            continue;
          }
          all = false;
          alpha[k] *= 0.5;
          cur(k).ls_backtracks++;
          if (alpha[k] < 1e-10) throw Error(ZEMA_E_LINESEARCH, ls_failure(k, E0[8 * k + 6], T1[8 * k + 6]));
        } else {  // initial guess of a starting scene
          if (!inv[k]) {
            acc[k] = 1;
            dprev[k] = T1[8 * k + 7];
            // the network's proposal is kept when its energy is not higher
            if (two && std::isfinite(T2[8 * k + 6]) && T2[8 * k + 6] <= T1[8 * k + 6]) {
              use2[k] = 1;
              dprev[k] = T2[8 * k + 7];
            }
            cur(k).warm_learned = use2[k];
            continue;
          }
          all = false;
          alpha[k] = alpha[k] * 0.5 < 1e-10 ? 0.0 : alpha[k] * 0.5;
        }
      }
      if (all) break;
    }
    tl += now_ms() - q;
    if (two) k_select_scene(s, use2.data(), s->ywarm.p, s->ytmp.p, s->ytmp.p);
    std::swap(s->y.p, s->ytmp.p);
    upload_kappa(s);
    for (int k = 0; k < ns; ++k) {
      if (inN[k]) {
        if (++it[k] >= s->P.newton_max) {
          cur(k).status = ZEMA_E_NEWTON;
          throw Error(ZEMA_E_NEWTON, "Newton did not converge");
        }
      }
      if (inB[k]) {
        phase[k] = NEWTON;
        it[k] = 0;
      }
      if (fin[k]) charge(k, done[k] - 1, ta, tp, 0.0, 0.0, 0.0);  // the step it finished
      if (live[k]) charge(k, done[k], wasN[k] && !fin[k] ? ta : 0.0, wasN[k] && !fin[k] ? tp : 0.0, tb, tc, tl);
      if (inB[k]) stats[(size_t)done[k] * ns + k].ms_warm += tw;
    }
  }
  s->masked = false;
  s->step += n_steps;
  ZCHK(hipStreamSynchronize(s->st));
  kt_fold(s);
  return 0;
}
}  // namespace

// ------------------------------------------------------------------ launch timing
namespace zema {
void kt_begin(zema_scene* s, int g) {
  KTimer& t = s->kt[g];
  if (!t.on) return;
  if (t.used + 2 > t.ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      ZCHK(hipEventCreate(&e));
      t.ev.push_back(e);
    }
  }
  ZCHK(hipEventRecord(t.ev[t.used], s->st));
}
void kt_end(zema_scene* s, int g, double bytes) {
  KTimer& t = s->kt[g];
  if (!t.on) return;
  ZCHK(hipEventRecord(t.ev[t.used + 1], s->st));
  t.used += 2;
  t.pending.push_back(bytes);
}
void kt_fold(zema_scene* s) {
  for (KTimer& t : s->kt) {
    for (size_t k = 0; k + 1 < t.used; k += 2) {
      float ms = 0.0f;
      ZCHK(hipEventSynchronize(t.ev[k + 1]));
      ZCHK(hipEventElapsedTime(&ms, t.ev[k], t.ev[k + 1]));
      t.ms += ms;
      t.launches++;
      t.bytes += t.pending[k / 2];
    }
    t.used = 0;
    t.pending.clear();
  }
}
void kt_add(zema_scene* s, int g, double ms, double bytes, long long launches) {
  KTimer& t = s->kt[g];
  if (!t.on) return;
  t.ms += ms;
  t.launches += launches;
  t.bytes += bytes;
}
}  // namespace zema

zema_scene::~zema_scene() {
  for (zema::KTimer& t : kt)
    for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  if (pcg_graph.exec) (void)hipGraphExecDestroy(pcg_graph.exec);
  if (cap_st) (void)hipStreamDestroy(cap_st);
  for (hipEvent_t e : poll_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : chunk_ev)
    if (e) (void)hipEventDestroy(e);
  if (poll_h) (void)hipHostFree(poll_h);
}

namespace {

template <class F>
int guard(zema_scene* s, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    if (s) s->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (s) s->err = e.what();
    return ZEMA_E_DEVICE;
  }
}

}  // namespace

// ================================================================== C interface
extern "C" {

const char* zema_status_string(int st) {
  switch (st) {
    case ZEMA_OK: return "ok";
    case ZEMA_E_ARG: return "invalid argument";
    case ZEMA_E_MESH: return "degenerate or inverted mesh";
    case ZEMA_E_INTERSECT: return "intersecting state";
    case ZEMA_E_CAPACITY: return "output capacity too small";
    case ZEMA_E_NEWTON: return "Newton did not converge";
    case ZEMA_E_LINESEARCH: return "line search failed";
    case ZEMA_E_PCG: return "PCG breakdown or no convergence";
    case ZEMA_E_NONFINITE: return "non-finite value";
    case ZEMA_E_DEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* zema_last_error(const zema_scene* s) { return s ? s->err.c_str() : "null scene"; }

int zema_scene_create(const zema_params* params, const zema_soft_desc* soft, int32_t n_soft,
                      const zema_affine_desc* affine, int32_t n_affine, void* hip_stream, zema_scene** out) {
  if (!params || !out || n_soft < 0 || n_affine < 0 || (n_soft && !soft) || (n_affine && !affine)) return ZEMA_E_ARG;
  if (!(params->dt > 0.0) || !(params->dhat > 0.0)) return ZEMA_E_ARG;
  if (params->precision != ZEMA_FP64 && params->precision != ZEMA_MIXED) return ZEMA_E_ARG;
  if (params->warm_start != ZEMA_WARM_EXPLICIT && params->warm_start != ZEMA_WARM_LEARNED) return ZEMA_E_ARG;
  zema_scene* s = new zema_scene();
  s->P = *params;
  s->st = (hipStream_t)hip_stream;
  int rc = guard(s, [&]() {
    int so[2] = {0, n_soft}, ao[2] = {0, n_affine};
    double mu = params->mu;
    build_scene(s, soft, n_soft, affine, n_affine, so, ao, 1, &mu);
    return set_state_impl(s, s->ytmp.p, s->pdir.p, 0.0, 0);
  });
  if (rc) {
    delete s;
    return rc;
  }
  *out = s;
  return 0;
}

int zema_batch_create(const zema_params* params, int32_t n_scenes, const zema_soft_desc* soft,
                      const int32_t* soft_off, const zema_affine_desc* affine, const int32_t* aff_off,
                      void* hip_stream, zema_scene** out) {
  if (!params || !out || n_scenes <= 0 || !soft_off || !aff_off) return ZEMA_E_ARG;
  *out = nullptr;
  const zema_params& P0 = params[0];
  for (int k = 0; k < n_scenes; ++k) {
    const zema_params& P = params[k];
    if (!(P.dt > 0.0) || !(P.dhat > 0.0)) return ZEMA_E_ARG;
    if (P.precision != ZEMA_FP64 && P.precision != ZEMA_MIXED) return ZEMA_E_ARG;
    if (P.warm_start != ZEMA_WARM_EXPLICIT && P.warm_start != ZEMA_WARM_LEARNED) return ZEMA_E_ARG;
    // everything but the friction coefficient is shared by the scenes of a batch
    bool same = P.dt == P0.dt && P.dhat == P0.dhat && P.kappa == P0.kappa && P.eps_v == P0.eps_v &&
                P.gravity[0] == P0.gravity[0] && P.gravity[1] == P0.gravity[1] && P.gravity[2] == P0.gravity[2] &&
                P.newton_tol == P0.newton_tol && P.pcg_rtol == P0.pcg_rtol && P.ccd_s == P0.ccd_s &&
                P.newton_max == P0.newton_max && P.pcg_max == P0.pcg_max && P.precision == P0.precision &&
                P.warm_start == P0.warm_start;
    if (!same) return ZEMA_E_ARG;
  }
  int n_soft = soft_off[n_scenes], n_aff = aff_off[n_scenes];
  if (n_soft < 0 || n_aff < 0 || (n_soft && !soft) || (n_aff && !affine)) return ZEMA_E_ARG;
  zema_scene* s = new zema_scene();
  s->P = P0;
  s->st = (hipStream_t)hip_stream;
  int rc = guard(s, [&]() {
    std::vector<double> mu(n_scenes);
    for (int k = 0; k < n_scenes; ++k) mu[k] = params[k].mu;
    build_scene(s, soft, n_soft, affine, n_aff, soft_off, aff_off, n_scenes, mu.data());
    return set_state_impl(s, s->ytmp.p, s->pdir.p, 0.0, 0);
  });
  if (rc) {
    delete s;
    return rc;
  }
  *out = s;
  return 0;
}

int zema_batch_layout(const zema_scene* s, int32_t* n_scenes, int64_t* ranges) {
  if (!s || !n_scenes) return ZEMA_E_ARG;
  *n_scenes = s->ns;
  if (ranges)
    for (int k = 0; k < s->ns; ++k) {
      const SceneRange& R = s->scn[k];
      int64_t r[8] = {R.v0, R.v1, R.f0, R.f1, R.t0, R.t1, R.s0, R.s1};
      for (int q = 0; q < 8; ++q) ranges[8 * k + q] = r[q];
    }
  return 0;
}

void zema_scene_destroy(zema_scene* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  delete s;
}

int zema_sizes(const zema_scene* s, int64_t* o) {
  if (!s || !o) return ZEMA_E_ARG;
  o[0] = s->ndof;
  o[1] = s->nsv;
  o[2] = s->nt;
  o[3] = s->nsurf;
  o[4] = s->ntri;
  o[5] = s->nedge;
  o[6] = s->nfree;
  o[7] = s->n_bodies;
  return 0;
}

int zema_set_state(zema_scene* s, const double* y, const double* ydot, double kappa, int32_t step) {
  if (!s || !y || !ydot) return ZEMA_E_ARG;
  return guard(s, [&]() { return set_state_impl(s, y, ydot, kappa, step); });
}

int zema_get_state(zema_scene* s, double* y, double* ydot, double* kappa, int32_t* step) {
  if (!s) return ZEMA_E_ARG;
  return guard(s, [&]() {
    if (y) ZCHK(hipMemcpyAsync(y, s->y.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
    if (ydot) ZCHK(hipMemcpyAsync(ydot, s->ydot.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    if (kappa) *kappa = s->scn[0].kappa;
    if (step) *step = s->step;
    return 0;
  });
}

int zema_set_kappa(zema_scene* s, double kappa) {
  if (!s || !(kappa > 0.0)) return ZEMA_E_ARG;
  return guard(s, [&]() {
    for (SceneRange& R : s->scn) R.kappa = kappa;
    upload_kappa(s);
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_surface_positions(zema_scene* s, const double* y, double* xs) {
  if (!s || !y || !xs) return ZEMA_E_ARG;
  return guard(s, [&]() {
    k_map_surface(s, y, xs);
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_contact_candidates(zema_scene* s, const double* xs0, const double* xs1, double r, int32_t* pt, int64_t pt_cap,
                            int64_t* n_pt, int32_t* ee, int64_t ee_cap, int64_t* n_ee) {
  if (!s || !xs0 || !n_pt || !n_ee || !(r >= 0.0)) return ZEMA_E_ARG;
  return guard(s, [&]() {
    k_candidates(s, xs0, xs1 ? xs1 : xs0, r);
    *n_pt = s->npt;
    *n_ee = s->nee;
    if (s->npt > pt_cap || s->nee > ee_cap) throw Error(ZEMA_E_CAPACITY, "candidate capacity");
    if (s->npt) ZCHK(hipMemcpyAsync(pt, s->pt.p, sizeof(int) * 2 * s->npt, hipMemcpyDeviceToDevice, s->st));
    if (s->nee) ZCHK(hipMemcpyAsync(ee, s->ee.p, sizeof(int) * 2 * s->nee, hipMemcpyDeviceToDevice, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_ip_assemble(zema_scene* s, const double* y, uint32_t flags, double* terms, double* grad) {
  if (!s || !y || !terms || s->ns != 1) return ZEMA_E_ARG;
  if ((flags & ZEMA_GRAD) && !grad) return ZEMA_E_ARG;
  return guard(s, [&]() {
    unsigned mask = (flags >> ZEMA_TERMS_SHIFT) & 0x3fu;
    if (!mask) mask = 0x3fu;
    if (flags & ZEMA_REBUILD) static_candidates(s, y);
    double T[8];
    assemble(s, y, (flags & ZEMA_GRAD) ? s->grad.p : nullptr, (flags & ZEMA_HESS) != 0, mask, T);
    std::memcpy(terms, T, sizeof(T));
    if (!std::isfinite(T[6])) throw Error(ZEMA_E_INTERSECT, "infeasible state (inverted tet or zero distance)");
    if (flags & ZEMA_GRAD)
      ZCHK(hipMemcpyAsync(grad, s->grad.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_hessian_matvec(zema_scene* s, const double* v, double* out) {
  if (!s || !v || !out) return ZEMA_E_ARG;
  if (!s->hess_valid) return ZEMA_E_ARG;
  return guard(s, [&]() {
    k_hess_matvec(s, v, out);
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_hessian_bsr(zema_scene* s, int32_t* row_ptr, int32_t* col, double* val, int64_t cap, int64_t* nnzb) {
  if (!s || !nnzb || cap < 0 || s->ns != 1) return ZEMA_E_ARG;
  if (!s->hess_valid) return ZEMA_E_ARG;
  return guard(s, [&]() {
    int64_t n = k_hessian_bsr(s, row_ptr, col, val, cap);
    *nnzb = n;
    if (n > cap || (n > 0 && (!row_ptr || !col || !val))) throw Error(ZEMA_E_CAPACITY, "BSR capacity");
    if (!n && row_ptr) {
      ZCHK(hipMemsetAsync(row_ptr, 0, sizeof(int) * ((size_t)s->nnodes + 1), s->st));
      ZCHK(hipStreamSynchronize(s->st));
    }
    return 0;
  });
}

int zema_surface_view(zema_scene* s, int32_t* tris, int32_t* edges, int32_t* vbody, int32_t* vsrc) {
  if (!s) return ZEMA_E_ARG;
  return guard(s, [&]() {
    if (tris && s->ntri)
      ZCHK(hipMemcpyAsync(tris, s->tris.p, sizeof(int) * 3 * s->ntri, hipMemcpyDeviceToDevice, s->st));
    if (edges && s->nedge)
      ZCHK(hipMemcpyAsync(edges, s->edges.p, sizeof(int) * 2 * s->nedge, hipMemcpyDeviceToDevice, s->st));
    if (vbody && s->nsurf)
      ZCHK(hipMemcpyAsync(vbody, s->sv_body.p, sizeof(int) * s->nsurf, hipMemcpyDeviceToDevice, s->st));
    if (vsrc && s->nsurf)
      ZCHK(hipMemcpyAsync(vsrc, s->sv_ref.p, sizeof(int) * s->nsurf, hipMemcpyDeviceToDevice, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_pcg_solve(zema_scene* s, const double* rhs, double* sol, double rtol, int32_t max_iter, int32_t* iters,
                   double* rel_res) {
  if (!s || !rhs || !sol || !iters || !rel_res || !s->hess_valid || s->ns != 1) return ZEMA_E_ARG;
  return guard(s, [&]() {
    int it = 0, one = 1, rc = 0, bd = 0;
    double rr = 0.0;
    k_pcg_solve(s, rhs, sol, rtol, max_iter, &one, &it, &rr, &rc, &bd);
    *iters = it;
    *rel_res = rr;
    if (rc) throw Error(rc, "PCG no convergence or singular preconditioner block");
    if (bd && !s->mixed) throw Error(ZEMA_E_PCG, "PCG breakdown: non-positive curvature");
    return 0;
  });
}

int zema_ccd_max_step(zema_scene* s, const double* y, const double* p, double* alpha) {
  if (!s || !y || !p || !alpha || s->ns != 1) return ZEMA_E_ARG;
  return guard(s, [&]() {
    swept_candidates(s, y, p);
    int rc = k_ccd(s, y, p, alpha);
    if (rc) throw Error(rc, "intersecting pair at CCD start");
    return 0;
  });
}

int zema_step(zema_scene* s, int32_t n_steps, zema_step_stats* stats) {
  if (!s || n_steps < 0 || (n_steps && !stats)) return ZEMA_E_ARG;
  if (s->P.warm_start == ZEMA_WARM_LEARNED && !s->mlp) {
    s->err = "learned initial guess selected but no network attached";
    return ZEMA_E_ARG;
  }
  if (s->ns > 1 && s->batch_async && n_steps > 0) {
    // scenes of a batch start their next step as they converge; a failure returns every
    // scene to the start of the step it was in (y^t, ydot^t are kept per scene)
    int rc = guard(s, [&]() {
      ZCHK(hipMemcpyAsync(s->yt.p, s->y.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
      ZCHK(hipMemcpyAsync(s->ydt.p, s->ydot.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
      return time_steps_async(s, n_steps, stats);
    });
    s->masked = false;
    s->stepped = rc == 0;
    if (rc) {
      for (int k = 0; k < n_steps * s->ns; ++k)
        if (stats[k].ms_total == 0.0) stats[k].status = rc;  // steps that did not complete
      (void)hipMemcpyAsync(s->y.p, s->yt.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st);
      (void)hipMemcpyAsync(s->ydot.p, s->ydt.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st);
      (void)hipStreamSynchronize(s->st);
      // each scene keeps the steps it completed; the batch's count is the least of them
      s->step = *std::min_element(s->scene_step.begin(), s->scene_step.end());
    }
    return rc;
  }
  for (int k = 0; k < n_steps; ++k) {
    // y^t / ydot^t are saved first so a failed step can restore them
    int rc = guard(s, [&]() {
      ZCHK(hipMemcpyAsync(s->yt.p, s->y.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
      ZCHK(hipMemcpyAsync(s->ydt.p, s->ydot.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
      return time_step(s, &stats[(size_t)k * s->ns]);
    });
    for (int j = 0; j < s->ns; ++j) stats[(size_t)k * s->ns + j].status = rc;
    s->stepped = rc == 0;
    s->masked = false;
    if (rc) {
      // restore y^t and ydot^t of the failed step
      (void)hipMemcpyAsync(s->y.p, s->yt.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st);
      (void)hipMemcpyAsync(s->ydot.p, s->ydt.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st);
      (void)hipStreamSynchronize(s->st);
      return rc;
    }
  }
  return 0;
}

// contact forces (N) per body at y on the static candidate set at y (host out)
static void contact_forces(zema_scene* s, const double* y, double* out) {
  static_candidates(s, y);
  double T[8];
  if (!assemble(s, y, s->grad.p, false, 16u, T)) throw Error(ZEMA_E_INTERSECT, "infeasible state");
  k_body_forces(s, out);
}

int zema_contact_forces(zema_scene* s, const double* y, double* forces) {
  if (!s || !y || !forces) return ZEMA_E_ARG;
  return guard(s, [&]() {
    contact_forces(s, y, forces);
    return 0;
  });
}

int zema_set_drive_target(zema_scene* s, int32_t body, const double* q) {
  if (!s || body < 0 || body >= (int)s->bodies.size() || s->bodies[body].mode != ZEMA_DRIVEN) return ZEMA_E_ARG;
  Body& B = s->bodies[body];
  if (q) {
    const double* prev = B.has_target ? B.target : (s->qt_h.size() >= 12 * (size_t)(body + 1) ? &s->qt_h[12 * body]
                                                                                            : B.qrest);
    for (int k = 0; k < 3; ++k) B.target_vel[k] = (q[k] - prev[k]) / s->P.dt;
    for (int k = 0; k < 12; ++k) B.target[k] = q[k];
  }
  B.has_target = q != nullptr;
  return 0;
}

int zema_set_springs(zema_scene* s, int32_t n, const int32_t* sv, const double* k, const double* targets) {
  if (!s || n < 0 || (n && (!sv || !k || !targets)) || (n && s->ns != 1)) return ZEMA_E_ARG;
  std::vector<Spring> v;
  std::vector<char> seen(std::max(s->nsurf, 1), 0);
  for (int i = 0; i < n; ++i) {
    if (sv[i] < 0 || sv[i] >= s->nsurf || seen[sv[i]] || !(k[i] >= 0.0)) return ZEMA_E_ARG;
    seen[sv[i]] = 1;
    Spring sp;
    sp.sv = sv[i];
    sp.k = k[i];
    for (int c = 0; c < 3; ++c) sp.target[c] = targets[3 * i + c];
    v.push_back(sp);
  }
  return guard(s, [&]() {
    std::vector<int> ids;
    std::vector<double> kt;
    for (const Spring& sp : v) {
      ids.push_back(sp.sv);
      kt.push_back(sp.k);
      for (int c = 0; c < 3; ++c) kt.push_back(sp.target[c]);
    }
    s->spr_sv.upload(ids, s->st);
    s->spr_kt.upload(kt, s->st);
    s->e_spr.reserve(v.size() + s->joints.size() + 1);
    s->springs = v;
    s->hess_valid = false;
    return 0;
  });
}

int zema_set_prismatic_joints(zema_scene* s, int32_t n, const int32_t* b12, const double* axes, const double* kappa) {
  if (!s || n < 0 || (n && (!b12 || !axes || !kappa)) || (n && s->ns != 1)) return ZEMA_E_ARG;
  const int nb = (int)s->bodies.size();
  std::vector<Joint> v;
  std::vector<double> jd;
  for (int i = 0; i < n; ++i) {
    Joint J;
    J.b1 = b12[2 * i];
    J.b2 = b12[2 * i + 1];
    if (J.b1 < 0 || J.b1 >= nb || J.b2 < 0 || J.b2 >= nb || J.b1 == J.b2 || !(kappa[i] >= 0.0)) return ZEMA_E_ARG;
    if (s->bodies[J.b1].dof0 < 0 && s->bodies[J.b2].dof0 < 0) return ZEMA_E_ARG;
    for (int k = 0; k < 3; ++k) J.d[k] = axes[3 * i + k];
    J.kappa = kappa[i];
    v.push_back(J);
    for (int k = 0; k < 3; ++k) jd.push_back(J.d[k]);
    jd.push_back(J.kappa);
    for (int k = 0; k < 3; ++k) jd.push_back(s->bodies[J.b1].c[k] - s->bodies[J.b2].c[k]);
    jd.push_back(0.0);
  }
  // per joint: bodies and the offsets of its triplets (gradient per node of a non-fixed
  // body, then with the Hessian every node pair) within the joints' block
  std::vector<int> ji;
  int off_h = 0, off_g = 0;
  for (const Joint& J : v) {
    const int nodes = 4 * ((s->bodies[J.b1].dof0 >= 0) + (s->bodies[J.b2].dof0 >= 0));
    ji.insert(ji.end(), {J.b1, J.b2, off_h, off_g});
    off_h += nodes + nodes * nodes;
    off_g += nodes;
  }
  return guard(s, [&]() {
    s->jnt_d.upload(jd, s->st);
    s->jnt_i.upload(ji, s->st);
    s->joints = v;
    s->e_spr.reserve(s->springs.size() + v.size() + 1);
    s->hess_valid = false;
    return 0;
  });
}

int zema_kinematic_al(zema_scene* s, double tol, int32_t max_updates, double* lam) {
  if (!s || !(tol >= 0.0) || max_updates < 0 || (tol > 0.0 && s->ns != 1)) return ZEMA_E_ARG;
  s->al_tol = tol;
  s->al_max = max_updates;
  if (lam)
    for (size_t b = 0; b < s->bodies.size(); ++b)
      for (int k = 0; k < 12; ++k) lam[12 * b + k] = s->bodies[b].lamA[k];
  return 0;
}

// the force controller of Sec. IV-A eq. 12
static double phi_control(double f, double k, double fs) {
  if (!(f < fs)) return 0.0;
  return (std::exp(-k * f) - std::exp(-k * fs)) / (1.0 - std::exp(-k * fs));
}

int zema_grasp_run(zema_scene* s, const zema_grasp_params* gp, zema_grasp_result* res, double* trace,
                   int32_t trace_cap) {
  if (!s || !gp || !res || s->ns != 1 || trace_cap < 0 || (trace_cap && !trace)) return ZEMA_E_ARG;
  if (!(gp->k > 0.0) || !(gp->f_star > 0.0) || gp->max_close_steps < 0 || gp->lift_steps < 0 ||
      gp->shake_steps < 0 || gp->object_body < 0 || gp->object_body >= s->n_bodies ||
      gp->ground_body >= s->n_bodies)
    return ZEMA_E_ARG;
  std::vector<int> fingers;
  for (int b = 0; b < (int)s->bodies.size(); ++b)
    if (s->bodies[b].mode == ZEMA_DRIVEN) fingers.push_back(b);
  const int nf = (int)fingers.size();
  *res = zema_grasp_result{};
  res->n_fingers = nf;
  if (!nf) return ZEMA_E_ARG;
  const int nsb = s->n_soft_bodies;
  return guard(s, [&]() {
    const double h = s->P.dt;
    const double gn = std::sqrt(s->P.gravity[0] * s->P.gravity[0] + s->P.gravity[1] * s->P.gravity[1] +
                                s->P.gravity[2] * s->P.gravity[2]);
    double up[3] = {0.0, 1.0, 0.0};
    if (gn > 0.0)
      for (int k = 0; k < 3; ++k) up[k] = -s->P.gravity[k] / gn;
    std::vector<double> F((size_t)3 * s->n_bodies), y((size_t)s->ndof);
    std::vector<double> fmag(nf);
    double fground = 0.0;
    auto measure = [&]() {
      contact_forces(s, s->y.p, F.data());
      for (int i = 0; i < nf; ++i) {
        const double* f = &F[3 * (nsb + fingers[i])];
        fmag[i] = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
      }
      fground = 0.0;
      if (gp->ground_body >= 0) {
        const double* f = &F[3 * gp->ground_body];
        fground = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
      }
    };
    int phase = 0, in_phase = 0, n = 0;
    const double two_pi = 6.283185307179586476925;
    for (;;) {
      measure();
      if (phase == 0) {
        bool all_zero = true;
        for (int i = 0; i < nf; ++i) all_zero = all_zero && phi_control(fmag[i], gp->k, gp->f_star) == 0.0;
        if (all_zero || in_phase >= gp->max_close_steps) {
          res->close_steps = in_phase;
          phase = 1;
          in_phase = 0;
        }
      }
      if (phase == 1 && in_phase >= gp->lift_steps) {
        phase = 2;
        in_phase = 0;
      }
      if (phase == 2 && in_phase >= gp->shake_steps) break;
      if (trace && n < trace_cap) {
        double* row = trace + (size_t)n * (2 + nf);
        row[0] = phase;
        row[1] = fground;
        for (int i = 0; i < nf; ++i) row[2 + i] = fmag[i];
      }
      // each finger's target: its current state plus the phase's increment
      ZCHK(hipMemcpyAsync(y.data(), s->y.p, sizeof(double) * s->ndof, hipMemcpyDeviceToHost, s->st));
      ZCHK(hipStreamSynchronize(s->st));
      for (int i = 0; i < nf; ++i) {
        Body& B = s->bodies[fingers[i]];
        double q[12], d[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 12; ++k) q[k] = y[B.dof0 + k];
        if (phase == 0) {
          const double ph = phi_control(fmag[i], gp->k, gp->f_star);
          for (int k = 0; k < 3; ++k) d[k] = ph * h * B.tvel[k];
        } else if (phase == 1) {
          for (int k = 0; k < 3; ++k) d[k] = gp->lift_speed * h * up[k];
        } else {
          const double a0 = gp->shake_amplitude * std::sin(two_pi * gp->shake_frequency * in_phase * h);
          const double a1 = gp->shake_amplitude * std::sin(two_pi * gp->shake_frequency * (in_phase + 1) * h);
          for (int k = 0; k < 3; ++k) d[k] = (a1 - a0) * gp->shake_axis[k];
        }
        for (int k = 0; k < 3; ++k) q[k] += d[k];
        for (int k = 0; k < 3; ++k) B.target_vel[k] = d[k] / h;
        for (int k = 0; k < 12; ++k) B.target[k] = q[k];
        B.has_target = true;
      }
      zema_step_stats st{};
      ZCHK(hipMemcpyAsync(s->yt.p, s->y.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
      ZCHK(hipMemcpyAsync(s->ydt.p, s->ydot.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
      int rc = 0;
      std::string what;
      try {
        rc = time_step(s, &st);
      } catch (const Error& e) {
        rc = e.code;
        what = e.what();
      }
      if (rc) {  // the scene keeps the last accepted state
        ZCHK(hipMemcpyAsync(s->y.p, s->yt.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
        ZCHK(hipMemcpyAsync(s->ydot.p, s->ydt.p, sizeof(double) * s->ndof, hipMemcpyDeviceToDevice, s->st));
        ZCHK(hipStreamSynchronize(s->st));
        res->status = rc;
        res->total_steps = n;
        throw Error(rc, "grasp procedure, step " + std::to_string(n) + ": " + what);
      }
      ++n;
      ++in_phase;
    }
    res->total_steps = n;
    res->ground_force = fground;
    double fmax = 0.0;
    for (int i = 0; i < nf; ++i) fmax = std::max(fmax, fmag[i]);
    res->finger_force_max = fmax;
    res->success = fmax > 0.0 && fground == 0.0 ? 1 : 0;
    return 0;
  });
}

int zema_step_group(zema_scene* const* scenes, int32_t n_scenes, int32_t n_steps, zema_step_stats* const* stats,
                    int32_t* status) {
  if (!scenes || n_scenes <= 0 || n_steps < 0 || !status || (n_steps && !stats)) return ZEMA_E_ARG;
  for (int k = 0; k < n_scenes; ++k)
    if (!scenes[k] || (n_steps && !stats[k])) return ZEMA_E_ARG;
  for (int k = 0; k < n_scenes; ++k)
    for (int j = 0; j < k; ++j)
      if (scenes[j] == scenes[k]) return ZEMA_E_ARG;  // one host thread per object
  std::vector<std::thread> workers;
  workers.reserve(n_scenes);
  for (int k = 0; k < n_scenes; ++k)
    workers.emplace_back([=]() { status[k] = zema_step(scenes[k], n_steps, stats[k]); });
  for (std::thread& t : workers) t.join();
  for (int k = 0; k < n_scenes; ++k)
    if (status[k]) return status[k];
  return 0;
}

int zema_intersection_count(zema_scene* s, const double* y, int64_t* n_intersect, int64_t* n_inverted,
                            int64_t* n_uncertain, int32_t* uncertain_pairs, int64_t cap) {
  if (!s || !y || !n_intersect || !n_inverted || !n_uncertain || (cap > 0 && !uncertain_pairs)) return ZEMA_E_ARG;
  return guard(s, [&]() {
    s->unc_pairs.reserve((size_t)2 * std::max<int64_t>(cap, 1));
    k_intersections(s, y, n_intersect, n_inverted, n_uncertain, s->unc_pairs);
    int64_t nu_pairs = std::min<int64_t>(*n_uncertain, cap);
    if (nu_pairs > 0)
      ZCHK(hipMemcpyAsync(uncertain_pairs, s->unc_pairs.p, sizeof(int) * 2 * nu_pairs, hipMemcpyDeviceToDevice,
                          s->st));
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_kernel_timer(zema_scene* s, int32_t group, int32_t enable) {
  if (!s || group < 0 || group >= KT_N) return ZEMA_E_ARG;
  return guard(s, [&]() {
    ZCHK(hipStreamSynchronize(s->st));
    kt_fold(s);
    KTimer& t = s->kt[group];
    t.on = enable != 0;
    t.ms = 0.0;
    t.launches = 0;
    t.bytes = 0.0;
    return 0;
  });
}

int zema_kernel_time(zema_scene* s, int32_t group, double* ms, int64_t* launches, double* bytes) {
  if (!s || group < 0 || group >= KT_N || !ms || !launches) return ZEMA_E_ARG;
  return guard(s, [&]() {
    ZCHK(hipStreamSynchronize(s->st));
    kt_fold(s);
    *ms = s->kt[group].ms;
    *launches = s->kt[group].launches;
    if (bytes) *bytes = s->kt[group].bytes;
    return 0;
  });
}

int zema_friction_table(zema_scene* s, int64_t* n, int32_t* ids5, double* vals8, int64_t cap) {
  if (!s || !n) return ZEMA_E_ARG;
  return guard(s, [&]() {
    *n = s->nfric;
    if (s->nfric > cap) throw Error(ZEMA_E_CAPACITY, "friction table capacity");
    if (s->nfric) {
      ZCHK(hipMemcpyAsync(ids5, s->f_ids.p, sizeof(int) * 5 * s->nfric, hipMemcpyDeviceToHost, s->st));
      ZCHK(hipMemcpyAsync(vals8, s->f_vals.p, sizeof(double) * 8 * s->nfric, hipMemcpyDeviceToHost, s->st));
    }
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}


// ---------------------------------------------------------------- learned initial guess

static int mguard(zema_mlp* m, const std::function<int()>& f) {
  try {
    return f();
  } catch (const Error& e) {
    if (m) m->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (m) m->err = e.what();
    return ZEMA_E_DEVICE;
  }
}

int zema_mlp_create(void* hip_stream, zema_mlp** out) {
  if (!out) return ZEMA_E_ARG;
  *out = nullptr;
  zema_mlp* m = new (std::nothrow) zema_mlp();
  if (!m) return ZEMA_E_DEVICE;
  m->st = (hipStream_t)hip_stream;
  int rc = mguard(m, [&]() {
    ZCHK(hipGetDevice(&m->dev));
    for (DBuf<float>* b : {&m->theta, &m->mom, &m->vel, &m->grad}) {
      b->resize(kMlpParams);
      ZCHK(hipMemset(b->p, 0, sizeof(float) * kMlpParams));
    }
    m->loss.resize(1);
    return 0;
  });
  if (rc) {
    delete m;
    return rc;
  }
  *out = m;
  return 0;
}

void zema_mlp_destroy(zema_mlp* m) {
  if (m && m->st) (void)hipStreamSynchronize(m->st);
  delete m;
}

const char* zema_mlp_last_error(const zema_mlp* m) { return m ? m->err.c_str() : "null network"; }

int zema_mlp_set_weights(zema_mlp* m, const float* theta) {
  if (!m || !theta) return ZEMA_E_ARG;
  return mguard(m, [&]() {
    ZCHK(hipMemcpyAsync(m->theta.p, theta, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, m->st));
    ZCHK(hipMemsetAsync(m->mom.p, 0, sizeof(float) * kMlpParams, m->st));
    ZCHK(hipMemsetAsync(m->vel.p, 0, sizeof(float) * kMlpParams, m->st));
    ZCHK(hipStreamSynchronize(m->st));
    m->step = 0;
    return 0;
  });
}

int zema_mlp_get_weights(zema_mlp* m, float* theta) {
  if (!m || !theta) return ZEMA_E_ARG;
  return mguard(m, [&]() {
    ZCHK(hipMemcpyAsync(theta, m->theta.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, m->st));
    ZCHK(hipStreamSynchronize(m->st));
    return 0;
  });
}

int zema_mlp_forward(zema_mlp* m, const float* feat, int64_t n, float* out) {
  if (!m || n < 0 || (n && (!feat || !out))) return ZEMA_E_ARG;
  return mguard(m, [&]() {
    mlp_forward(m, m->st, feat, (long)n, out);
    ZCHK(hipGetLastError());
    ZCHK(hipStreamSynchronize(m->st));
    return 0;
  });
}

int zema_mlp_grad(zema_mlp* m, const float* feat, const float* target, int64_t n, float* grad, double* loss) {
  if (!m || n <= 0 || !feat || !target || !grad || !loss) return ZEMA_E_ARG;
  return mguard(m, [&]() {
    *loss = mlp_grad(m, feat, target, nullptr, (long)n, (long)n, false, 0.0f);
    ZCHK(hipMemcpyAsync(grad, m->grad.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, m->st));
    ZCHK(hipStreamSynchronize(m->st));
    return 0;
  });
}

int zema_mlp_grad_noalloc(zema_mlp* m, const float* feat, const float* target, int64_t n, float* grad,
                          double* loss) {
  if (!m || !feat || !target || !grad || !loss) return ZEMA_E_ARG;
  if (n <= 0 || n > ZEMA_MLP_NOALLOC_MAX_ROWS) {
    m->err = "zema_mlp_grad_noalloc: n must be in 1 .. ZEMA_MLP_NOALLOC_MAX_ROWS";
    return ZEMA_E_ARG;
  }
  return mguard(m, [&]() {
    *loss = mlp_grad_noalloc(m, feat, target, (long)n, grad);
    return 0;
  });
}

int zema_mlp_train_step(zema_mlp* m, const float* feat, const float* target, int64_t n_rows, const int32_t* idx,
                        int64_t batch, float lr, double* loss) {
  if (!m || n_rows <= 0 || batch <= 0 || !feat || !target || !idx || !loss || !(lr > 0.0f)) return ZEMA_E_ARG;
  return mguard(m, [&]() {
    *loss = mlp_grad(m, feat, target, idx, (long)n_rows, (long)batch, true, lr);
    return 0;
  });
}

int zema_tune(zema_scene* s, int32_t knob, int32_t value) {
  if (!s) return ZEMA_E_ARG;
  if (knob == ZEMA_TUNE_PCG_GRAPH && (value == 0 || value == 1)) {
    s->use_graph = value != 0;
    return 0;
  }
  if (knob == ZEMA_TUNE_SPMV_LANES && (value == 4 || value == 8 || value == 16 || value == 32)) {
    s->tune_lanes = value;
    return 0;
  }
  if (knob == ZEMA_TUNE_UPDATE_BLOCK && (value == 64 || value == 128 || value == 256)) {
    s->tune_ublock = value;
    return 0;
  }
  if (knob == ZEMA_TUNE_PCG_FORM && (value == 0 || value == 1)) {
    s->pcg_form = value;
    return 0;
  }
  if (knob == ZEMA_TUNE_BATCH_ASYNC && (value == 0 || value == 1)) {
    s->batch_async = value != 0;
    return 0;
  }
  if (knob == ZEMA_TUNE_CG_ROWS && value >= 0 && value <= 64) {
    s->tune_cg_rows = value;
    return 0;
  }
  if (knob == ZEMA_TUNE_WARM_FIT && value >= 0 && value <= 2) {
    s->warm_fit = value;
    return 0;
  }
  return ZEMA_E_ARG;
}

int zema_tune_get(zema_scene* s, int32_t knob, int32_t* value) {
  if (!s || !value) return ZEMA_E_ARG;
  switch (knob) {
    case ZEMA_TUNE_PCG_GRAPH:
      *value = s->use_graph ? 1 : 0;
      return 0;
    case ZEMA_TUNE_SPMV_LANES:
      *value = s->tune_lanes;
      return 0;
    case ZEMA_TUNE_UPDATE_BLOCK:
      *value = s->tune_ublock;
      return 0;
    case ZEMA_TUNE_PCG_FORM:
      *value = s->pcg_form;
      return 0;
    case ZEMA_TUNE_BATCH_ASYNC:
      *value = s->batch_async ? 1 : 0;
      return 0;
    case ZEMA_TUNE_CG_ROWS:
      *value = s->tune_cg_rows;
      return 0;
    case ZEMA_TUNE_WARM_FIT:
      *value = s->warm_fit;
      return 0;
    default:
      return ZEMA_E_ARG;
  }
}

int zema_autotune(zema_scene* s, int32_t* lanes, int32_t* update_block, double* us_per_iter) {
  if (!s || !lanes || !update_block || !us_per_iter || s->ns != 1 || !s->hess_valid) return ZEMA_E_ARG;
  return guard(s, [&]() {
    int l, u;
    k_autotune(s, &l, &u, us_per_iter);
    *lanes = l;
    *update_block = u;
    return 0;
  });
}

int zema_scene_set_mlp(zema_scene* s, zema_mlp* m) {
  if (!s) return ZEMA_E_ARG;
  s->mlp = m;
  return 0;
}

int zema_scene_features(zema_scene* s, float* feat) {
  if (!s || (s->nsv && !feat)) return ZEMA_E_ARG;
  return guard(s, [&]() {
    k_features(s, feat);
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_warm_fit(zema_scene* s, int32_t mode, const float* in, float* out) {
  if (!s || mode < 0 || mode > 2 || (s->nsv && (!in || !out))) return ZEMA_E_ARG;
  return guard(s, [&]() {
    if (s->nsv && in != out)
      ZCHK(hipMemcpyAsync(out, in, sizeof(float) * 3 * (size_t)s->nsv, hipMemcpyDeviceToDevice, s->st));
    k_warm_fit(s, mode, out);
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

int zema_scene_warm_target(zema_scene* s, float* target) {
  if (!s || (s->nsv && !target)) return ZEMA_E_ARG;
  if (!s->stepped) {
    s->err = "no completed step since the state was set";
    return ZEMA_E_ARG;
  }
  return guard(s, [&]() {
    k_warm_target(s, target);
    ZCHK(hipStreamSynchronize(s->st));
    return 0;
  });
}

}  // extern "C"
