// Schemas: the property tree (Sec. VI: per-item, array, sub-group and jagged
// vector properties, nested), its flattening into per-object leaves, record
// slots and jagged groups, and the natural (C) record layouts built from it.
#include <algorithm>

#include "plan.h"
#include "rl_internal.h"

namespace rl {

namespace {

using Prop = rl_schema::Prop;
constexpr int kMaxDepth = 16;

bool valid_type(int t) { return t >= RL_U8 && t <= RL_F64; }
bool offset_type_ok(rl_type t) { return t == RL_U32 || t == RL_I32 || t == RL_U64; }
uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Reads `count` sibling subtrees from props[at...] into out.
rl_status parse(const rl_prop* props, uint32_t n, uint32_t& at, uint32_t count, std::vector<Prop>& out,
                int depth) {
  if (depth > kMaxDepth) return fail(RL_EINVAL, "properties nested deeper than %d levels", kMaxDepth);
  for (uint32_t k = 0; k < count; ++k) {
    if (at >= n) return fail(RL_EINVAL, "property %u: children run past the end of the list", at);
    const rl_prop& p = props[at];
    const uint32_t here = at++;
    Prop q;
    q.kind = p.kind;
    q.type = p.type;
    q.extent = 1;
    q.group = -1;
    q.name = p.name ? p.name : "";
    switch (p.kind) {
      case RL_PROP_ITEM:
        if (!valid_type(p.type)) return fail(RL_EINVAL, "property %u: bad type %d", here, (int)p.type);
        if (p.n_children) return fail(RL_EINVAL, "property %u: an item has no children", here);
        break;
      case RL_PROP_ARRAY:
        if (p.extent < 1 || p.extent > (uint32_t)kMaxExtent)
          return fail(RL_EINVAL, "property %u: extent %u outside 1..%d", here, p.extent, kMaxExtent);
        q.extent = p.extent;
        break;
      case RL_PROP_SUBGROUP:
        break;
      case RL_PROP_JAGGED:
        if (!offset_type_ok(p.type)) return fail(RL_EINVAL, "property %u: offset type must be U32, I32 or U64", here);
        break;
      default:
        return fail(RL_EINVAL, "property %u: bad kind %d", here, (int)p.kind);
    }
    if (p.kind != RL_PROP_ITEM) {
      if (!p.n_children) return fail(RL_EINVAL, "property %u: no child properties", here);
      rl_status st = parse(props, n, at, p.n_children, q.children, depth + 1);
      if (st) return st;
    }
    out.push_back(std::move(q));
  }
  return RL_OK;
}

// Flattening walk (pre-order, array elements in turn).  group < 0: outside
// any jagged vector.
rl_status flatten(rl_schema* s, const Prop& p, int32_t group) {
  switch (p.kind) {
    case RL_PROP_ITEM: {
      const rl_schema::Leaf leaf{p.type, type_size(p.type), -1, 0, -1};
      if (group < 0) {
        s->slots.push_back({0, (int)s->leaves.size(), -1});
        s->leaves.push_back(leaf);
      } else {
        s->members[group].push_back(leaf);
      }
      return RL_OK;
    }
    case RL_PROP_ARRAY:
      for (uint32_t e = 0; e < p.extent; ++e)
        for (const Prop& c : p.children) {
          rl_status st = flatten(s, c, group);
          if (st) return st;
        }
      return RL_OK;
    case RL_PROP_SUBGROUP:
      for (const Prop& c : p.children) {
        rl_status st = flatten(s, c, group);
        if (st) return st;
      }
      return RL_OK;
    default: {
      if (group >= 0) return fail(RL_EUNSUPPORTED, "a jagged vector inside another jagged vector");
      int32_t g = p.group;
      if (g < 0) {
        g = (int32_t)s->offset_types.size();
        if (g >= kMaxGroups) return fail(RL_EINVAL, "at most %d jagged groups", kMaxGroups);
        s->offset_types.push_back(p.type);
        s->members.emplace_back();
        s->group_prop.push_back(&p);
      } else {
        s->group_prop[g] = &p;
      }
      s->slots.push_back({1, g, -1});
      s->slots.push_back({2, g, -1});
      for (const Prop& c : p.children) {
        rl_status st = flatten(s, c, g);
        if (st) return st;
      }
      return RL_OK;
    }
  }
}

rl_status finish(rl_schema* s) {
  for (const Prop& p : s->tree) {
    rl_status st = flatten(s, p, -1);
    if (st) return st;
  }
  for (size_t g = 0; g < s->members.size(); ++g) {
    if (s->members[g].empty()) return fail(RL_EINVAL, "group %zu has no member field", g);
    if (s->members[g].size() > (size_t)kMaxMembers)
      return fail(RL_EINVAL, "group %zu: at most %d member leaves", g, kMaxMembers);
  }
  if (s->leaves.size() + 2 * s->members.size() > (size_t)kMaxLeaves)
    return fail(RL_EINVAL, "at most %d per-object leaves (plus 2 per group)", kMaxLeaves);
  return RL_OK;
}

// ---- natural record layouts

// Sizes of the items met by a walk, in walk order: record slots (per-object
// leaves in their storage types; ptr/len pairs) or one group's member leaves.
struct Walk {
  const rl_schema* s;
  const std::vector<rl_type>* storage;   // per-object walk
  int32_t group;                         // member walk: the group; -1: per-object walk
  size_t next = 0;
  uint64_t item() {
    if (group >= 0) return s->members[group][next++].size;
    const rl_schema::Slot& sl = s->slots[next++];
    return type_size((*storage)[sl.index]);
  }
};

void struct_of(Walk& w, const std::vector<Prop>& props, std::vector<uint64_t>& rel, uint64_t& size,
               uint64_t& align);

// A nested struct made of `props`, placed as the next member at pos.
void nested(Walk& w, const std::vector<Prop>& props, std::vector<uint64_t>& rel, uint64_t& pos, uint64_t& align) {
  std::vector<uint64_t> sub;
  uint64_t sz = 0, al = 1;
  struct_of(w, props, sub, sz, al);
  pos = round_up(pos, al);
  for (uint64_t o : sub) rel.push_back(pos + o);
  pos += sz;
  align = std::max(align, al);
}

void member(Walk& w, const Prop& p, std::vector<uint64_t>& rel, uint64_t& pos, uint64_t& align) {
  switch (p.kind) {
    case RL_PROP_ITEM: {
      const uint64_t sz = w.item();
      pos = round_up(pos, sz);
      rel.push_back(pos);
      pos += sz;
      align = std::max(align, sz);
      return;
    }
    case RL_PROP_JAGGED:   // (u64 ptr, u32 len): two members of this struct
      w.next += 2;
      pos = round_up(pos, 8);
      rel.push_back(pos);
      rel.push_back(pos + 8);
      pos += 12;
      align = std::max<uint64_t>(align, 8);
      return;
    case RL_PROP_SUBGROUP:
      nested(w, p.children, rel, pos, align);
      return;
    default:
      for (uint32_t e = 0; e < p.extent; ++e) nested(w, p.children, rel, pos, align);
      return;
  }
}

void struct_of(Walk& w, const std::vector<Prop>& props, std::vector<uint64_t>& rel, uint64_t& size,
               uint64_t& align) {
  uint64_t pos = 0;
  align = 1;
  for (const Prop& p : props) member(w, p, rel, pos, align);
  size = pos ? round_up(pos, align) : 0;
}

}  // namespace

void natural_record(const rl_schema* s, const std::vector<rl_type>& storage, std::vector<uint64_t>& offs,
                    uint64_t& stride) {
  Walk w{s, &storage, -1};
  uint64_t align = 1;
  offs.clear();
  struct_of(w, s->tree, offs, stride, align);
}

void natural_member_record(const rl_schema* s, uint32_t g, std::vector<uint32_t>& offs, uint32_t& stride,
                           uint32_t& align) {
  Walk w{s, nullptr, (int32_t)g};
  std::vector<uint64_t> rel;
  uint64_t sz = 0, al = 1;
  struct_of(w, s->group_prop[g]->children, rel, sz, al);
  offs.assign(rel.begin(), rel.end());
  stride = (uint32_t)sz;
  align = (uint32_t)al;
}

}  // namespace rl

using namespace rl;

// ------------------------------------------------------------------ entry points

extern "C" rl_status rl_schema_create_tree(const rl_prop* props, uint32_t n_props, rl_schema** out) {
  if (!out) return fail(RL_EINVAL, "rl_schema_create_tree: out is NULL");
  *out = nullptr;
  if (n_props && !props) return fail(RL_EINVAL, "rl_schema_create_tree: props is NULL");
  auto* s = new rl_schema();
  uint32_t at = 0;
  rl_status st = RL_OK;
  while (at < n_props && !st) st = parse(props, n_props, at, 1, s->tree, 0);
  if (!st) st = finish(s);
  if (st) {
    delete s;
    return st;
  }
  *out = s;
  return RL_OK;
}

// A flat field list as a tree: an extent over one item is an array of it;
// a run of per-object fields sharing a sub-group id is a sub-group (a
// member field in between ends the run); the member fields of group g
// form one jagged property, placed where g's first field is declared.
extern "C" rl_status rl_schema_create(const rl_field* fields, uint32_t n_fields, const rl_jagged* groups,
                                      uint32_t n_groups, rl_schema** out) {
  if (!out) return fail(RL_EINVAL, "rl_schema_create: out is NULL");
  *out = nullptr;
  if (n_fields && !fields) return fail(RL_EINVAL, "rl_schema_create: fields is NULL");
  if (n_groups && !groups) return fail(RL_EINVAL, "rl_schema_create: groups is NULL");
  if (n_groups > (uint32_t)kMaxGroups) return fail(RL_EINVAL, "at most %d jagged groups", kMaxGroups);
  auto* s = new rl_schema();
  auto bad = [&](rl_status st) {
    delete s;
    return st;
  };
  for (uint32_t g = 0; g < n_groups; ++g) {
    if (!offset_type_ok(groups[g].offset_type))
      return bad(fail(RL_EINVAL, "group %u: offset type must be U32, I32 or U64", g));
    s->offset_types.push_back(groups[g].offset_type);
  }
  s->members.resize(n_groups);
  s->group_prop.assign(n_groups, nullptr);
  // first pass: validate; the sub-group and group a field joins
  int32_t prev_sub = -1;
  std::vector<int> sub_closed;
  for (uint32_t k = 0; k < n_fields; ++k) {
    const rl_field& f = fields[k];
    if (!valid_type(f.type)) return bad(fail(RL_EINVAL, "field %u: bad type %d", k, (int)f.type));
    if (f.extent < 1 || f.extent > (uint32_t)kMaxExtent)
      return bad(fail(RL_EINVAL, "field %u: extent %u outside 1..%d", k, f.extent, kMaxExtent));
    if (f.group < -1 || f.group >= (int32_t)n_groups)
      return bad(fail(RL_EINVAL, "field %u: group %d out of range", k, f.group));
    if (f.subgroup < -1) return bad(fail(RL_EINVAL, "field %u: bad subgroup", k));
    if (f.group >= 0 && f.subgroup >= 0)
      return bad(fail(RL_EINVAL, "field %u: a member field cannot be in a sub-group", k));
    if (f.group < 0) {
      if (f.subgroup >= 0 && f.subgroup != prev_sub &&
          std::find(sub_closed.begin(), sub_closed.end(), f.subgroup) != sub_closed.end())
        return bad(fail(RL_EINVAL, "field %u: sub-group %d is not consecutive", k, f.subgroup));
      if (prev_sub >= 0 && f.subgroup != prev_sub) sub_closed.push_back(prev_sub);
      prev_sub = f.subgroup;
    }
    s->fields.push_back(f);
    s->names.push_back(f.name ? f.name : "");
  }
  // second pass: the tree
  auto leaf_prop = [](const rl_field& f) {
    Prop item{RL_PROP_ITEM, f.type, 1, -1, f.name ? f.name : "", {}};
    if (f.extent == 1) return item;
    Prop arr{RL_PROP_ARRAY, f.type, f.extent, -1, item.name, {}};
    arr.children.push_back(item);
    return arr;
  };
  std::vector<int> group_at(n_groups, -1);   // index of group g's property in the top level
  int32_t open_sub = -1;                     // sub-group of the last top-level property, if open
  for (uint32_t k = 0; k < n_fields; ++k) {
    const rl_field& f = fields[k];
    if (f.group >= 0) {
      if (group_at[f.group] < 0) {
        group_at[f.group] = (int)s->tree.size();
        s->tree.push_back(Prop{RL_PROP_JAGGED, s->offset_types[f.group], 1, f.group, "", {}});
        open_sub = -1;
      }
      s->tree[group_at[f.group]].children.push_back(leaf_prop(f));
      continue;
    }
    if (f.subgroup < 0) {
      s->tree.push_back(leaf_prop(f));
      open_sub = -1;
      continue;
    }
    if (open_sub != f.subgroup) {
      s->tree.push_back(Prop{RL_PROP_SUBGROUP, f.type, 1, -1, "", {}});
      open_sub = f.subgroup;
    }
    s->tree.back().children.push_back(leaf_prop(f));
  }
  rl_status st = finish(s);
  if (st) return bad(st);
  // the leaves' field and element, as declared
  size_t leaf = 0;
  std::vector<uint32_t> mcount(n_groups, 0);
  for (uint32_t k = 0; k < n_fields; ++k) {
    const rl_field& f = fields[k];
    for (uint32_t e = 0; e < f.extent; ++e) {
      rl_schema::Leaf& l = f.group < 0 ? s->leaves[leaf++] : s->members[f.group][mcount[f.group]++];
      l.field = (int32_t)k;
      l.element = e;
      l.subgroup = f.subgroup;
    }
  }
  *out = s;
  return RL_OK;
}

extern "C" void rl_schema_destroy(rl_schema* schema) { delete schema; }

extern "C" rl_status rl_schema_info(const rl_schema* s, uint32_t* n_leaves, uint32_t* n_groups,
                                    uint32_t* n_slots) {
  if (!s) return fail(RL_EINVAL, "schema is NULL");
  if (n_leaves) *n_leaves = (uint32_t)s->leaves.size();
  if (n_groups) *n_groups = (uint32_t)s->offset_types.size();
  if (n_slots) *n_slots = (uint32_t)s->slots.size();
  return RL_OK;
}
